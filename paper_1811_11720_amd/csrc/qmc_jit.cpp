// qmc_jit.cpp -- descriptor-specialised evaluation kernels compiled at run time.
//
// The paper compiles each generated sector integrand into its kernel (Sec. 3.1,
// Sec. 4).  Here the integrand's monomial table is turned into straight-line
// HIP code when it is first integrated: U and F become a multivariate Horner
// scheme (greedy: factor out the variable that occurs in most remaining
// terms), the power classes become literal constants, and the result is
// compiled with hiprtc for gfx950 and instantiated into the same evaluation
// body as the ahead-of-time kernels (qmc_device.h).  Coefficients stay in
// device memory, so integrands that differ only in coefficients share a
// module.  Modules are cached per (device, source).
#include <hip/hip_runtime.h>
#include <hip/hiprtc.h>

#include <algorithm>
#include <array>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <sstream>
#include <string>
#include <vector>

#include "qmc_internal.h"
#include "qmc_jit.h"

namespace {

const char* kDeviceSrc =
#include "qmc_device_src.inc"
    ;

int Tri_N(int d) { return d * (d + 1) / 2; }

struct Term {
  uint32_t ci;
  std::array<uint8_t, QMCD_MAXD> e;
};

class Emitter {
 public:
  explicit Emitter(int dim) : dim_(dim) {}
  std::string tmp() { return "t" + std::to_string(ntmp_++); }
  void line(const std::string& s) { body_ << "    " << s << "\n"; }
  std::string coef(uint32_t i) {
    std::string n = "c" + std::to_string(i);
    if (!coefs_.count(i)) coefs_[i] = n;
    return n;
  }
  // x_j^e from previously formed powers (x_j^2 = x_j x_j, x_j^(2k) = (x_j^k)^2, ...)
  std::string power(int j, int e) {
    auto key = std::make_pair(j, e);
    auto it = pows_.find(key);
    if (it != pows_.end()) return it->second;
    std::string n = "x" + std::to_string(j) + "_" + std::to_string(e);
    std::string v;
    if (e == 1) {
      v = "x[" + std::to_string(j) + "]";
    } else if (e % 2 == 0) {
      std::string h = power(j, e / 2);
      v = h + " * " + h;
    } else {
      v = power(j, e - 1) + " * " + power(j, 1);
    }
    pre_ << "    const double " << n << " = " << v << ";\n";
    pows_[key] = n;
    return n;
  }
  // The coefficients are members of the functor, read once per tile by
  // bind() (through the constant address space: scalar loads) before the point
  // loop.  Read inside the evaluation they sit in the shift loop's conditional
  // block, where they are reloaded for every shift of every point.
  std::string members() const {
    std::ostringstream o;
    for (auto& kv : coefs_) o << "  double " << kv.second << ";\n";
    o << "  __device__ __forceinline__ void bind(const EvalArgs& a) {\n";
    for (auto& kv : coefs_) o << "    " << kv.second << " = as_const(a.coef)[" << kv.first << "];\n";
    o << "  }\n";
    return o.str();
  }
  std::string pre() const { return pre_.str(); }
  std::string body() const { return body_.str(); }
  int dim() const { return dim_; }

 private:
  int dim_;
  int ntmp_ = 0;
  std::map<uint32_t, std::string> coefs_;
  std::map<std::pair<int, int>, std::string> pows_;
  std::ostringstream pre_, body_;
};

// Choice of the factor at each step of the multivariate Horner scheme.  A
// step takes x_j^e out of the terms whose exponent of x_j is at least e and
// joins them to the remaining terms with one fma (a multiply when none
// remain).  The splits of least total operation count are found by an
// exhaustive search memoised over term sets (power formation not counted);
// a set of more than kMaxTerms terms, or one not yet solved once `max_states`
// sets are stored, takes the greedy split instead: the variable that occurs
// in most terms, at its smallest exponent among them.
class HornerPlan {
 public:
  explicit HornerPlan(int dim, size_t max_states = 1u << 14) : d_(dim), max_(max_states) {}

  template <class T>
  void split(const std::vector<T>& terms, int& j, int& e) {
    std::vector<Ex> ex;
    ex.reserve(terms.size());
    for (auto& t : terms) ex.push_back(t.e);
    std::sort(ex.begin(), ex.end());
    cost(ex);
    auto it = memo_.find(key(ex));
    if (it != memo_.end()) {
      j = it->second.j;
      e = it->second.e;
      return;
    }
    int cnt = -1;
    for (int v = 0; v < d_; ++v) {
      int c = 0, lo = 255;
      for (auto& t : ex)
        if (t[v]) {
          ++c;
          lo = std::min<int>(lo, t[v]);
        }
      if (c > cnt) {
        cnt = c;
        j = v;
        e = lo;
      }
    }
  }

 private:
  using Ex = std::array<uint8_t, QMCD_MAXD>;
  struct Best {
    int cost, j, e;
  };
  static constexpr int kUnsolved = 1 << 30;
  static constexpr size_t kMaxTerms = 48;  // larger sets split greedily

  std::string key(const std::vector<Ex>& ex) const {
    std::string k;
    k.reserve(ex.size() * d_);
    for (auto& t : ex) k.append(reinterpret_cast<const char*>(t.data()), d_);
    return k;
  }
  // least operation count for the (sorted) term set, kUnsolved past the budget
  int cost(const std::vector<Ex>& ex) {
    bool all_const = true;
    for (auto& t : ex)
      for (int v = 0; v < d_; ++v)
        if (t[v]) all_const = false;
    if (all_const) return (int)ex.size() - 1;
    if (ex.size() > kMaxTerms) return kUnsolved;
    std::string k = key(ex);
    auto it = memo_.find(k);
    if (it != memo_.end()) return it->second.cost;
    if (memo_.size() >= max_) return kUnsolved;
    Best best{kUnsolved, -1, 0};
    for (int v = 0; v < d_; ++v) {
      std::set<int> levels;
      for (auto& t : ex)
        if (t[v]) levels.insert(t[v]);
      for (int lv : levels) {
        std::vector<Ex> A, B;
        for (auto& t : ex) {
          if (t[v] >= lv) {
            Ex u = t;
            u[v] = (uint8_t)(u[v] - lv);
            A.push_back(u);
          } else {
            B.push_back(t);
          }
        }
        std::sort(A.begin(), A.end());
        const int ca = cost(A);
        const int cb = B.empty() ? 0 : cost(B);
        if (ca >= kUnsolved || cb >= kUnsolved) return kUnsolved;
        if (ca + cb + 1 < best.cost) best = Best{ca + cb + 1, v, lv};
      }
    }
    if (memo_.size() >= max_) return kUnsolved;
    memo_.emplace(std::move(k), best);
    return best.cost;
  }

  int d_;
  size_t max_;
  std::map<std::string, Best> memo_;
};

// Multivariate Horner: returns the name holding sum_i c_i prod_j x_j^e_ij.
std::string horner(std::vector<Term> terms, Emitter& em, HornerPlan& plan) {
  const int d = em.dim();
  bool all_const = true;
  for (auto& t : terms)
    for (int j = 0; j < d; ++j)
      if (t.e[j]) all_const = false;
  if (all_const) {
    std::string acc = em.coef(terms[0].ci);
    if (terms.size() == 1) return acc;
    std::string v = em.tmp();
    std::string expr = acc;
    for (size_t i = 1; i < terms.size(); ++i) expr += " + " + em.coef(terms[i].ci);
    em.line("const double " + v + " = " + expr + ";");
    return v;
  }
  int best = -1, emin = 0;
  plan.split(terms, best, emin);
  std::vector<Term> A, B;
  for (auto& t : terms) (t.e[best] >= emin ? A : B).push_back(t);
  for (auto& t : A) t.e[best] = (uint8_t)(t.e[best] - emin);
  std::string va = horner(A, em, plan);
  std::string p = em.power(best, emin);
  std::string v = em.tmp();
  if (B.empty()) {
    em.line("const double " + v + " = " + p + " * " + va + ";");
  } else {
    // coefficients (c*) live in scalar registers: a scalar addend with a
    // vector multiplicand takes the three-address fma
    std::string vb = horner(B, em, plan);
    if (vb[0] == 'c' && va[0] != 'c')
      em.line("const double " + v + " = fma_s(" + p + ", " + va + ", " + vb + ");");
    else
      em.line("const double " + v + " = __builtin_fma(" + p + ", " + va + ", " + vb + ");");
  }
  return v;
}

// ---------------------------------------------------------------- complex integrands

// A term whose coefficient is coef[ci] * mult (mult from differentiating).
struct CTerm {
  uint32_t ci;
  int mult;
  std::array<uint8_t, QMCD_MAXD> e;
};

struct Val {
  std::string name;
  bool real;  // a real scalar (coefficient); otherwise a cplx value in the complex domain
};

// A coefficient as the kernel reads it: from its arguments, or, with the values
// given, as an exact hexadecimal constant.  Constants take no registers across
// the point loop, where the table-read values of a large integrand overflow
// the scalar registers and are spilled and reloaded at every point.
std::string coef_value(const double* values, uint32_t i) {
  if (!values) return "as_const(a.coef)[" + std::to_string(i) + "]";
  char buf[64];
  std::snprintf(buf, sizeof buf, "%a", values[i]);
  return buf;
}

class CEmitter {
 public:
  CEmitter(int dim, bool cplx_domain, const double* values) : dim_(dim), cx_(cplx_domain), values_(values) {}
  std::string tmp() { return std::string(cx_ ? "w" : "r") + std::to_string(ntmp_++); }
  void line(const std::string& s) { body_ << "    " << s << "\n"; }
  std::string coef(uint32_t i, int mult) {
    std::string base = "c" + std::to_string(i);
    coefs_.insert(i);
    if (mult == 1) return base;
    std::string n = base + "m" + std::to_string(mult);
    if (!scaled_.count(n)) scaled_[n] = base + " * " + std::to_string(mult) + ".0";
    return n;
  }
  std::string power(int j, int e) {
    auto key = std::make_pair(j, e);
    auto it = pows_.find(key);
    if (it != pows_.end()) return it->second;
    std::string n = std::string(cx_ ? "z" : "x") + std::to_string(j) + "_" + std::to_string(e);
    std::string v;
    if (e == 1) {
      v = std::string(cx_ ? "z[" : "x[") + std::to_string(j) + "]";
    } else if (e % 2 == 0) {
      std::string h = power(j, e / 2);
      v = cx_ ? "cmul(" + h + ", " + h + ")" : h + " * " + h;
    } else {
      std::string a = power(j, e - 1), b = power(j, 1);
      v = cx_ ? "cmul(" + a + ", " + b + ")" : a + " * " + b;
    }
    pre_ << "    const " << (cx_ ? "cplx " : "double ") << n << " = " << v << ";\n";
    pows_[key] = n;
    return n;
  }
  std::string decls() const {
    std::ostringstream o;
    for (uint32_t i : coefs_) o << "    const double c" << i << " = " << coef_value(values_, i) << ";\n";
    for (auto& kv : scaled_) o << "    const double " << kv.first << " = " << kv.second << ";\n";
    return o.str();
  }
  std::string pre() const { return pre_.str(); }
  std::string body() const { return body_.str(); }
  int dim() const { return dim_; }
  bool cx() const { return cx_; }

 private:
  int dim_;
  bool cx_;
  const double* values_;
  int ntmp_ = 0;
  std::set<uint32_t> coefs_;
  std::map<std::string, std::string> scaled_;
  std::map<std::pair<int, int>, std::string> pows_;
  std::ostringstream pre_, body_;
};

// Multivariate Horner over a real (x) or complex (z) variable vector.
Val chorner(std::vector<CTerm> terms, CEmitter& em, HornerPlan& plan) {
  const int d = em.dim();
  if (terms.empty()) return Val{"0.0", true};
  bool all_const = true;
  for (auto& t : terms)
    for (int j = 0; j < d; ++j)
      if (t.e[j]) all_const = false;
  if (all_const) {
    std::string expr = em.coef(terms[0].ci, terms[0].mult);
    if (terms.size() == 1) return Val{expr, true};
    for (size_t i = 1; i < terms.size(); ++i) expr += " + " + em.coef(terms[i].ci, terms[i].mult);
    std::string v = "s" + em.tmp();
    em.line("const double " + v + " = " + expr + ";");
    return Val{v, true};
  }
  int best = -1, emin = 0;
  plan.split(terms, best, emin);
  std::vector<CTerm> A, B;
  for (auto& t : terms) (t.e[best] >= emin ? A : B).push_back(t);
  for (auto& t : A) t.e[best] = (uint8_t)(t.e[best] - emin);
  Val va = chorner(A, em, plan);
  std::string p = em.power(best, emin);
  std::string v = em.tmp();
  if (!em.cx()) {
    if (B.empty()) {
      em.line("const double " + v + " = " + p + " * " + va.name + ";");
    } else {
      Val vb = chorner(B, em, plan);
      em.line("const double " + v + " = __builtin_fma(" + p + ", " + va.name + ", " + vb.name + ");");
    }
    return Val{v, true};
  }
  // complex domain: p is cplx; va, vb real (coefficient) or cplx
  if (B.empty()) {
    if (va.real)
      em.line("const cplx " + v + " = cscale(" + va.name + ", " + p + ");");
    else
      em.line("const cplx " + v + " = cmul(" + p + ", " + va.name + ");");
    return Val{v, false};
  }
  Val vb = chorner(B, em, plan);
  std::string cb = vb.real ? "cmk(" + vb.name + ", 0.0)" : vb.name;
  if (va.real)
    em.line("const cplx " + v + " = cfmar(" + va.name + ", " + p + ", " + cb + ");");
  else
    em.line("const cplx " + v + " = cfma(" + p + ", " + va.name + ", " + cb + ");");
  return Val{v, false};
}

std::string generate_complex_fn(const qmcj::Spec& s) {
  const int d = (int)s.dim;
  std::vector<CTerm> tu, tf;
  for (uint32_t i = 0; i < s.n_u + s.n_f; ++i) {
    CTerm t;
    t.ci = i;
    t.mult = 1;
    t.e.fill(0);
    for (int j = 0; j < d; ++j) t.e[j] = s.expo[(size_t)i * d + j];
    (i < s.n_u ? tu : tf).push_back(t);
  }
  std::ostringstream o;
  o << "namespace qmcd {\nstruct JitComplex {\n";
  // gradient and Hessian of F at real x, per monomial m_i = c_i prod_j x_j^e_ij:
  //   t_j = m_i e_ij / x_j adds to dF/dx_j; t_j e_il / x_l to d2F/dx_j dx_l (l != j);
  //   t_j (e_ij - 1) / x_j to d2F/dx_j^2.  Reciprocals are formed once per point;
  //   x_j = 0 only where the transform weight is 0 and the point is discarded.
  {
    std::ostringstream gb;
    std::set<std::pair<int, int>> erx;  // (j, k): k / x_j
    std::set<std::pair<int, int>> pw;   // (j, e): x_j^e
    int nm = 0;
    // accumulators are updated monomial by monomial so only they stay live
    for (auto& t : tf) {
      std::vector<int> nz;
      for (int j = 0; j < d; ++j)
        if (t.e[j]) nz.push_back(j);
      if (nz.empty()) continue;  // constant term: no derivative
      std::string mname = "m" + std::to_string(nm++);
      std::string prod = "c" + std::to_string(t.ci);
      for (int j : nz) {
        pw.insert({j, (int)t.e[j]});
        prod += " * xp" + std::to_string(j) + "_" + std::to_string((int)t.e[j]);
      }
      gb << "    {\n      const double " << mname << " = " << prod << ";\n";
      for (size_t q = 0; q < nz.size(); ++q) {
        int j = nz[q];
        int ej = t.e[j];
        erx.insert({j, ej});
        std::string tj = "t" + std::to_string(j);
        gb << "      const double " << tj << " = " << mname << " * rx" << j << "_" << ej << ";\n";
        gb << "      g[" << j << "] += " << tj << ";\n";
        if (ej >= 2) {
          erx.insert({j, ej - 1});
          int k = j * (j + 1) / 2 + j;
          gb << "      H[" << k << "] = __builtin_fma(" << tj << ", rx" << j << "_" << (ej - 1) << ", H[" << k << "]);\n";
        }
      }
      for (size_t q = 0; q < nz.size(); ++q)
        for (size_t r = q + 1; r < nz.size(); ++r) {
          int j = nz[q], l = nz[r];
          int k = l * (l + 1) / 2 + j;
          erx.insert({l, (int)t.e[l]});
          gb << "      H[" << k << "] = __builtin_fma(t" << j << ", rx" << l << "_" << (int)t.e[l] << ", H[" << k
             << "]);\n";
        }
      gb << "    }\n";
    }
    o << "  __device__ __forceinline__ void grad_hess(const double (&x)[" << d << "], double (&g)[" << d
      << "], double (&H)[" << Tri_N(d) << "], const EvalArgs& a) const {\n";
    std::set<uint32_t> used;
    for (auto& t : tf) {
      bool any = false;
      for (int j = 0; j < d; ++j) any = any || t.e[j];
      if (any) used.insert(t.ci);
    }
    for (uint32_t i : used) o << "    const double c" << i << " = " << coef_value(s.coef, i) << ";\n";
    std::set<int> rjs;
    for (auto& p : erx) rjs.insert(p.first);
    for (int j : rjs) o << "    const double rx" << j << " = fast_rcp(x[" << j << "]);\n";
    for (auto& p : erx)
      o << "    const double rx" << p.first << "_" << p.second << " = "
        << (p.second == 1 ? "rx" + std::to_string(p.first) : std::to_string(p.second) + ".0 * rx" + std::to_string(p.first))
        << ";\n";
    std::map<int, int> emax;
    for (auto& p : pw) emax[p.first] = std::max(emax[p.first], p.second);
    for (auto& kv : emax) {
      int j = kv.first;
      o << "    const double xp" << j << "_1 = x[" << j << "];\n";
      for (int e = 2; e <= kv.second; ++e)
        o << "    const double xp" << j << "_" << e << " = xp" << j << "_" << (e / 2) << " * xp" << j << "_"
          << (e - e / 2) << ";\n";
    }
    o << "    for (int j = 0; j < " << d << "; ++j) g[j] = 0.0;\n";
    o << "    for (int j = 0; j < " << Tri_N(d) << "; ++j) H[j] = 0.0;\n";
    o << gb.str();
    o << "  }\n";
  }
  for (int which = 0; which < 2; ++which) {
    CEmitter em(d, true, s.coef);
    HornerPlan plan(d, 0);  // greedy: complex products make the operation count a poor cost model
    Val v = chorner(which == 0 ? tu : tf, em, plan);
    o << "  __device__ __forceinline__ cplx " << (which == 0 ? "U" : "F") << "(const cplx (&z)[" << d
      << "], const EvalArgs& a) const {\n";
    o << em.decls() << em.pre() << em.body();
    o << "    return " << (v.real ? "cmk(" + v.name + ", 0.0)" : v.name) << ";\n  }\n";
  }
  o << "  __device__ __forceinline__ cplx uf(const cplx (&z)[" << d
    << "], const EvalArgs& a, uint32_t& sign) const {\n    return uf_fp64_fixed<" << d << ", " << s.pu_mode << ", "
    << s.pu_k << ", " << s.pf_mode << ", " << s.pf_k << ">(*this, z, a, sign);\n  }\n";
  if (s.vr && s.vr_params) {
    // the fitted map with its parameters as constants (j is unrolled at every call)
    o << "  __device__ __forceinline__ double vr_map(double y, int j, double& w) const {\n"
      << "    constexpr double P[" << 6 * d << "] = {";
    for (int i = 0; i < 6 * d; ++i) o << (i ? ", " : "") << coef_value(s.vr_params, (uint32_t)i);
    o << "};\n    return vr_map_v(y, P[6 * j], P[6 * j + 1], P[6 * j + 2], P[6 * j + 3], P[6 * j + 4], P[6 * j + 5], w);\n  }\n";
  }
  o << "};\n}  // namespace qmcd\n";
  return o.str();
}

struct Module {
  hipModule_t mod = nullptr;
  hipFunction_t f32 = nullptr, f64 = nullptr, batch = nullptr;
  int occ_blocks = 0, occ_batch = 0;
};

std::mutex g_mu;
std::map<std::string, std::shared_ptr<Module>> g_cache;
thread_local std::string g_jit_err;

}  // namespace

namespace qmcj {

const char* last_error() { return g_jit_err.c_str(); }

std::string generate(const Spec& s) {
  const int d = (int)s.dim;
  const char* tk = s.tk == qmcd::TK_KOROBOV3 ? "qmcd::TK_KOROBOV3"
                   : s.tk == qmcd::TK_KOROBOV ? "qmcd::TK_KOROBOV"
                   : s.tk == qmcd::TK_BAKER   ? "qmcd::TK_BAKER"
                   : s.tk == qmcd::TK_SIDI    ? "qmcd::TK_SIDI"
                                               : "qmcd::TK_NONE";
  if (s.cplx) {
    const char* vrm = !s.vr ? "qmcd::VRM_OFF" : s.vr_params ? "qmcd::VRM_FN" : "qmcd::VRM_ON";
    std::ostringstream o;
    o << "#define QMC_RTC 1\n" << kDeviceSrc << "\n" << generate_complex_fn(s);
    for (int w = 0; w < 2; ++w) {
      o << "extern \"C\" __global__ __launch_bounds__(QMCD_BLOCK) void qmc_jit_eval" << (w ? "64" : "32")
        << "(qmcd::EvalArgs a) {\n  qmcd::eval_complex_body<" << d << ", " << tk << ", " << (w ? "false" : "true")
        << ", " << s.S << ", true, qmcd::JitComplex, " << vrm << ">(a, qmcd::JitComplex());\n}\n";
    }
    // persistent batch entry: the table-driven complex batch kernels' tile
    // loop and shift groups, with this integrand's evaluation
    o << "extern \"C\" __global__ __launch_bounds__(QMCD_BLOCK) void qmc_jit_batch(const qmcd::EvalArgs* __restrict__ "
         "items, const uint32_t* __restrict__ order, const uint32_t* __restrict__ prefix, uint32_t nitems, "
         "uint32_t* __restrict__ counter) {\n  qmcd::batch_tiles<"
      << qmck::S_COMPLEX << ">(items, order, prefix, nitems, counter, [&](const qmcd::EvalArgs& a, const qmcd::Sched& sc) {\n"
      << "    qmcd::eval_complex_sched<" << d << ", " << tk << ", false, " << qmck::S_COMPLEX << ", true, qmcd::JitComplex, "
      << vrm << ">(a, qmcd::JitComplex(), sc);\n  });\n}\n";
    return o.str();
  }
  Emitter em(d);
  std::vector<Term> tu, tf;
  for (uint32_t i = 0; i < s.n_u + s.n_f; ++i) {
    Term t;
    t.ci = i;
    t.e.fill(0);
    for (int j = 0; j < d; ++j) t.e[j] = s.expo[(size_t)i * d + j];
    (i < s.n_u ? tu : tf).push_back(t);
  }
  HornerPlan plan(d);
  std::string U = horner(tu, em, plan);
  std::string F = s.n_f ? horner(tf, em, plan) : std::string();
  std::ostringstream o;
  o << "#define QMC_RTC 1\n" << kDeviceSrc << "\n";
  o << "namespace qmcd {\nstruct JitReal {\n";
  // the single-root form is only chosen when U and F are bounded away from 0
  // and infinity on [0, 1]^d, so f is finite there
  if (s.ru > 0 && s.rf > 0 && s.n_f) o << "  static constexpr bool kBounded = true;\n";
  o << em.members();
  o << "  __device__ __forceinline__ double operator()(const double (&x)[" << d
    << "], const EvalArgs& a) const {\n";
  o << em.pre() << em.body();
  if (s.ru > 0 && s.rf > 0 && s.n_f) {
    // U^ru F^rf by binary powering, then one reciprocal square root
    int nt = 0;
    auto power = [&](const std::string& base, int e) {
      std::string acc, b = base;
      while (e) {
        if (e & 1) {
          if (acc.empty()) {
            acc = b;
          } else {
            std::string t = "r" + std::to_string(nt++);
            o << "    const double " << t << " = " << acc << " * " << b << ";\n";
            acc = t;
          }
        }
        e >>= 1;
        if (e) {
          std::string t = "r" + std::to_string(nt++);
          o << "    const double " << t << " = " << b << " * " << b << ";\n";
          b = t;
        }
      }
      return acc;
    };
    std::string pu = power(U, s.ru), pf = power(F, s.rf);
    o << "    return a.prefactor * fast_rsqrt(" << pu << " * " << pf << ");\n  }\n};\n}  // namespace qmcd\n";
  } else {
    o << "    double num = a.prefactor, den = 1.0;\n";
    o << "    apply_pow<double>(" << U << ", " << s.pu_mode << ", " << s.pu_k << ", a.pow_u, num, den);\n";
    if (s.n_f) o << "    apply_pow<double>(" << F << ", " << s.pf_mode << ", " << s.pf_k << ", a.pow_f, num, den);\n";
    o << "    return num * fast_rcp(den);\n  }\n};\n}  // namespace qmcd\n";
  }
  o << "extern \"C\" __global__ __launch_bounds__(QMCD_BLOCK) void qmc_jit_batch(const qmcd::EvalArgs* __restrict__ "
       "items, const uint32_t* __restrict__ order, const uint32_t* __restrict__ prefix, uint32_t nitems, "
       "uint32_t* __restrict__ counter) {\n  qmcd::batch_tiles<"
    << qmck::S_REAL << ">(items, order, prefix, nitems, counter, [&](const qmcd::EvalArgs& a, const qmcd::Sched& sc) {\n"
    << "    qmcd::eval_real_sched<" << d << ", " << tk << ", false, " << qmck::S_REAL << ", true, qmcd::JitReal, "
    << (s.vr ? "qmcd::VRM_ON" : "qmcd::VRM_OFF") << ">(a, qmcd::JitReal(), sc);\n  });\n}\n";
  for (int w = 0; w < 2; ++w) {
    o << "extern \"C\" __global__ __launch_bounds__(QMCD_BLOCK) void qmc_jit_eval" << (w ? "64" : "32")
      << "(qmcd::EvalArgs a) {\n  qmcd::eval_real_body<" << d << ", " << tk << ", " << (w ? "false" : "true")
      << ", " << s.S << ", true, qmcd::JitReal, " << (s.vr ? "qmcd::VRM_ON" : "qmcd::VRM_OFF")
      << ">(a, qmcd::JitReal());\n}\n";
  }
  return o.str();
}

// hiprtc: source -> gfx950 code object
static int compile(const std::string& src, std::vector<char>& code) {
  hiprtcProgram prog;
  if (hiprtcCreateProgram(&prog, src.c_str(), "qmc_jit.hip", 0, nullptr, nullptr) != HIPRTC_SUCCESS) {
    g_jit_err = "hiprtcCreateProgram failed";
    return -1;
  }
  const char* opts[] = {"--offload-arch=gfx950", "-O3", "-std=c++17", "-mcode-object-version=5",
                        "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"};
  hiprtcResult rc = hiprtcCompileProgram(prog, (int)(sizeof opts / sizeof opts[0]), opts);
  if (rc != HIPRTC_SUCCESS) {
    size_t ls = 0;
    hiprtcGetProgramLogSize(prog, &ls);
    std::string log(ls + 1, '\0');
    hiprtcGetProgramLog(prog, &log[0]);
    g_jit_err = "hiprtc compile failed: " + log.substr(0, 2000);
    hiprtcDestroyProgram(&prog);
    return -1;
  }
  size_t cs = 0;
  hiprtcGetCodeSize(prog, &cs);
  code.resize(cs);
  hiprtcGetCode(prog, code.data());
  hiprtcDestroyProgram(&prog);
  return 0;
}

int compile_only(const Spec& s, size_t* code_bytes) {
  std::vector<char> code;
  std::string src = generate(s);
  if (const char* dump = std::getenv("QMC_JIT_DUMP")) {
    if (FILE* fh = std::fopen(dump, "w")) {
      std::fputs(src.c_str(), fh);
      std::fclose(fh);
    }
  }
  int rc = compile(src, code);
  if (code_bytes) *code_bytes = code.size();
  return rc;
}

int get(int device, const Spec& s, Kernel* out) {
  std::string src = generate(s);
  std::string key = std::to_string(device) + "|" + src;
  {
    std::lock_guard<std::mutex> g(g_mu);
    auto it = g_cache.find(key);
    if (it != g_cache.end()) {
      out->f32 = it->second->f32;
      out->f64 = it->second->f64;
      out->occ_blocks = it->second->occ_blocks;
      out->batch = it->second->batch;
      out->occ_batch = it->second->occ_batch;
      return 0;
    }
  }
  std::vector<char> code;
  if (compile(src, code)) return -1;
  auto m = std::make_shared<Module>();
  hipError_t e = hipModuleLoadData(&m->mod, code.data());
  if (e == hipSuccess) e = hipModuleGetFunction(&m->f32, m->mod, "qmc_jit_eval32");
  if (e == hipSuccess) e = hipModuleGetFunction(&m->f64, m->mod, "qmc_jit_eval64");
  if (e == hipSuccess) e = hipModuleGetFunction(&m->batch, m->mod, "qmc_jit_batch");
  if (e != hipSuccess) {
    g_jit_err = std::string("module load failed: ") + hipGetErrorString(e);
    return -2;
  }
  int occ = 0;
  if (hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&occ, m->f32, QMCD_BLOCK, 0) != hipSuccess) occ = 0;
  m->occ_blocks = occ;
  if (m->batch && hipModuleOccupancyMaxActiveBlocksPerMultiprocessor(&occ, m->batch, QMCD_BLOCK, 0) == hipSuccess)
    m->occ_batch = occ;
  {
    std::lock_guard<std::mutex> g(g_mu);
    g_cache[key] = m;
  }
  out->f32 = m->f32;
  out->f64 = m->f64;
  out->occ_blocks = m->occ_blocks;
  out->batch = m->batch;
  out->occ_batch = m->occ_batch;
  return 0;
}

hipError_t launch(const Kernel& k, bool idx32, const qmcd::EvalArgs& a, dim3 grid, hipStream_t st) {
  qmcd::EvalArgs copy = a;
  void* params[] = {&copy};
  return hipModuleLaunchKernel(idx32 ? k.f32 : k.f64, grid.x, grid.y, grid.z, QMCD_BLOCK, 1, 1, 0, st, params,
                               nullptr);
}

hipError_t launch_batch(const Kernel& k, const qmcd::EvalArgs* items, const uint32_t* order, const uint32_t* prefix,
                        uint32_t nitems, uint32_t* counter, uint32_t blocks, hipStream_t st) {
  if (!k.batch) return hipErrorInvalidValue;
  void* params[] = {(void*)&items, (void*)&order, (void*)&prefix, (void*)&nitems, (void*)&counter};
  return hipModuleLaunchKernel(k.batch, blocks, 1, 1, QMCD_BLOCK, 1, 1, 0, st, params, nullptr);
}

}  // namespace qmcj
