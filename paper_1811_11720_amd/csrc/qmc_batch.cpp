// qmc_batch.cpp -- many integrals in one persistent launch per kernel variant.
//
// A round evaluates the current lattice of every job.  Each job is cut into
// tiles of T points x S shifts (T depends only on the job's own n, so the
// per-shift sums of a job are the same whether it runs alone or in any
// mix).  Jobs are grouped by kernel variant (dimension class, real/complex,
// fp64/fp32 evaluation) and ordered heaviest first; per variant one
// persistent kernel drains the tile list, then one fixed-order reduction sums
// every job's tile columns.  The launches of a round are captured into a HIP
// graph on a private stream and replayed on the context's stream.
//
// run_requests adds the paper's growth loop (Sec. 3.3.1) on top: all
// unconverged requests move to their next lattice and run together in the
// next round.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <cstdio>
#include <numeric>

#include "qmc_host.h"

namespace qmch {

namespace {

double cost_per_eval(const qmc_integrand* f) {
  double c = (double)(f->n_u + f->n_f) * f->dim + 10.0 * f->dim;
  if (f->flags & QMC_DEFORM) c = c * 6.0 + 2.0 * f->dim * f->dim * f->dim;
  return c;
}

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

}  // namespace

uint64_t batch_tile_points(const qmc_context* c, uint64_t tuned, bool cplx, uint64_t n) {
  const uint64_t tmin = tuned ? tuned : (cplx ? c->batch_tile_complex : c->batch_tile_real);
  const uint64_t tp = std::max<uint64_t>(tmin, (n + c->batch_max_ktiles - 1) / c->batch_max_ktiles);
  return (tp + QMCD_BLOCK - 1) / QMCD_BLOCK * QMCD_BLOCK;
}

uint64_t batch_ktiles_bound(const qmc_context* c, uint64_t n) {
  // every tile holds a whole number (>= 1) of blocks and at least n / batch_max_ktiles points
  const uint64_t tp = batch_tile_points(c, QMCD_BLOCK, false, n);
  return (n + tp - 1) / tp;
}

size_t batch_job_bytes(size_t rows, uint64_t ktiles, uint32_t m, uint32_t dim) {
  // arena entries of one job (run_batch's layout) plus its share of the alignment padding
  return sizeof(qmcd::EvalArgs) + 4 + 8 + rows * (sizeof(qmck::RowRef) + 8 * ktiles + 8) + (size_t)m * dim * 8 + 8 +
         256;
}

int run_batch(qmc_context* c, std::vector<BatchJob*>& jobs, double* kernel_seconds) {
  const uint32_t J = (uint32_t)jobs.size();
  if (kernel_seconds) *kernel_seconds = 0.0;
  if (J == 0) return QMC_OK;
  struct Plan {
    qmck::BatchVariant var;
    int variant;  // var.index()
    uint32_t rows, ktiles, groups;
    uint64_t tile_points;
    size_t part_off, sh_off, row0;
    double cost;
    bool use_jit = false;  // the integrand's specialised batch kernel (QMC_SPECIALISE)
    qmcj::Kernel jk;
  };
  std::vector<Plan> plan(J);
  std::vector<hipFunction_t> jit_fns;  // distinct specialised kernels in this call
  size_t n_part = 0, n_sh = 0, n_rows = 0;
  for (uint32_t i = 0; i < J; ++i) {
    BatchJob& b = *jobs[i];
    const qmc_integrand* f = b.f;
    const bool cplx = (f->flags & QMC_DEFORM) != 0, fp32 = (f->flags & QMC_EVAL_FP32) != 0;
    Plan& p = plan[i];
    const int dclass = qmck::dim_class(f->dim, cplx);
    qmcd::EvalArgs probe;
    int tsel = 0;
    int trc = set_transform(probe, b.t, tsel);
    if (trc) return trc;
    p.var = qmck::BatchVariant{dclass, qmck::batch_tkc(tsel, f->has_vr), cplx, fp32};
    p.variant = p.var.index();
    if (!cplx && !fp32 && (f->flags & QMC_SPECIALISE) && c->jit && specialised_kernel(c, b.f, tsel, &p.jk) == 0 &&
        p.jk.batch) {
      // jobs of one specialised kernel form a launch of their own
      p.use_jit = true;
      auto it = std::find(jit_fns.begin(), jit_fns.end(), p.jk.batch);
      p.variant = qmck::BATCH_VARIANTS + (int)(it - jit_fns.begin());
      if (it == jit_fns.end()) jit_fns.push_back(p.jk.batch);
    }
    const uint32_t S = cplx ? qmck::S_COMPLEX : qmck::S_REAL;
    const uint64_t tp = batch_tile_points(c, p.use_jit ? 0 : c->batch_tile[p.variant], cplx, b.n);
    p.tile_points = tp;
    p.ktiles = (uint32_t)((b.n + tp - 1) / tp);
    p.groups = (b.m + S - 1) / S;
    p.rows = cplx ? 2 * b.m : b.m;
    p.part_off = n_part;
    n_part += (size_t)p.rows * p.ktiles;
    p.sh_off = n_sh;
    n_sh += (size_t)b.m * f->dim;
    p.row0 = n_rows;
    n_rows += p.rows;
    p.cost = cost_per_eval(f) * (double)b.n * b.m;
  }
  // variants present, items ordered heaviest first
  std::map<int, std::vector<uint32_t>> by_var;
  for (uint32_t i = 0; i < J; ++i) by_var[plan[i].variant].push_back(i);
  for (auto& kv : by_var)
    std::stable_sort(kv.second.begin(), kv.second.end(), [&](uint32_t x, uint32_t y) { return plan[x].cost > plan[y].cost; });
  const uint32_t NV = (uint32_t)by_var.size();

  // device layout
  size_t off = 0;
  const size_t o_items = off;
  off = align256(off + (size_t)J * sizeof(qmcd::EvalArgs));
  const size_t o_order = off;
  off = align256(off + (size_t)J * 4);
  const size_t o_prefix = off;
  off = align256(off + (size_t)(J + NV) * 4);
  const size_t o_rows = off;
  off = align256(off + n_rows * sizeof(qmck::RowRef));
  const size_t o_sh = off;
  off = align256(off + n_sh * 8);
  const size_t upload = off;  // everything above comes from the host
  const size_t o_part = off;
  off = align256(off + n_part * 8);
  const size_t o_out = off;
  off = align256(off + n_rows * 8 + (size_t)J * 8);
  const size_t o_cnt = off;
  off = align256(off + (size_t)NV * 4);
  char* ws = nullptr;
  int rc = scratch(c, off, &ws);
  if (rc) return rc;
  rc = stage(c, std::max(upload, n_rows * 8 + (size_t)J * 8));
  if (rc) return rc;
  char* h = (char*)c->h_stage;
  std::memset(h, 0, upload);

  qmcd::EvalArgs* items = (qmcd::EvalArgs*)(h + o_items);
  qmck::RowRef* rows = (qmck::RowRef*)(h + o_rows);
  double* shifts = (double*)(h + o_sh);
  double* d_part = (double*)(ws + o_part);
  double* d_out = (double*)(ws + o_out);
  unsigned long long* d_sign = (unsigned long long*)(ws + o_out + n_rows * 8);
  for (uint32_t i = 0; i < J; ++i) {
    BatchJob& b = *jobs[i];
    const Plan& p = plan[i];
    qmcd::EvalArgs& a = items[i];
    int tsel = 0;
    rc = fill_integrand_args(a, b.f, b.t, tsel);
    if (rc) return rc;
    a.n = b.n;
    a.n_d = (double)b.n;
    a.inv_n = 1.0 / (double)b.n;
    for (uint32_t j = 0; j < b.f->dim; ++j) {
      a.z[j] = b.z[j] % b.n;
      a.step[j] = mulmod(QMCD_BLOCK % b.n, a.z[j], b.n);
    }
    a.m = b.m;
    a.shifts = (const double*)(ws + o_sh) + p.sh_off;
    a.partial = d_part + p.part_off;
    a.nblocks = p.ktiles;
    a.sign_count = d_sign + i;
    a.tile_points = p.tile_points;
    a.ktiles = p.ktiles;
    a.item = i;
    std::memcpy(shifts + p.sh_off, b.shifts, (size_t)b.m * b.f->dim * 8);
    for (uint32_t r = 0; r < p.rows; ++r) {
      rows[p.row0 + r].p = d_part + p.part_off + (size_t)r * p.ktiles;
      rows[p.row0 + r].ncols = p.ktiles;
    }
  }
  uint32_t* order = (uint32_t*)(h + o_order);
  uint32_t* prefix = (uint32_t*)(h + o_prefix);
  struct Launch {
    qmck::BatchVariant var;
    int variant;
    uint32_t first, count, prefix_off;
    bool jit;
    qmcj::Kernel jk;
  };
  std::vector<Launch> launches;
  uint32_t pos = 0, ppos = 0;
  for (auto& kv : by_var) {
    Launch L;
    L.var = plan[kv.second.front()].var;
    L.variant = kv.first;
    L.jit = plan[kv.second.front()].use_jit;
    L.jk = plan[kv.second.front()].jk;
    L.first = pos;
    L.count = (uint32_t)kv.second.size();
    L.prefix_off = ppos;
    uint64_t acc = 0;
    for (uint32_t q = 0; q < L.count; ++q) {
      uint32_t i = kv.second[q];
      order[pos + q] = i;
      prefix[ppos + q] = (uint32_t)acc;
      acc += (uint64_t)plan[i].ktiles * plan[i].groups;
    }
    if (acc >= 0xFFFFFFFFull) return fail(QMC_EINVAL, "batch has more than 2^32 tiles");
    prefix[ppos + L.count] = (uint32_t)acc;
    pos += L.count;
    ppos += L.count + 1;
    launches.push_back(L);
  }
  HIPCHK(hipMemcpyAsync(ws, h, upload, hipMemcpyHostToDevice, c->stream));

  auto enqueue = [&](hipStream_t st) -> int {
    HIPCHK(qmck::launch_fill_u32((uint32_t*)(ws + o_cnt), NV, 0u, st));
    HIPCHK(qmck::launch_fill_u64(d_sign, J, 0ull, st));
    for (uint32_t v = 0; v < (uint32_t)launches.size(); ++v) {
      const Launch& L = launches[v];
      if (L.jit) {
        const uint32_t blocks = (uint32_t)std::max(1, L.jk.occ_batch) * (uint32_t)c->cus;
        HIPCHK(qmcj::launch_batch(L.jk, (const qmcd::EvalArgs*)(ws + o_items), (const uint32_t*)(ws + o_order) + L.first,
                                  (const uint32_t*)(ws + o_prefix) + L.prefix_off, L.count,
                                  (uint32_t*)(ws + o_cnt) + v, blocks, st));
        continue;
      }
      const int sv = L.var.cplx ? 0 : c->batch_sv[L.variant];
      int occ = qmck::occupancy_batch(L.var, sv);
      uint32_t blocks = (uint32_t)std::max(1, occ) * (uint32_t)c->cus;
      HIPCHK(qmck::launch_batch(L.var, sv, (const qmcd::EvalArgs*)(ws + o_items),
                                (const uint32_t*)(ws + o_order) + L.first,
                                (const uint32_t*)(ws + o_prefix) + L.prefix_off, L.count,
                                (uint32_t*)(ws + o_cnt) + v, blocks, st));
    }
    HIPCHK(qmck::launch_finalize_rows((const qmck::RowRef*)(ws + o_rows), (uint32_t)n_rows, d_out, st));
    return QMC_OK;
  };

  if (c->batch_graph) {
    if (!c->cap_stream) HIPCHK(hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking));
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(c->cap_stream, hipStreamCaptureModeThreadLocal));
    int erc = enqueue(c->cap_stream);
    hipError_t ec = hipStreamEndCapture(c->cap_stream, &g);
    if (erc) {
      if (g) (void)hipGraphDestroy(g);
      return erc;
    }
    if (ec != hipSuccess) return fail(QMC_EDEVICE, "hipStreamEndCapture failed: %s", hipGetErrorString(ec));
    hipGraphExec_t ge = nullptr;
    hipError_t ei = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (ei != hipSuccess) return fail(QMC_EDEVICE, "hipGraphInstantiate failed: %s", hipGetErrorString(ei));
    // the device interval starts here, after the host has built the graph
    hipError_t er = hipEventRecord(c->ev0, c->stream);
    hipError_t el = er != hipSuccess ? er : hipGraphLaunch(ge, c->stream);
    if (el != hipSuccess) {
      (void)hipGraphExecDestroy(ge);
      return fail(QMC_EDEVICE, "hipGraphLaunch failed: %s", hipGetErrorString(el));
    }
    HIPCHK(hipEventRecord(c->ev1, c->stream));
    HIPCHK(hipMemcpyAsync(c->h_stage, d_out, n_rows * 8 + (size_t)J * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    (void)hipGraphExecDestroy(ge);
  } else {
    HIPCHK(hipEventRecord(c->ev0, c->stream));
    rc = enqueue(c->stream);
    if (rc) return rc;
    HIPCHK(hipEventRecord(c->ev1, c->stream));
    HIPCHK(hipMemcpyAsync(c->h_stage, d_out, n_rows * 8 + (size_t)J * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
  }
  float ms = 0;
  HIPCHK(hipEventElapsedTime(&ms, c->ev0, c->ev1));
  if (kernel_seconds) *kernel_seconds = ms * 1e-3;
  const unsigned long long* sg = (const unsigned long long*)(c->h_stage + n_rows);
  for (uint32_t i = 0; i < J; ++i) {
    const Plan& p = plan[i];
    jobs[i]->sums.assign(c->h_stage + p.row0, c->h_stage + p.row0 + p.rows);
    jobs[i]->sign_points = sg[i];
  }
  return QMC_OK;
}

int run_requests(qmc_context* c, const qmc_request* reqs, uint32_t count, qmc_result* out, double* shift_sums) {
  auto t0 = std::chrono::steady_clock::now();
  struct St {
    qmc_integrand* f;
    std::vector<double> shifts;
    std::vector<uint64_t> z;
    uint64_t n;
    uint32_t mcur = 0, first_new = 0;  // shifts [first_new, mcur) run next
    std::vector<double> sre, sim;      // per-shift sums at the current lattice
    uint64_t signs = 0;
    bool done = false;
    qmc_result r{};
    BatchJob job;
  };
  std::vector<St> st(count);
  for (uint32_t i = 0; i < count; ++i) {
    const qmc_request& q = reqs[i];
    if (!q.f) return fail(QMC_EINVAL, "request %u has no integrand", i);
    St& s = st[i];
    s.f = const_cast<qmc_integrand*>(q.f);
    if (s.f->ctx != c) return fail(QMC_EINVAL, "request %u: integrand belongs to another context", i);
    if (s.f->genz) return fail(QMC_EUNSUPPORTED, "request %u: Genz integrands run through qmc_integrate", i);
    if (q.m < 1 || q.m > QMC_MAX_SHIFTS) return fail(QMC_EINVAL, "request %u: m=%u", i, q.m);
    const uint32_t dim = s.f->dim;
    if (q.z) {
      int rc = check_lattice(q.n, dim, q.z);
      if (rc) return rc;
      s.n = q.n;
      s.z.assign(q.z, q.z + dim);
    } else {
      uint64_t nn = 0;
      if (next_registered(c, q.n, dim, &nn, true, &s.z) != QMC_OK)
        return fail(QMC_ENOTFOUND, "request %u: no registered lattice with %u components", i, dim);
      s.n = nn;
    }
    s.shifts.resize((size_t)q.m * dim);
    make_shifts(q.seed, q.m, dim, s.shifts.data());
    s.mcur = q.m;
    s.r.m = q.m;
    s.r.path = 2;
  }
  double dev = 0.0;
  for (;;) {
    std::vector<BatchJob*> jobs;
    std::vector<uint32_t> idx;
    for (uint32_t i = 0; i < count; ++i) {
      St& s = st[i];
      if (s.done) continue;
      s.job.f = s.f;
      s.job.n = s.n;
      s.job.z = s.z.data();
      s.job.m = s.mcur - s.first_new;
      s.job.shifts = s.shifts.data() + (size_t)s.first_new * s.f->dim;
      s.job.t = reqs[i].t;
      jobs.push_back(&s.job);
      idx.push_back(i);
    }
    if (jobs.empty()) break;
    double ks = 0.0;
    int rc = run_batch(c, jobs, &ks);
    if (rc) return rc;
    dev += ks;
    for (uint32_t i : idx) {
      St& s = st[i];
      const qmc_request& q = reqs[i];
      const bool cplx = (s.f->flags & QMC_DEFORM) != 0;
      const uint32_t madd = s.mcur - s.first_new, m = s.mcur;
      s.sre.resize(s.first_new);
      s.sim.resize(s.first_new);
      s.sre.insert(s.sre.end(), s.job.sums.begin(), s.job.sums.begin() + madd);
      if (cplx)
        s.sim.insert(s.sim.end(), s.job.sums.begin() + madd, s.job.sums.begin() + 2 * (size_t)madd);
      else
        s.sim.resize(m, 0.0);
      s.signs = (s.first_new ? s.signs : 0) + s.job.sign_points;
      s.r.iterations += 1;
      s.r.evaluations += s.n * (uint64_t)madd;
      s.r.n = s.n;
      s.r.m = m;
      std::vector<double> qs(m);
      for (uint32_t k = 0; k < m; ++k) qs[k] = s.sre[k] / (double)s.n;
      estimate(qs.data(), m, s.r.re, s.r.err_re);
      s.r.im = s.r.err_im = 0.0;
      if (cplx) {
        for (uint32_t k = 0; k < m; ++k) qs[k] = s.sim[k] / (double)s.n;
        estimate(qs.data(), m, s.r.im, s.r.err_im);
      }
      s.r.flags &= ~(uint32_t)(QMC_NONFINITE | QMC_DEFORM_SIGN);
      if (s.signs) s.r.flags |= QMC_DEFORM_SIGN;
      if (s.f->has_vr && s.f->vr_fallback) s.r.flags |= QMC_VR_FALLBACK;
      const bool finite = std::isfinite(s.r.re) && std::isfinite(s.r.im);
      if (!finite) s.r.flags |= QMC_NONFINITE;
      const bool grow = q.rel_tol > 0 || q.abs_tol > 0;
      if (!grow) {
        s.done = true;
        continue;
      }
      if (finite && goal_met(s.r, q.rel_tol, q.abs_tol, q.errormode, cplx)) {
        s.r.flags |= QMC_CONVERGED;
        s.done = true;
        continue;
      }
      GrowthStep g = growth_step(c, q, s.r, s.n, m, s.f->dim, cplx, UINT64_MAX, QMC_MAX_SHIFTS, true);
      if (g.kind == GrowthStep::STOP) {
        s.r.flags |= QMC_MAXEVAL_HIT;
        s.done = true;
      } else if (g.kind == GrowthStep::LATTICE) {
        s.n = g.n;
        s.z.swap(g.z);
        s.first_new = 0;
      } else {
        s.first_new = m;
        s.mcur = g.m;
        s.shifts.resize((size_t)g.m * s.f->dim);
        make_shifts(q.seed, g.m, s.f->dim, s.shifts.data());
      }
    }
  }
  const double wall = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
  size_t off = 0;
  for (uint32_t i = 0; i < count; ++i) {
    St& s = st[i];
    s.r.device_seconds = dev;  // shared launches: the batch's total device time
    s.r.wall_seconds = wall;
    if (out) out[i] = s.r;
    if (shift_sums) {  // the requested m shifts of each request
      const uint32_t m = reqs[i].m;
      std::memcpy(shift_sums + off, s.sre.data(), (size_t)m * 8);
      off += m;
      if (s.f->flags & QMC_DEFORM) {
        std::memcpy(shift_sums + off, s.sim.data(), (size_t)m * 8);
        off += m;
      }
    }
  }
  return QMC_OK;
}

// ---------------------------------------------------------------- autotuning

// Kernel variant of a request (dimension class, transform class, complex, fp32).
static int variant_of(const qmc_request& q, qmck::BatchVariant& v) {
  const qmc_integrand* f = q.f;
  qmcd::EvalArgs probe;
  int tsel = 0;
  int rc = set_transform(probe, q.t, tsel);
  if (rc) return rc;
  const bool cplx = (f->flags & QMC_DEFORM) != 0;
  v = qmck::BatchVariant{qmck::dim_class(f->dim, cplx), qmck::batch_tkc(tsel, f->has_vr), cplx,
                         (f->flags & QMC_EVAL_FP32) != 0};
  return QMC_OK;
}

// Cache lines: "gfx950 <class's largest dimension> <tkc> <complex> <fp32> <sv index> <tile points>".
void load_tune_cache(qmc_context* c) {
  if (c->tune_cache.empty()) return;
  FILE* fh = std::fopen(c->tune_cache.c_str(), "r");
  if (!fh) return;
  int dmax, tkc, cx, f32, sv;
  unsigned long long tile;
  char arch[64];
  while (std::fscanf(fh, "%63s %d %d %d %d %d %llu", arch, &dmax, &tkc, &cx, &f32, &sv, &tile) == 7) {
    if (std::strcmp(arch, "gfx950") != 0 || tkc < 0 || tkc >= qmck::TKC_COUNT || cx < 0 || cx > 1 || f32 < 0 ||
        f32 > 1 || dmax < 1 || dmax > (int)QMC_MAX_DIM)
      continue;
    const int dc = qmck::dim_class((uint32_t)dmax, cx != 0);
    if (qmck::dim_class_max(dc, cx != 0) != dmax) continue;  // not a class boundary
    const int v = qmck::BatchVariant{dc, tkc, cx != 0, f32 != 0}.index();
    if (sv >= 0 && sv < qmck::BATCH_SV_VARIANTS) c->batch_sv[v] = sv;
    if (tile >= 256 && tile <= (1ull << 24)) c->batch_tile[v] = tile;
  }
  std::fclose(fh);
}

// Time each candidate schedule of every variant present in the sample
// (one round, first lattice of each request) and keep the fastest.
int autotune(qmc_context* c, const qmc_request* reqs, uint32_t count, uint32_t* configs_tried) {
  std::map<int, std::vector<uint32_t>> by_var;
  std::map<int, qmck::BatchVariant> vars;
  for (uint32_t i = 0; i < count; ++i) {
    if (!reqs[i].f || reqs[i].f->ctx != c) return fail(QMC_EINVAL, "request %u: bad integrand", i);
    qmck::BatchVariant v;
    int rc = variant_of(reqs[i], v);
    if (rc) return rc;
    // jobs that run in a specialised kernel would time that kernel, not the variant's
    if (!v.cplx && !v.fp32 && (reqs[i].f->flags & QMC_SPECIALISE) && c->jit) continue;
    by_var[v.index()].push_back(i);
    vars[v.index()] = v;
  }
  uint32_t tried = 0;
  for (auto& kv : by_var) {
    const qmck::BatchVariant& var = vars[kv.first];
    const int vi = kv.first;
    std::vector<qmc_request> sub;
    for (uint32_t i : kv.second) {
      qmc_request q = reqs[i];
      q.rel_tol = q.abs_tol = 0.0;  // one lattice
      sub.push_back(q);
    }
    const std::vector<uint64_t> tiles = var.cplx ? std::vector<uint64_t>{512, 1024, 4096}
                                                 : std::vector<uint64_t>{1024, 4096, 16384};
    const int nsv = var.cplx ? 1 : qmck::BATCH_SV_VARIANTS;
    double best = 1e300;
    int best_sv = 0;
    uint64_t best_tile = tiles[0];
    for (int sv = 0; sv < nsv; ++sv) {
      if (!qmck::batch_kernel(var, sv)) continue;
      for (uint64_t tile : tiles) {
        c->batch_sv[vi] = sv;
        c->batch_tile[vi] = tile;
        double t_best = 1e300;
        for (int rep = 0; rep < 2; ++rep) {
          std::vector<qmc_result> out(sub.size());
          int rc = run_requests(c, sub.data(), (uint32_t)sub.size(), out.data(), nullptr);
          if (rc) return rc;
          t_best = std::min(t_best, out[0].device_seconds);
        }
        ++tried;
        if (t_best < best) {
          best = t_best;
          best_sv = sv;
          best_tile = tile;
        }
      }
    }
    c->batch_sv[vi] = best_sv;
    c->batch_tile[vi] = best_tile;
    if (!c->tune_cache.empty()) {
      if (FILE* fh = std::fopen(c->tune_cache.c_str(), "a")) {
        std::fprintf(fh, "gfx950 %d %d %d %d %d %llu\n", qmck::dim_class_max(var.dclass, var.cplx), var.tkc,
                     var.cplx ? 1 : 0, var.fp32 ? 1 : 0,
                     best_sv, (unsigned long long)best_tile);
        std::fclose(fh);
      }
    }
  }
  if (configs_tried) *configs_tried = tried;
  return QMC_OK;
}

}  // namespace qmch

extern "C" int qmc_autotune_batch(qmc_context* c, const qmc_request* reqs, uint32_t count, uint32_t* configs_tried) {
  if (!c || (!reqs && count)) return qmch::fail(QMC_EINVAL, "NULL argument");
  std::lock_guard<std::recursive_mutex> g(c->mu);
  if (c->broken) return qmch::fail(QMC_EDEVICE, "context is unusable after a device error");
  HIPCHK(hipSetDevice(c->device));
  return qmch::autotune(c, reqs, count, configs_tried);
}
