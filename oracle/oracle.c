/*
 * Reference oracle for the randomly shifted rank-1 lattice (R1SL) QMC path.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is a plain, slow, fp64 CPU statement of
 * what the integrator computes.  It is called by the test-suite, by the
 * package smoke check and by the CPU-baseline leg of the benchmark; the
 * product never links or calls it.  It shares no code with the GPU library.
 *
 * Every function follows a passage of Borowka et al., "A GPU compatible
 * quasi-Monte Carlo integrator interfaced to pySecDec" (CPC 2019):
 *   - lattice rule, shifts, per-shift estimates ........ Sec. 2.1, eq. (lattice)
 *   - error estimate from the m shifts ................. Sec. 2.1, eq. (lattice-error)
 *   - Korobov weight and map ........................... Sec. 2.3, eq. (korobov)
 *   - baker's (tent) map ............................... Sec. 2.3, eq. (baker)
 *   - variance-reduction map (PolySingular) ............ Sec. 2.4, eq. (ISfit), App. A.5 table
 *   - CDF of |f| per dimension for the fit ............. Sec. 2.4
 *   - CBC criterion (Korobov space, alpha = 2) ......... Sec. 2.2, App. A.3
 * Readings where the paper is silent (each listed in the design notes):
 *   - shifts come from SplitMix64 (Steele, Lea and Flood 2014), 53-bit
 *     conversion (x >> 11) * 2^-53, drawn shift-major;
 *   - u = r/n + Delta, minus 1 when >= 1, r = (k z_j) mod n exactly;
 *   - a point whose transform weight is exactly 0 contributes exactly 0 and
 *     the integrand is not evaluated there;
 *   - the baker map has weight 1 (it preserves Lebesgue measure);
 *   - contour deformation z_j = x_j - i lambda x_j (1 - x_j) dF/dx_j, with the
 *     Jacobian determinant as weight, principal branch for the powers and
 *     arg = -pi on the negative real axis (Feynman -i0);
 *   - per-shift sums are accumulated in double-double.
 *
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off -fopenmp -shared -fPIC
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OR_MAX_DIM 32

enum { OR_T_NONE = 0, OR_T_KOROBOV = 1, OR_T_BAKER = 2, OR_T_SIDI = 3 };

typedef struct {
  uint32_t dim;
  uint32_t n_u, n_f;      /* monomials of U, then of F; n_f = 0 means F == 1 */
  const double* coef;     /* [n_u + n_f] */
  const uint8_t* expo;    /* [(n_u + n_f) * dim], row-major */
  double pow_u, pow_f, prefactor;
  int32_t deform;         /* 1: complex result under contour deformation */
  double lambda;
  int32_t genz;           /* 0: U^a F^b; 1..6: Genz family with coef = [c_0..c_d-1, w_0..w_d-1] */
} oracle_desc;

/* ------------------------------------------------------------------ */
/* double-double accumulator (Knuth TwoSum); error ~ n * 2^-106        */

typedef struct { double hi, lo; } dd_t;

static inline void dd_add(dd_t* a, double b) {
  double s = a->hi + b;
  double bb = s - a->hi;
  double err = (a->hi - (s - bb)) + (b - bb);
  double lo = a->lo + err;
  double hi = s + lo;
  a->lo = lo - (hi - s);
  a->hi = hi;
}

static inline void dd_add_dd(dd_t* a, dd_t b) {
  dd_add(a, b.hi);
  dd_add(a, b.lo);
}

/* ------------------------------------------------------------------ */
/* shifts: SplitMix64                                                   */

uint64_t oracle_splitmix64_next(uint64_t* state) {
  uint64_t z = (*state += 0x9e3779b97f4a7c15ULL);
  z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
  z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
  return z ^ (z >> 31);
}

/* Delta[s][j] in [0,1), s = 0..m-1, j = 0..d-1, drawn in that order. */
void oracle_shifts(uint64_t seed, uint32_t m, uint32_t d, double* out) {
  uint64_t st = seed;
  for (uint64_t i = 0; i < (uint64_t)m * d; ++i)
    out[i] = (double)(oracle_splitmix64_next(&st) >> 11) * 0x1.0p-53;
}

/* ------------------------------------------------------------------ */
/* lattice: r_j = (k z_j) mod n, exact through a 128-bit product         */

static inline uint64_t lattice_index(uint64_t k, uint64_t zj, uint64_t n) {
  return (uint64_t)(((unsigned __int128)k * zj) % n);
}

void oracle_lattice_indices(uint64_t n, uint32_t d, const uint64_t* z, uint64_t k0,
                            uint64_t count, uint64_t* out) {
  for (uint64_t i = 0; i < count; ++i)
    for (uint32_t j = 0; j < d; ++j) out[i * d + j] = lattice_index(k0 + i, z[j], n);
}

/* fractional part of r/n + Delta (eq. lattice, curly brackets) */
static inline double shifted_coord(uint64_t r, uint64_t n, double delta) {
  double u = (double)r / (double)n + delta;
  if (u >= 1.0) u -= 1.0;
  return u;
}

/* ------------------------------------------------------------------ */
/* periodizing transforms (Sec. 2.3)                                    */

static double binom(int a, int b) {
  double c = 1.0;
  for (int i = 1; i <= b; ++i) c = c * (double)(a - b + i) / (double)i;
  return c;
}

/* eq. (korobov): omega(u) = (r0+r1+1) C(r0+r1, r0) u^r0 (1-u)^r1 */
double oracle_korobov_omega(double u, int r0, int r1) {
  return (double)(r0 + r1 + 1) * binom(r0 + r1, r0) * pow(u, r0) * pow(1.0 - u, r1);
}

/* phi(u) = int_0^u omega: for integer r0, r1 this is the regularized
 * incomplete beta function I_u(r0+1, r1+1), i.e. the binomial tail
 * sum_{k=r0+1}^{R} C(R,k) u^k (1-u)^(R-k) with R = r0+r1+1. */
double oracle_korobov_phi(double u, int r0, int r1) {
  int R = r0 + r1 + 1;
  double s = 0.0;
  for (int k = r0 + 1; k <= R; ++k) s += binom(R, k) * pow(u, k) * pow(1.0 - u, R - k);
  return s;
}

/* eq. (baker): phi(u) = 2u for u <= 1/2, 2 - 2u otherwise; weight 1 */
double oracle_baker_phi(double u) { return u <= 0.5 ? 2.0 * u : 2.0 - 2.0 * u; }

/* eq. (sidi): omega_r(u) = c_r sin(pi u)^r, normalised by
 * c_r = pi 2^-r Gamma(r+1) / Gamma((r+1)/2)^2 */
double oracle_sidi_omega(double u, int r) {
  double g = tgamma(0.5 * (r + 1.0));
  double c = M_PI * pow(2.0, -r) * tgamma(r + 1.0) / (g * g);
  return c * pow(sin(M_PI * u), r);
}

/* Gauss-Legendre nodes and weights on [-1, 1] (Newton on P_N) */
#define OR_GL_N 32
static double gl_x[OR_GL_N], gl_w[OR_GL_N];
static int gl_ready = 0;
static void gl_init(void) {
  if (gl_ready) return;
  for (int i = 0; i < OR_GL_N; ++i) {
    double x = cos(M_PI * (i + 0.75) / (OR_GL_N + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = x;
      for (int k = 2; k <= OR_GL_N; ++k) {
        double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = OR_GL_N * (x * p1 - p0) / (x * x - 1.0);
      double dx = p1 / dp;
      x -= dx;
      if (fabs(dx) < 1e-17) break;
    }
    gl_x[i] = x;
    gl_w[i] = 2.0 / ((1.0 - x * x) * dp * dp);
  }
  gl_ready = 1;
}
/* filled once when the library loads, before any (threaded) caller */
__attribute__((constructor)) static void gl_ctor(void) { gl_init(); }

/* phi_r(u) = int_0^u omega_r(t) dt by composite Gauss-Legendre (8 panels of
 * 32 nodes; the integrand is entire, so this is exact to rounding) */
double oracle_sidi_phi(double u, int r) {
  gl_init();
  const int panels = 8;
  double h = u / panels, s = 0.0;
  for (int p = 0; p < panels; ++p) {
    double a = p * h, ps = 0.0;
    for (int i = 0; i < OR_GL_N; ++i) ps += gl_w[i] * oracle_sidi_omega(a + 0.5 * h * (gl_x[i] + 1.0), r);
    s += 0.5 * h * ps;
  }
  return s;
}

/* ------------------------------------------------------------------ */
/* variance-reduction map (Sec. 2.4, eq. ISfit; App. A.5 PolySingular)  */

void oracle_vr_map(const double* a, double y, double* x, double* dxdy) {
  double p0 = a[0], p1 = a[1], p2 = fabs(a[2]), p3 = fabs(a[3]), p4 = a[4], p5 = a[5];
  double c3 = 1.0 - p2 - p3 - p4 - p5;
  double t0 = y * (p0 - 1.0) / (p0 - y);
  double t1 = y * (p1 - 1.0) / (p1 - y);
  *x = p2 * t0 + p3 * t1 + p4 * y + p5 * y * y + c3 * y * y * y;
  /* d/dy [y (p-1)/(p-y)] = p (p-1) / (p-y)^2 */
  *dxdy = p2 * p0 * (p0 - 1.0) / ((p0 - y) * (p0 - y)) + p3 * p1 * (p1 - 1.0) / ((p1 - y) * (p1 - y)) +
          p4 + 2.0 * p5 * y + 3.0 * c3 * y * y;
}

/* Residuals of the variance-reduction fit (Sec. 2.4): the map p of eq. ISfit
   is fitted to the inverse of the per-dimension CDF, sampled at the points
   (cdf[b], edge[b]); r[b] = p(cdf[b]; a) - edge[b]. */
void oracle_vr_residuals(const double* a, const double* cdf, const double* edge, uint32_t count, double* r) {
  for (uint32_t b = 0; b < count; ++b) {
    double x, dx;
    oracle_vr_map(a, cdf[b], &x, &dx);
    r[b] = x - edge[b];
  }
}

/* ------------------------------------------------------------------ */
/* integrand f = prefactor * U^pow_u * F^pow_f                          */

static double ipow(double x, int e) {
  double r = 1.0;
  for (int i = 0; i < e; ++i) r *= x;
  return r;
}

static double poly_real(const oracle_desc* D, uint32_t first, uint32_t count, const double* x) {
  double s = 0.0;
  for (uint32_t i = first; i < first + count; ++i) {
    double t = D->coef[i];
    for (uint32_t j = 0; j < D->dim; ++j) t *= ipow(x[j], D->expo[(size_t)i * D->dim + j]);
    s += t;
  }
  return s;
}

static double f_real(const oracle_desc* D, const double* x) {
  double U = poly_real(D, 0, D->n_u, x);
  double f = D->prefactor * pow(U, D->pow_u);
  if (D->n_f > 0) f *= pow(poly_real(D, D->n_u, D->n_f, x), D->pow_f);
  return f;
}

static double complex cipow(double complex z, int e) {
  double complex r = 1.0;
  for (int i = 0; i < e; ++i) r *= z;
  return r;
}

static double complex poly_cplx(const oracle_desc* D, uint32_t first, uint32_t count,
                                const double complex* z) {
  double complex s = 0.0;
  for (uint32_t i = first; i < first + count; ++i) {
    double complex t = D->coef[i];
    for (uint32_t j = 0; j < D->dim; ++j) t *= cipow(z[j], D->expo[(size_t)i * D->dim + j]);
    s += t;
  }
  return s;
}

/* principal branch; on the negative real axis the -i0 side (arg = -pi) */
static double complex cpow_feynman(double complex w, double p) {
  if (cimag(w) == 0.0) w = CMPLX(creal(w), -0.0);
  return cexp(p * clog(w));
}

/* dF/dx_j and d2F/dx_j dx_l by exponent arithmetic (no division by x) */
static void grad_hess_F(const oracle_desc* D, const double* x, double* g, double* H) {
  uint32_t d = D->dim;
  for (uint32_t j = 0; j < d; ++j) g[j] = 0.0;
  for (uint32_t j = 0; j < d * d; ++j) H[j] = 0.0;
  for (uint32_t i = D->n_u; i < D->n_u + D->n_f; ++i) {
    const uint8_t* e = D->expo + (size_t)i * d;
    for (uint32_t j = 0; j < d; ++j) {
      if (e[j] == 0) continue;
      double t = D->coef[i] * e[j] * ipow(x[j], e[j] - 1);
      for (uint32_t q = 0; q < d; ++q)
        if (q != j) t *= ipow(x[q], e[q]);
      g[j] += t;
      for (uint32_t l = 0; l < d; ++l) {
        double h;
        if (l == j) {
          if (e[j] < 2) continue;
          h = D->coef[i] * e[j] * (e[j] - 1) * ipow(x[j], e[j] - 2);
          for (uint32_t q = 0; q < d; ++q)
            if (q != j) h *= ipow(x[q], e[q]);
        } else {
          if (e[l] == 0) continue;
          h = D->coef[i] * e[j] * e[l] * ipow(x[j], e[j] - 1) * ipow(x[l], e[l] - 1);
          for (uint32_t q = 0; q < d; ++q)
            if (q != j && q != l) h *= ipow(x[q], e[q]);
        }
        H[j * d + l] += h;
      }
    }
  }
}

/* determinant by Gaussian elimination with partial pivoting */
static double complex cdet(double complex* A, int d) {
  double complex det = 1.0;
  for (int c = 0; c < d; ++c) {
    int p = c;
    for (int r = c + 1; r < d; ++r)
      if (cabs(A[r * d + c]) > cabs(A[p * d + c])) p = r;
    if (cabs(A[p * d + c]) == 0.0) return 0.0;
    if (p != c) {
      for (int k = 0; k < d; ++k) {
        double complex t = A[c * d + k];
        A[c * d + k] = A[p * d + k];
        A[p * d + k] = t;
      }
      det = -det;
    }
    det *= A[c * d + c];
    for (int r = c + 1; r < d; ++r) {
      double complex fct = A[r * d + c] / A[c * d + c];
      for (int k = c; k < d; ++k) A[r * d + k] -= fct * A[c * d + k];
    }
  }
  return det;
}

/* deformed integrand: z = x - i lambda x (1-x) grad F(x);
 * f = prefactor * det(dz/dx) * U(z)^pow_u * F(z)^pow_f.
 * *sign_flag is set when Im F(z) > 0 (contour on the wrong side). */
static double complex f_complex(const oracle_desc* D, const double* x, int* sign_flag) {
  uint32_t d = D->dim;
  double g[OR_MAX_DIM], H[OR_MAX_DIM * OR_MAX_DIM];
  double complex z[OR_MAX_DIM], J[OR_MAX_DIM * OR_MAX_DIM];
  grad_hess_F(D, x, g, H);
  for (uint32_t j = 0; j < d; ++j) z[j] = x[j] - I * D->lambda * x[j] * (1.0 - x[j]) * g[j];
  for (uint32_t j = 0; j < d; ++j)
    for (uint32_t l = 0; l < d; ++l) {
      double v = x[j] * (1.0 - x[j]) * H[j * d + l];
      if (j == l) v += (1.0 - 2.0 * x[j]) * g[j];
      J[j * d + l] = (j == l ? 1.0 : 0.0) - I * D->lambda * v;
    }
  double complex det = cdet(J, (int)d);
  double complex U = poly_cplx(D, 0, D->n_u, z);
  double complex f = D->prefactor * det * cpow_feynman(U, D->pow_u);
  if (D->n_f > 0) {
    double complex F = poly_cplx(D, D->n_u, D->n_f, z);
    if (cimag(F) > 0.0) *sign_flag = 1;
    f *= cpow_feynman(F, D->pow_f);
  }
  return f;
}

/* The six test families of Genz as the paper lists them (Sec. 5.3), with
 * parameters c_i > 0 and 0 <= w_i <= 1. */
static double f_genz(const oracle_desc* D, const double* x) {
  const uint32_t d = D->dim;
  const double* c = D->coef;
  const double* w = D->coef + d;
  double s = 0.0, p = 1.0;
  switch (D->genz) {
    case 1: /* oscillatory */
      s = 2.0 * M_PI * w[0];
      for (uint32_t j = 0; j < d; ++j) s += c[j] * x[j];
      return cos(s);
    case 2: /* product peak */
      for (uint32_t j = 0; j < d; ++j) p *= 1.0 / (1.0 / (c[j] * c[j]) + (x[j] - w[j]) * (x[j] - w[j]));
      return p;
    case 3: /* corner peak */
      s = 1.0;
      for (uint32_t j = 0; j < d; ++j) s += c[j] * x[j];
      return pow(s, -(double)(d + 1));
    case 4: /* Gaussian */
      for (uint32_t j = 0; j < d; ++j) s += c[j] * c[j] * (x[j] - w[j]) * (x[j] - w[j]);
      return exp(-s);
    case 5: /* continuous (C^0) */
      for (uint32_t j = 0; j < d; ++j) s += c[j] * fabs(x[j] - w[j]);
      return exp(-s);
    case 6: /* discontinuous */
      if (x[0] > w[0] || (d > 1 && x[1] > w[1])) return 0.0;
      for (uint32_t j = 0; j < d; ++j) s += c[j] * x[j];
      return exp(s);
  }
  return NAN;
}

/* f at one point x in [0,1]^d (no transform): real or complex */
int oracle_eval_point(const oracle_desc* D, const double* x, double* re, double* im) {
  int flag = 0;
  if (D->genz) {
    *re = f_genz(D, x);
    *im = 0.0;
  } else if (D->deform) {
    double complex f = f_complex(D, x, &flag);
    *re = creal(f);
    *im = cimag(f);
  } else {
    *re = f_real(D, x);
    *im = 0.0;
  }
  return flag;
}

/* ------------------------------------------------------------------ */
/* one lattice point: u -> phi (transform) -> p (VR) -> f, weight       */

typedef struct {
  const oracle_desc* D;
  uint64_t n;
  const uint64_t* z;
  int tkind, r0, r1;
  const double* vr; /* d*6 or NULL */
} point_ctx;

/* returns 1 when the contribution is non-finite; adds into re/im */
static int contribution(const point_ctx* P, uint64_t k, const double* delta, double* re, double* im,
                        int* sign_flag) {
  const oracle_desc* D = P->D;
  uint32_t d = D->dim;
  double x[OR_MAX_DIM];
  double w = 1.0;
  for (uint32_t j = 0; j < d; ++j) {
    double u = shifted_coord(lattice_index(k, P->z[j], P->n), P->n, delta[j]);
    double y;
    if (P->tkind == OR_T_KOROBOV) {
      y = oracle_korobov_phi(u, P->r0, P->r1);
      w *= oracle_korobov_omega(u, P->r0, P->r1);
    } else if (P->tkind == OR_T_BAKER) {
      y = oracle_baker_phi(u);
    } else if (P->tkind == OR_T_SIDI) {
      y = oracle_sidi_phi(u, P->r0);
      w *= oracle_sidi_omega(u, P->r0);
    } else {
      y = u;
    }
    if (P->vr) {
      double xx, dx;
      oracle_vr_map(P->vr + 6 * j, y, &xx, &dx);
      x[j] = xx;
      w *= dx;
    } else {
      x[j] = y;
    }
  }
  *re = 0.0;
  *im = 0.0;
  if (w == 0.0) return 0;
  double fr, fi;
  int fl = oracle_eval_point(D, x, &fr, &fi);
  if (fl) *sign_flag = 1;
  *re = w * fr;
  *im = w * fi;
  return !(isfinite(*re) && isfinite(*im));
}

/*
 * Per-shift sums S_s = sum_{k in [k0,k1)} w(x_k) f(x_k) for each requested
 * shift (eq. lattice without the 1/n), together with A_s = sum |.| per
 * component (the scale for tolerances), the count of non-finite
 * contributions and of points with Im F(z) > 0.
 * shifts: [m * d]; shift_ids: which rows to sum (n_ids of them).
 * Outputs are indexed by position in shift_ids.
 */
int oracle_shift_sums(const oracle_desc* D, uint64_t n, const uint64_t* z, uint32_t m,
                      const double* shifts, int tkind, int r0, int r1, const double* vr,
                      uint64_t k0, uint64_t k1, const uint32_t* shift_ids, uint32_t n_ids,
                      double* sum_re, double* sum_im, double* abs_re, double* abs_im,
                      uint64_t* nonfinite, uint64_t* sign_points, int nthreads) {
  if (D->dim == 0 || D->dim > OR_MAX_DIM || n == 0 || k1 > n || k0 > k1) return -1;
  point_ctx P = {D, n, z, tkind, r0, r1, vr};
  const uint64_t CH = 1 << 14;
  uint64_t nchunks = (k1 - k0 + CH - 1) / CH;
  for (uint32_t t = 0; t < n_ids; ++t) {
    uint32_t s = shift_ids[t];
    if (s >= m) return -1;
    const double* delta = shifts + (size_t)s * D->dim;
    dd_t* cre = (dd_t*)calloc(nchunks ? nchunks : 1, sizeof(dd_t));
    dd_t* cim = (dd_t*)calloc(nchunks ? nchunks : 1, sizeof(dd_t));
    dd_t* are = (dd_t*)calloc(nchunks ? nchunks : 1, sizeof(dd_t));
    dd_t* aim = (dd_t*)calloc(nchunks ? nchunks : 1, sizeof(dd_t));
    uint64_t* nf = (uint64_t*)calloc(nchunks ? nchunks : 1, sizeof(uint64_t));
    uint64_t* sp = (uint64_t*)calloc(nchunks ? nchunks : 1, sizeof(uint64_t));
#pragma omp parallel for schedule(dynamic, 1) num_threads(nthreads > 0 ? nthreads : 1)
    for (uint64_t c = 0; c < nchunks; ++c) {
      uint64_t a = k0 + c * CH, b = a + CH < k1 ? a + CH : k1;
      dd_t r = {0, 0}, i = {0, 0}, ar = {0, 0}, ai = {0, 0};
      uint64_t bad = 0, sgn = 0;
      for (uint64_t k = a; k < b; ++k) {
        double vr_, vi_;
        int flag = 0;
        bad += (uint64_t)contribution(&P, k, delta, &vr_, &vi_, &flag);
        sgn += (uint64_t)flag;
        dd_add(&r, vr_);
        dd_add(&i, vi_);
        dd_add(&ar, fabs(vr_));
        dd_add(&ai, fabs(vi_));
      }
      cre[c] = r;
      cim[c] = i;
      are[c] = ar;
      aim[c] = ai;
      nf[c] = bad;
      sp[c] = sgn;
    }
    dd_t r = {0, 0}, i = {0, 0}, ar = {0, 0}, ai = {0, 0};
    uint64_t bad = 0, sgn = 0;
    for (uint64_t c = 0; c < nchunks; ++c) { /* fixed merge order */
      dd_add_dd(&r, cre[c]);
      dd_add_dd(&i, cim[c]);
      dd_add_dd(&ar, are[c]);
      dd_add_dd(&ai, aim[c]);
      bad += nf[c];
      sgn += sp[c];
    }
    sum_re[t] = r.hi + r.lo;
    if (sum_im) sum_im[t] = i.hi + i.lo;
    if (abs_re) abs_re[t] = ar.hi + ar.lo;
    if (abs_im) abs_im[t] = ai.hi + ai.lo;
    if (nonfinite) nonfinite[t] = bad;
    if (sign_points) sign_points[t] = sgn;
    free(cre);
    free(cim);
    free(are);
    free(aim);
    free(nf);
    free(sp);
  }
  return 0;
}

/*
 * Histograms of |f| over one shifted lattice, the data from which the
 * per-dimension CDF of Sec. 2.4 is estimated: for every point x_k (no
 * periodizing transform, no VR map), hist[j][floor(x_kj * bins)] += |f(x_k)|
 * for every dimension j.  |f| is the modulus for complex integrands.
 */
int oracle_histogram(const oracle_desc* D, uint64_t n, const uint64_t* z, const double* delta,
                     uint32_t bins, double* hist) {
  uint32_t d = D->dim;
  if (d == 0 || d > OR_MAX_DIM || bins == 0) return -1;
  dd_t* acc = (dd_t*)calloc((size_t)d * bins, sizeof(dd_t));
  double x[OR_MAX_DIM];
  for (uint64_t k = 0; k < n; ++k) {
    for (uint32_t j = 0; j < d; ++j) x[j] = shifted_coord(lattice_index(k, z[j], n), n, delta[j]);
    double fr, fi;
    oracle_eval_point(D, x, &fr, &fi);
    double a = D->deform ? hypot(fr, fi) : fabs(fr);
    for (uint32_t j = 0; j < d; ++j) {
      uint32_t b = (uint32_t)floor(x[j] * (double)bins);
      if (b >= bins) b = bins - 1;
      dd_add(&acc[(size_t)j * bins + b], a);
    }
  }
  for (size_t i = 0; i < (size_t)d * bins; ++i) hist[i] = acc[i].hi + acc[i].lo;
  free(acc);
  return 0;
}

/* ------------------------------------------------------------------ */
/* CBC (Sec. 2.2, App. A.3): Korobov space alpha = 2, kernel             */
/* omega(x) = 2 pi^2 (x^2 - x + 1/6), product weights, beta = 1          */

static double cbc_kernel(uint64_t r, uint64_t n) {
  double x = (double)r / (double)n;
  return 2.0 * M_PI * M_PI * (x * x - x + 1.0 / 6.0);
}

/* sum over k in [k0, k1) of prod_j (1 + gamma_j omega({k z_j / n})) - 1 */
/* sum over k in [k0, k1) of prod_j (1 + gamma_j omega({k z_j / n})) - 1, as
 * the two words of a double-double: a range's sum can be many orders of
 * magnitude larger than the whole lattice's, so callers that split k add the
 * words exactly (one double per range would lose the small total). */
void oracle_cbc_partial(uint64_t n, uint32_t d, const uint64_t* z, const double* gamma, uint64_t k0, uint64_t k1,
                        double* hi_lo) {
  dd_t s = {0, 0};
  for (uint64_t k = k0; k < k1; ++k) {
    double p = 1.0;
    for (uint32_t j = 0; j < d; ++j) p *= 1.0 + gamma[j] * cbc_kernel(lattice_index(k, z[j], n), n);
    dd_add(&s, p - 1.0);
  }
  hi_lo[0] = s.hi;
  hi_lo[1] = s.lo;
}

/* e^2(z) = -1 + (1/n) sum_k prod_j (1 + gamma_j omega({k z_j / n})) */
double oracle_cbc_criterion(uint64_t n, uint32_t d, const uint64_t* z, const double* gamma) {
  double s[2];
  oracle_cbc_partial(n, d, z, gamma, 0, n, s);
  return (s[0] + s[1]) / (double)n;
}

static uint64_t gcd_u64(uint64_t a, uint64_t b) {
  while (b) {
    uint64_t t = a % b;
    a = b;
    b = t;
  }
  return a;
}

/* Brute-force CBC: z_1 = 1; each next component minimises e^2 over all
 * candidates 1..(n-1)/2 coprime to n; ties within rtol -> smallest z. */
int oracle_cbc_brute(uint64_t n, uint32_t d, const double* gamma, double tie_rtol, uint64_t* z) {
  if (n < 2 || d == 0) return -1;
  double* p = (double*)malloc(n * sizeof(double));
  for (uint64_t k = 0; k < n; ++k) p[k] = 1.0;
  z[0] = 1;
  for (uint64_t k = 0; k < n; ++k) p[k] *= 1.0 + gamma[0] * cbc_kernel(k % n, n);
  uint64_t half = (n - 1) / 2 ? (n - 1) / 2 : 1;
  double* crit = (double*)malloc((half + 1) * sizeof(double));
  for (uint32_t s = 1; s < d; ++s) {
    double best = INFINITY;
    for (uint64_t c = 1; c <= half; ++c) {
      crit[c] = INFINITY;
      if (gcd_u64(c, n) != 1) continue;
      dd_t acc = {0, 0};
      for (uint64_t k = 0; k < n; ++k)
        dd_add(&acc, p[k] * (1.0 + gamma[s] * cbc_kernel(lattice_index(k, c, n), n)) - 1.0);
      crit[c] = (acc.hi + acc.lo) / (double)n;
      if (crit[c] < best) best = crit[c];
    }
    uint64_t pick = 0;
    for (uint64_t c = 1; c <= half; ++c)
      if (crit[c] <= best + tie_rtol * fabs(best)) {
        pick = c;
        break;
      }
    z[s] = pick;
    for (uint64_t k = 0; k < n; ++k) p[k] *= 1.0 + gamma[s] * cbc_kernel(lattice_index(k, pick, n), n);
  }
  free(p);
  free(crit);
  return 0;
}

int oracle_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}
