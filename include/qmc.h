/*
 * qmc.h -- C interface of the MI355X rank-1 lattice quasi-Monte Carlo integrator.
 *
 * The library integrates f over the unit hypercube [0,1]^d with a randomly
 * shifted rank-1 lattice rule (Borowka et al., CPC 2019, Sec. 2.1, eq. lattice):
 *
 *     Q^(s) = (1/n) sum_{k=0}^{n-1} w(u_k) f(x(u_k)),
 *     u_k   = { k z / n + Delta_s },   s = 0..m-1,
 *
 * returning the mean of the m per-shift estimates and the error of eq.
 * lattice-error.  x(u) applies a periodizing transform (Sec. 2.3: Korobov
 * eq. korobov, baker eq. baker, or none) and optionally the per-dimension
 * variance-reduction map of Sec. 2.4 (eq. ISfit).  The integrand is a
 * sector-decomposed parameter integral prefactor * U(x)^pow_u * F(x)^pow_f
 * with U, F given as monomial tables; under contour deformation it is
 * complex.  Every step of a call runs in the library's HIP kernels on one
 * gfx950 GPU; per-shift sums are reduced on the device in a fixed order.
 *
 * Conventions for every entry point:
 *   - status codes: QMC_OK (0) on success, QMC_PENDING (1) for a request
 *     still running, negative on error.  No entry point aborts the process;
 *     qmc_last_error() returns a message for the calling thread's last error.
 *   - "host" pointers are ordinary CPU memory; all input arrays are copied
 *     during the call, so the caller may free them on return.  Outputs are
 *     written into caller-owned host memory.  No entry point takes a device
 *     pointer except the optional workspace of qmc_context_create.
 *   - handles (qmc_context, qmc_integrand) are owned by the library and freed
 *     only by their destroy function.
 *   - calls on one context are serialised internally; submit/poll/wait/cancel
 *     may be called from any thread.
 */
#ifndef QMC_H
#define QMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- status */
enum {
  QMC_OK = 0,
  QMC_PENDING = 1,     /* qmc_poll: request not finished yet */
  QMC_EINVAL = -1,     /* an argument is out of range or inconsistent */
  QMC_ENOMEM = -2,     /* device or host memory, or the workspace, is too small */
  QMC_EDEVICE = -3,    /* a HIP call failed; the context is no longer usable */
  QMC_EBUSY = -4,      /* handle still referenced by a pending request */
  QMC_ENOTFOUND = -5,  /* unknown ticket, or no registered lattice */
  QMC_ECANCELED = -6,  /* request was cancelled */
  QMC_EUNSUPPORTED = -7 /* no HIP device / library built without it */
};

/* limits of the device kernels */
#define QMC_MAX_DIM 16        /* integration variables per integrand */
#define QMC_MAX_DIM_DEFORM 12 /* ... per integrand with QMC_DEFORM */
#define QMC_MAX_EXP 15        /* exponent of one variable in one monomial */
#define QMC_MAX_MONOMIALS 1024 /* n_u + n_f */
#define QMC_MAX_SHIFTS 1024   /* m */

/* Message describing the last error on the calling thread ("" if none). */
const char* qmc_last_error(void);

/* Library version as 10000*major + 100*minor + patch. */
int qmc_version(void);

/* ---------------------------------------------------------------- context */
typedef struct qmc_context qmc_context;

/*
 * Create a context on HIP device `device`, launching on `hip_stream`
 * (a hipStream_t; NULL = the library creates its own stream).
 * workspace/workspace_bytes: optional caller-owned device memory (for
 * example a torch tensor's data pointer) from which per-call scratch
 * (shifts, per-block partial sums) is carved; NULL = the library allocates
 * and grows its own scratch.  The workspace must stay valid until
 * qmc_context_destroy.  Errors: QMC_EINVAL (bad device), QMC_EDEVICE.
 */
int qmc_context_create(int device, void* hip_stream, void* workspace, size_t workspace_bytes,
                       qmc_context** out);

/* Destroy; QMC_EBUSY while submitted requests are unfinished.  If integrands
 * created on the context are still alive the context is only marked closed
 * (further calls on it fail) and is freed when its last integrand is
 * destroyed. */
int qmc_context_destroy(qmc_context* ctx);

/*
 * Register the generating vector z[0..dim) for lattice size n in the
 * context's table, used when an integration grows n (App. A.1,
 * generatingvectors).  Requires gcd(z_j, n) = 1 and 2 <= n < 2^53.
 * Re-registering n replaces its vector.
 */
int qmc_register_lattice(qmc_context* ctx, uint64_t n, uint32_t dim, const uint64_t* z);

/*
 * Smallest registered n >= preferred_n whose vector has >= dim components
 * (App. A.2, get_next_n); the largest such n if none is >= preferred_n.
 * QMC_ENOTFOUND if no registered vector has dim components.
 */
int qmc_next_lattice(qmc_context* ctx, uint64_t preferred_n, uint32_t dim, uint64_t* n_out);

/*
 * Fast component-by-component construction of a generating vector on the
 * device (Sec. 2.2; App. A.3): prime n in [3, 2^33 + 1], z[0] = 1, each next
 * component minimising the shift-averaged worst-case error of the Korobov
 * space with kernel omega(x) = 2 pi^2 (x^2 - x + 1/6) and product weights
 * gammas (host [dim], > 0; NULL = gamma_j = j^-2).  Candidates are
 * 1..(n-1)/2; among those within a relative 1e-9 of the minimum the smallest
 * wins.  The sums over all candidates are a cyclic convolution of length n-1
 * (Nuyens and Cools).  For n < 2^31 it is done with power-of-two FFTs of
 * length N = 2^ceil(log2(2n-3)): device memory 48 N + 16 n bytes (13 GB at
 * n = 1e8).  For n >= 2^31, n - 1 must be 2^a 3^b 5^c 7^d (the paper's
 * largest lattice, 15173222401, is of this form): the convolution runs
 * without padding through real-packed mixed-radix FFTs of length (n-1)/2,
 * device memory 32 (n - 1) bytes (70 GB at n = 2.2e9; the 15173222401-point
 * lattice would need 486 GB, more than one GPU holds).  Memory is allocated
 * for the call and freed before it returns.  z: host [dim].  QMC_EINVAL for
 * a composite or out-of-range n or an n >= 2^31 of another form, QMC_ENOMEM
 * when the buffers do not fit.  The result can be registered with
 * qmc_register_lattice.
 */
int qmc_cbc(qmc_context* ctx, uint64_t n, uint32_t dim, const double* gammas, uint64_t* z);

/*
 * max_n > 0: when the growth loop of qmc_integrate / qmc_integrate_request /
 * qmc_integrate_batch wants a lattice of want <= max_n points and none is
 * registered, it builds the lattice of the smallest prime >= want with
 * qmc_cbc (max(dim, 10) components, gamma_j = j^-2) and registers it, instead
 * of falling back to the largest registered lattice.  0 (the default) turns
 * this off.  max_n < 2^31.  The serving loop never builds lattices.
 */
int qmc_set_lattice_builder(qmc_context* ctx, uint64_t max_n);

/* ---------------------------------------------------------------- integrand */
typedef struct qmc_integrand qmc_integrand;

enum {
  QMC_DEFORM = 1u,     /* complex result: contour deformation with parameter lambda */
  QMC_EVAL_FP32 = 2u,  /* evaluate U, F and the powers in fp32, accumulate in fp64 */
  QMC_SPECIALISE = 4u  /* batches and serving: run the fp64 jobs of this integrand (real or deformed) in a kernel generated
                          for its structure (compiled at first use, a few seconds; shared by integrands of the
                          same structure) instead of the table-driven kernels.  The per-shift sums of a job
                          then come from that kernel, still the same alone or in any batch.  Single
                          integrations ignore the flag: they compile an integrand's specialised kernel
                          for a job of at least 2^24 evaluations, and once it is compiled it runs every
                          later single job of that integrand handle, whatever its size. */
};

/*
 * f(x) = prefactor * U(x)^pow_u * F(x)^pow_f, U and F sums of monomials
 * coef_i * prod_j x_j^expo[i*dim + j].  Monomials 0..n_u-1 form U, the next
 * n_f form F; n_f = 0 means F == 1.  With QMC_DEFORM every x_j is replaced
 * by z_j = x_j - i*lambda*x_j*(1-x_j)*dF/dx_j and the determinant of dz/dx
 * multiplies f; powers take the principal branch with arg = -pi on the
 * negative real axis.  Without QMC_DEFORM a negative base with a
 * non-integer power gives NaN, which is reported, never dropped.
 */
typedef struct {
  uint32_t dim;          /* 1..QMC_MAX_DIM */
  uint32_t n_u, n_f;     /* n_u >= 1, n_u + n_f <= QMC_MAX_MONOMIALS */
  const double* coef;    /* host [n_u + n_f], finite */
  const uint8_t* expo;   /* host [(n_u + n_f) * dim], row-major, each <= QMC_MAX_EXP */
  double pow_u, pow_f, prefactor; /* finite */
  uint32_t flags;        /* QMC_DEFORM | QMC_EVAL_FP32 | QMC_SPECIALISE */
  double lambda;         /* deformation parameter, used iff QMC_DEFORM */
} qmc_integrand_desc;

/* Copy a descriptor to the device (one host-to-device copy). */
int qmc_create_integrand(qmc_context* ctx, const qmc_integrand_desc* desc, qmc_integrand** out);

/*
 * One of the six Genz test functions the paper benchmarks (Sec. 5.3):
 * family 1 oscillatory cos(2 pi w_1 + sum c_i x_i), 2 product peak
 * prod (c_i^-2 + (x_i - w_i)^2)^-1, 3 corner peak (1 + sum c_i x_i)^-(d+1),
 * 4 Gaussian exp(-sum c_i^2 (x_i - w_i)^2), 5 continuous
 * exp(-sum c_i |x_i - w_i|), 6 discontinuous (0 if x_1 > w_1 or x_2 > w_2,
 * else exp(sum c_i x_i)).  c: host [dim], finite, > 0; w: host [dim] in
 * [0, 1]; both copied.  The handle works with qmc_integrate and qmc_set_vr;
 * the batch and serving calls and qmc_histogram return QMC_EUNSUPPORTED.
 */
int qmc_create_genz(qmc_context* ctx, int family, uint32_t dim, const double* c, const double* w,
                    qmc_integrand** out);

/* Free an integrand made by qmc_create_integrand or qmc_create_genz;
 * QMC_EBUSY while a pending request references it. */
int qmc_destroy_integrand(qmc_integrand* f);

/*
 * Set the variance-reduction map (Sec. 2.4, eq. ISfit in the PolySingular
 * form of App. A.5): params[6*j + 0..5] = (p0..p5) for dimension j, with
 * p0 >= 1.001 and p1 <= -0.001.  NULL switches the map off.
 */
int qmc_set_vr(qmc_integrand* f, const double* params);

/*
 * Histograms for the variance-reduction fit (Sec. 2.4): over the lattice
 * (n, z) shifted by the first shift of SplitMix64(seed), with no transform
 * and no VR map, hist[j*bins + b] = sum of |f(x)| over points with
 * floor(x_j * bins) = b (|f| = modulus for complex integrands; non-finite
 * values count 0).  Each |f| is rounded to an integer multiple of 2^-s,
 * with s the largest integer such that n * max|f| * 2^s <= 2^127, and the
 * multiples are summed exactly as 128-bit integers: the result is bitwise
 * reproducible, no bin can overflow, every |f| >= n * max|f| * 2^-74 keeps
 * full double precision, and each bin is that exact sum rounded once to a
 * double.  hist: host [dim * bins].  2 <= bins <= 65536; device scratch 16 * dim *
 * bins bytes.
 */
int qmc_histogram(qmc_context* ctx, const qmc_integrand* f, uint64_t n, const uint64_t* z, uint64_t seed,
                  uint32_t bins, double* hist);

/*
 * Fit the PolySingular map of eq. ISfit (App. A.5) to the inverse CDF of
 * each dimension's histogram by Levenberg-Marquardt under the paper's
 * bounds (host only, no GPU; App. A.1's default stopping rule: 40
 * iterations, step tolerance 3e-3): params[6*j + 0..5] receives (p0..p5)
 * with p0 >= 1.001, p1 <= -0.001, p2 >= 0, p3 >= 0.  A
 * dimension whose fit is not strictly increasing on [0,1] gets the identity
 * map and its bit in *fallback_mask (optional).  hist: host [dim * bins].
 */
int qmc_fit_vr_from_histogram(uint32_t dim, uint32_t bins, const double* hist, double* params,
                              uint32_t* fallback_mask);

/* qmc_histogram + qmc_fit_vr_from_histogram + qmc_set_vr on f.  params
 * (optional) receives the fitted [dim*6]. */
int qmc_fit_vr(qmc_context* ctx, qmc_integrand* f, uint64_t n, const uint64_t* z, uint64_t seed, uint32_t bins,
               double* params, uint32_t* fallback_mask);

/* ---------------------------------------------------------------- transforms */
enum { QMC_T_NONE = 0, QMC_T_KOROBOV = 1, QMC_T_BAKER = 2, QMC_T_SIDI = 3 };

/* Korobov<r0,r1> (eq. korobov, 0 <= r0, r1 <= 12), baker (eq. baker), none,
 * Sidi<r> (eq. sidi, weight proportional to sin(pi u)^r, 1 <= r = r0 <= 25;
 * r1 is ignored). */
typedef struct {
  int32_t kind;
  int32_t r0, r1;
} qmc_transform;

/* ---------------------------------------------------------------- results */
enum {
  QMC_CONVERGED = 1u,   /* error goal met */
  QMC_MAXEVAL_HIT = 2u, /* stopped by max_evals or the end of the lattice table */
  QMC_NONFINITE = 4u,   /* some contributions were not finite */
  QMC_VR_FALLBACK = 8u, /* a fitted VR map was rejected; identity used */
  QMC_DEFORM_SIGN = 16u /* some points had Im F(z) > 0 (reported only) */
};

enum { QMC_ERRMODE_ALL = 0, QMC_ERRMODE_LARGEST = 1 };

/* Mirrors the paper's result struct (App. A.2): integral, error, n, m,
 * iterations, evaluations; plus status flags and timings. */
typedef struct {
  double re, im;          /* estimate; im = 0 for real integrands */
  double err_re, err_im;  /* sqrt of eq. lattice-error per component; +inf if m = 1 */
  uint64_t n;             /* lattice size of the returned (last) iteration */
  uint32_t m;             /* shifts of the last lattice (more than requested after the
                             Monte Carlo fallback) */
  uint32_t iterations;    /* lattices evaluated (earlier ones discarded) */
  uint64_t evaluations;   /* total integrand evaluations over all iterations */
  uint32_t flags;         /* QMC_CONVERGED | ... */
  uint32_t path;          /* kernels used: 0 = descriptor-interpreting grid, 1 = specialised to this
                             integrand, 2 = persistent batch kernels */
  uint64_t nonfinite;     /* contributions that were NaN or +-inf (last iteration) */
  double device_seconds;  /* summed duration of the evaluation kernels (HIP events) */
  double queue_seconds;   /* submit-to-start wait (serving); 0 otherwise */
  double wall_seconds;    /* host wall time of the request */
  double fp32_err_re, fp32_err_im; /* QMC_EVAL_FP32 results: the fp32 evaluation's error in re, im,
                             estimated on a sample of the last lattice (every 32nd tile of the
                             batch tiling: all points when it has one tile) that is evaluated in
                             fp64 as well: |sum (w f_fp32 - w f_fp64)| / |sum w f_fp64| over the
                             sample and all shifts (complex modulus), times |estimate|; 0 for
                             fp64 evaluation */
} qmc_result;

/*
 * One integration.  dim must equal the integrand's dim; gcd(z_j, n) = 1;
 * 2 <= n < 2^53; 1 <= m <= QMC_MAX_SHIFTS.  Shifts are drawn from
 * SplitMix64(seed) (see qmc_shifts).
 * rel_tol <= 0: exactly this lattice (the paper's "Case 2", Sec. 3.3.2).
 * rel_tol > 0:  grow n through the registered table until the error goal
 *               (errormode "largest" for complex results) is met, as in the
 *               paper's "Case 1" (Sec. 3.3.1); only the last lattice counts.
 *               When the goal needs a lattice larger than the table holds,
 *               the largest one is used and, once there, shifts are added
 *               (m -> max(m+1, ceil(m (err/goal)^2)), at most QMC_MAX_SHIFTS;
 *               Monte Carlo scaling); the added shifts continue the same
 *               SplitMix64 stream, so earlier shifts' sums are kept.
 * shift_sums: optional host [m] (real) or [2m] (complex: re[0..m) then
 * im[0..m)) receiving the raw per-shift sums sum_k w f of the last lattice
 * for the first m (requested) shifts.
 */
int qmc_integrate(qmc_context* ctx, const qmc_integrand* f, uint32_t dim, uint64_t n,
                  const uint64_t* z, uint32_t m, uint64_t seed, qmc_transform t, double rel_tol,
                  qmc_result* out, double* shift_sums);

/* Full request: the paper's epsrel/epsabs/maxeval/errormode (App. A.1). */
typedef struct {
  const qmc_integrand* f;
  uint64_t n;            /* first lattice size (minn, rounded up through the table if z == NULL) */
  const uint64_t* z;     /* host [dim] generating vector for n, or NULL = from the table */
  uint32_t m;            /* shifts (minm) */
  uint32_t errormode;    /* QMC_ERRMODE_ALL or QMC_ERRMODE_LARGEST (complex only) */
  uint64_t seed;
  qmc_transform t;
  double rel_tol, abs_tol; /* both <= 0: one lattice only */
  uint64_t max_evals;      /* 0 = unlimited */
} qmc_request;

/*
 * One request with all of its options (rel_tol, abs_tol, max_evals,
 * errormode) through the single-integral kernels, the loop of qmc_integrate.
 */
int qmc_integrate_request(qmc_context* ctx, const qmc_request* req, qmc_result* out, double* shift_sums);

/*
 * Run `count` requests together; results in out[count].  Each round, the
 * current lattice of every unfinished request is evaluated by persistent
 * kernels (one per dimension class / real-complex / fp64-fp32 variant) that
 * drain a shared tile list, replayed as one HIP graph; requests that miss
 * their goal move to the next registered lattice for the next round
 * (Sec. 3.3.1), with the same Monte Carlo fallback as qmc_integrate.  A
 * request's tiling depends only on its own n and m, so its
 * per-shift sums are bitwise the same alone or in any batch.  QMC_EVAL_FP32
 * integrands run here (U, F and powers in fp32, compensated fp64 sums).
 * shift_sums (optional) gets each request's per-shift sums of its last
 * lattice for its requested m shifts, back to back ([m] or [2m] each).
 * device_seconds is the batch's total evaluation-kernel time, summed over its
 * rounds (HIP events around each round's evaluation kernels; the row
 * reduction after them is not included, as for a single lattice).
 */
int qmc_integrate_batch(qmc_context* ctx, const qmc_request* reqs, uint32_t count,
                        qmc_result* out, double* shift_sums);

/*
 * Autotune the batch kernels on a sample of requests: for every kernel variant
 * (dimension class; Korobov r=3, baker or any other transform / VR map;
 * real/complex; fp64/fp32) present in the sample, time each
 * compiled points-per-decode variant, shifts-per-thread group (8, 4 or 2 for
 * real kernels; complex kernels hold one shift per thread) and candidate tile
 * size on one round and keep the fastest for this context (and append it to
 * the file named by the environment variable QMC_TUNE_CACHE, read at context
 * creation, one line "gfx950 <largest dimension of the class> <transform
 * class> <complex> <fp32> <points-per-decode index> <tile points> <shifts per
 * group, 0 = 8>").  The points-per-decode and group choices never change
 * results; the tile size fixes the summation order, so tune before
 * integrating, not between calls whose sums must match bitwise.  Requests whose real fp64 jobs run in a specialised
 * kernel (QMC_SPECIALISE) are left out.  *configs_tried (optional) counts
 * timed schedules.
 */
int qmc_autotune_batch(qmc_context* ctx, const qmc_request* reqs, uint32_t count, uint32_t* configs_tried);

/* ---------------------------------------------------------------- serving */

/*
 * Continuous batching.  qmc_submit queues `count` requests as one ticket and
 * returns at once (arrays are copied).  A scheduler thread of the context
 * admits tickets in arrival order while their device memory (estimated at the
 * largest lattice they may reach) fits the budget (QMC_SERVE_MEM, default
 * 8 GiB), and runs rounds of the batch kernels over every admitted request's
 * current lattice; each request applies its own goal and growth rule
 * (Sec. 3.3.1) between rounds, so requests arriving while others run join the
 * next round.  Rounds are bounded: each unfinished request gets about an equal
 * share of a round's cost budget (QMC_SERVE_ROUND_COST, default 2^39 units of
 * evaluations weighted by integrand size, about a tenth of a second of the
 * device), its whole current lattice when that fits, else the next slice of
 * the lattice's tiles, whose partial sums stay on the device until the
 * lattice is done; sliced or not, a lattice's per-shift sums are the same.  A request's memory is reserved for the largest lattice it may
 * reach and the smallest tiles any schedule may give it, and returns to the
 * budget when that request finishes.  With a caller-owned workspace the
 * budget is also capped by the workspace size.  Results equal
 * qmc_integrate_batch's for the same request, except that a served request
 * never adds shifts at the largest lattice (the Monte Carlo fallback of
 * qmc_integrate_batch): it stops there with QMC_MAXEVAL_HIT, so its memory
 * stays within its reservation.  QMC_ENOMEM if the ticket alone exceeds the
 * budget.  Integrands of a
 * pending ticket cannot be destroyed (QMC_EBUSY).  result.queue_seconds is
 * submit-to-admission, result.wall_seconds submit-to-completion.
 */
int qmc_submit(qmc_context* ctx, const qmc_request* reqs, uint32_t count, uint64_t* ticket);

/* QMC_OK and the ticket's results in out[count] (the ticket is then
 * released), QMC_PENDING, QMC_ECANCELED, QMC_EDEVICE, or QMC_ENOTFOUND. */
int qmc_poll(qmc_context* ctx, uint64_t ticket, qmc_result* out);

/* As qmc_poll, blocking up to timeout_s seconds (< 0: no limit). */
int qmc_wait(qmc_context* ctx, uint64_t ticket, double timeout_s, qmc_result* out);

/* Cancel a ticket: removed before admission or at the next round boundary. */
int qmc_cancel(qmc_context* ctx, uint64_t ticket);

/* Scheduler counters: rounds run, tickets queued and active, bytes admitted. */
int qmc_serve_stats(qmc_context* ctx, uint64_t* rounds, uint64_t* queued, uint64_t* active,
                    uint64_t* bytes_in_use);

/* ---------------------------------------------------------------- no allocation */

/* Bytes of the static device scratch of qmc_integrate_noalloc (one copy per device). */
#define QMC_NOALLOC_SCRATCH_BYTES (4 << 20)

/*
 * For callers that cannot allocate device or pinned host memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * qmc_integrate with rel_tol <= 0 (one lattice, the paper's "Case 2") that
 * calls no hipMalloc, hipFree, hipHostMalloc or other allocating routine.
 * Its scratch (shift table, per-block partial sums, the sums) is a static
 * device array of QMC_NOALLOC_SCRATCH_BYTES per device, found when the
 * context is created; the shift table SplitMix64(seed) is generated on the
 * device.  Arguments, result and shift_sums ([m] or [2m], optional) as for
 * qmc_integrate; the sums are bitwise those of qmc_integrate for the same
 * call whenever both run the same kernel: the table-driven kernels, or an
 * integrand's specialised kernel when qmc_integrate has already compiled it
 * (none is compiled here).  Errors as qmc_integrate, plus QMC_ENOMEM when
 * the launch needs more scratch than the static array holds (large m with
 * many blocks) and QMC_EUNSUPPORTED for QMC_EVAL_FP32 integrands.  Every
 * call on one device shares that device's array: calls that overlap on one
 * device, from different contexts or threads, race and give wrong results;
 * calls on one context are serialised.  The array keeps the last call's
 * contents; nothing in it needs clearing between calls.
 */
int qmc_integrate_noalloc(qmc_context* ctx, const qmc_integrand* f, uint32_t dim, uint64_t n,
                          const uint64_t* z, uint32_t m, uint64_t seed, qmc_transform t,
                          qmc_result* out, double* shift_sums);

/* ---------------------------------------------------------------- debug / parity */

/* The shifts SplitMix64(seed) gives: out[s*dim + j], s < m, j < dim; each
 * value is (x >> 11) * 2^-53 of the next 64-bit output, shift-major. Host only. */
int qmc_shifts(uint64_t seed, uint32_t m, uint32_t dim, double* out);

/* Lattice indices (k z_j) mod n for k in [k0, k0+count), computed by the
 * device index path (start index, then strided increments): out[i*dim + j]. */
int qmc_lattice_indices(qmc_context* ctx, uint64_t n, uint32_t dim, const uint64_t* z, uint64_t k0,
                        uint64_t count, uint64_t* out);

/* Raw per-shift sums over points k in [k0, k1) (a parity unit for large n). */
int qmc_shift_sums_range(qmc_context* ctx, const qmc_integrand* f, uint64_t n, const uint64_t* z,
                         uint32_t m, uint64_t seed, qmc_transform t, uint64_t k0, uint64_t k1,
                         double* shift_sums, uint64_t* nonfinite);

/*
 * Generate and compile (hiprtc, gfx950) the evaluation kernel specialised to
 * descriptor d and transform t, without loading it; needs no GPU.  Large
 * integrations use such kernels automatically (qmc_result.path = 1).
 * code_bytes (optional) receives the code-object size.  QMC_EINVAL with the
 * compiler log in qmc_last_error() if generation or compilation fails.
 */
int qmc_specialize_check(const qmc_integrand_desc* d, qmc_transform t, size_t* code_bytes);

#ifdef __cplusplus
}
#endif

#endif /* QMC_H */
