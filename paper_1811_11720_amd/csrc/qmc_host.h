// qmc_host.h -- host-side state shared by the runtime, batch executor and scheduler.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "qmc.h"
#include "qmc_internal.h"
#include "qmc_jit.h"

struct qmc_serve_state;  // qmc_serve.cpp

struct qmc_context {
  int device = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  // scratch: caller workspace or library-owned
  char* ws = nullptr;
  size_t ws_bytes = 0;
  bool own_ws = false;
  // pinned host staging
  double* h_stage = nullptr;
  size_t h_stage_bytes = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  std::map<uint64_t, std::vector<uint64_t>> lattices;  // guarded by lat_mu
  std::mutex lat_mu;                                  // innermost lock
  std::recursive_mutex mu;                            // taken through CtxLock
  std::atomic<int> lock_waiters{0};                   // threads waiting in CtxLock
  int inflight = 0;
  int live_integrands = 0;  // the context is freed only after its last integrand
  std::atomic<bool> closing{false};  // destroy requested while integrands were alive
  std::atomic<bool> broken{false};
  std::mutex serve_init;              // creation of the serving scheduler
  int max_blocks = 0;          // 0: from occupancy
  int cus = 256;               // compute units of the device
  int grid_rounds = 1;         // resident-block rounds per launch
  bool jit = true;             // specialise kernels to the integrand
  uint64_t jit_min_evals = 1ull << 24;
  int jit_S = 8;
  // batch executor
  uint64_t batch_tile_real = 4096;    // minimum points per tile (real integrands)
  uint64_t batch_tile_complex = 4096;  // ... (complex integrands)
  uint64_t batch_max_ktiles = 2048;   // tiles along k per integral at most
  bool batch_graph = true;            // replay each round's launches as a HIP graph
  // per kernel variant [dimension class][complex][fp32]: tuned schedule (0 = default)
  int batch_sv[qmck::BATCH_VARIANTS] = {};         // index into the compiled points-per-decode variants
  uint64_t batch_tile[qmck::BATCH_VARIANTS] = {};  // minimum points per tile (0 = the default)
  uint32_t batch_group[qmck::BATCH_VARIANTS] = {};  // shifts per thread group (0 = the kernel's S)
  std::string tune_cache;             // file the autotuner reads and appends
  hipStream_t cap_stream = nullptr;   // private stream used only for graph capture
  // instantiated graphs of recent batch rounds, keyed by every launch argument
  struct CachedGraph {
    std::vector<uint64_t> sig;
    hipGraphExec_t exec;
    uint64_t last_use;
  };
  static constexpr size_t kGraphCache = 16;
  std::vector<CachedGraph> graphs;
  uint64_t graph_tick = 0;
  // serving
  std::atomic<qmc_serve_state*> serve{nullptr};     // scheduler, created by the first qmc_submit
  size_t serve_mem_limit = (size_t)8 << 30;  // device bytes admitted requests may use
  uint64_t serve_max_n = (1ull << 31) - 1;   // growth stops above this lattice size
  double serve_round_cost = 0x1p39;          // cost units (evaluations x per-evaluation weight) per serving round
  uint64_t build_max_n = 0;  // > 0: the growth loop builds missing lattices up to this size (qmc_cbc)
};

// The context lock for API calls.  The serving scheduler takes the lock for
// every round and lets the threads counted here in before its next round, so
// calls made while requests are being served wait for at most one round.
struct CtxLock {
  qmc_context* c;
  explicit CtxLock(qmc_context* ctx) : c(ctx) {
    c->lock_waiters.fetch_add(1, std::memory_order_acq_rel);
    c->mu.lock();
    c->lock_waiters.fetch_sub(1, std::memory_order_acq_rel);
  }
  ~CtxLock() { c->mu.unlock(); }
  CtxLock(const CtxLock&) = delete;
  CtxLock& operator=(const CtxLock&) = delete;
};

struct qmc_integrand {
  qmc_context* ctx = nullptr;
  uint32_t dim = 0, n_u = 0, n_f = 0, flags = 0;
  int genz = 0;  // 1..6: a Genz test family (coef = [c | w]), no monomial table
  double pow_u = 1, pow_f = 1, prefactor = 1, lambda = 0;
  int pu_mode = 0, pu_k = 0, pf_mode = 0, pf_k = 0;
  std::vector<double> coef;
  std::vector<uint8_t> expo;
  bool has_vr = false;
  uint32_t vr_fallback = 0;  // dimensions whose fitted map was rejected (identity used)
  std::vector<double> vr;
  char* dmem = nullptr;  // coef | expo (u32 x 2 per monomial) | vr
  double* d_coef = nullptr;
  uint32_t* d_expo = nullptr;
  double* d_vr = nullptr;
  float* d_coef32 = nullptr;
  std::atomic<int> refs{0};  // pending serving requests that use this integrand
  std::map<int, qmcj::Kernel> jit;  // per (transform kind, VR on) key
  std::map<int, int> jit_failed;
};


namespace qmch {

// error reporting (thread-local message, returns code)
int fail(int code, const char* fmt, ...);
void make_shifts(uint64_t seed, uint32_t m, uint32_t dim, double* out);
uint64_t mulmod(uint64_t a, uint64_t b, uint64_t n);
int check_lattice(uint64_t n, uint32_t dim, const uint64_t* z);
int set_transform(qmcd::EvalArgs& a, const qmc_transform& t, int& tsel);
int scratch(qmc_context* c, size_t need, char** out);
int stage(qmc_context* c, size_t bytes);
void estimate(const double* q, uint32_t m, double& mean, double& err);
bool goal_met(const qmc_result& r, double rel, double abs_, uint32_t mode, bool cplx);
// Smallest registered lattice with n >= want (or the largest, if allow_smaller)
// and at least dim components; copies its first dim components into *z_out.
// Takes the table's own lock, so callers need not hold the context lock.
int next_registered(qmc_context* c, uint64_t want, uint32_t dim, uint64_t* n_out, bool allow_smaller,
                    std::vector<uint64_t>* z_out = nullptr);
uint64_t largest_registered(qmc_context* c);

// Next step of the Case-1 loop (Sec. 3.3.1) after a round that missed its goal:
// the next registered lattice of at least max(1.5 n, n err/goal) points (the
// round is discarded); when the table has none, its largest lattice; once
// there, more shifts, m -> max(m+1, ceil(m (err/goal)^2)) up to QMC_MAX_SHIFTS,
// continuing the same shift stream so the earlier shifts' sums are kept (at
// most max_m shifts).  No step may take the evaluations past q.max_evals
// (0 = no limit): a lattice too large for the remaining budget is replaced by
// the largest larger-than-current one that fits.  Lattices larger than max_n
// are not used.
struct GrowthStep {
  enum Kind { STOP = 0, LATTICE = 1, SHIFTS = 2 } kind = STOP;
  uint64_t n = 0;
  uint32_t m = 0;                // shift count after the step
  std::vector<uint64_t> z;       // LATTICE: generating vector [dim]
};
GrowthStep growth_step(qmc_context* c, const qmc_request& q, const qmc_result& r, uint64_t n, uint32_t m,
                       uint32_t dim, bool cplx, uint64_t max_n, uint32_t max_m, bool may_build = false);
// Builds (qmc_cbc) and registers the lattice of the smallest prime >= want
// with max(dim, 10) components; returns its size (0 on failure).
uint64_t build_lattice(qmc_context* c, uint64_t want, uint32_t dim);
// The integrand's specialised kernels for transform selector tsel (compiled
// on first use, shared by integrands of the same structure); 0 on success.
int specialised_kernel(qmc_context* c, qmc_integrand* f, int tsel, qmcj::Kernel* out);
// fill the integrand/transform part of an EvalArgs
int fill_integrand_args(qmcd::EvalArgs& a, const qmc_integrand* f, const qmc_transform& t, int& tsel);

// Launch plan of one lattice on the single-integral kernels (plan_lattice),
// then enqueued on the context stream with its scratch (launch_lattice).
struct LatticePlan {
  qmcd::EvalArgs a;
  qmcj::Kernel jk;
  bool use_jit = false, cplx = false, idx32 = true;
  int tsel = 0, dclass = 0;
  uint32_t nb = 0, groups = 0, rows = 0;
  size_t off_sh = 0, sz_sh = 0, off_part = 0, off_out = 0, sz_out = 0, bytes = 0;
};
int plan_lattice(qmc_context* c, qmc_integrand* f, uint64_t n, const uint64_t* z, uint32_t m, const qmc_transform& t,
                 uint64_t k0, uint64_t k1, bool may_compile, LatticePlan& p);
int launch_lattice(qmc_context* c, const qmc_integrand* f, LatticePlan& p, char* ws);
// Finds the current device's copy of the static scratch of qmc_integrate_noalloc.
int noalloc_init(int device);

// one integral's current lattice in a batch round
struct BatchJob {
  qmc_integrand* f = nullptr;
  uint64_t n = 0;
  const uint64_t* z = nullptr;   // [dim]
  uint32_t m = 0;
  const double* shifts = nullptr;  // [m][dim]
  qmc_transform t{};
  // in: evaluate only the tiles [tile_first, tile_first + tile_count) of the
  // job's tiling (tile_count 0: all of them) into ext_partial (rows x ktiles
  // doubles of device memory the caller keeps across calls; nullptr: batch
  // scratch); the sums are produced only with `finish` set, by the call that
  // evaluates the last of the tiles (calls run in order on one stream)
  uint32_t tile_first = 0, tile_count = 0;
  double* ext_partial = nullptr;
  bool finish = true;
  std::vector<double> sums;  // out: rows (m or 2m), when finished
  // where the rows are: sums.data(), or a range of the rows of the job it was
  // merged into (replicas of one lattice), kept alive by sums_keep
  const double* sums_at = nullptr;
  std::shared_ptr<const std::vector<double>> sums_keep;
  uint64_t sign_points = 0;  // out: points of this call's tiles with Im F(z) > 0
  // out, QMC_EVAL_FP32 jobs: per row, over a sample of the lattice's points
  // (every kFp32SampleEvery-th tile), the sum of the fp32-evaluated
  // contributions minus the fp64-evaluated ones, the sum of the fp64-evaluated
  // ones, and the sample's size
  std::vector<double> fp32_dev, fp32_ref;
  uint64_t fp32_dev_points = 0;
};
// Tiles of an fp32 job that are also evaluated in fp64 to estimate the fp32
// error: tiles 0, 32, 64, ... of its ktiles tiles, ceil(ktiles / 32) of them.
constexpr uint32_t kFp32SampleEvery = 32;
inline uint32_t batch_fp32_sample_tiles(uint32_t ktiles) { return (ktiles + kFp32SampleEvery - 1) / kFp32SampleEvery; }
// Tiling of a batch job as run_batch lays it out: kernel variant (or the
// integrand's specialised batch kernel), points per tile, tiles along k,
// shift groups (tiles in all: ktiles x groups) and rows (m or 2m).
struct BatchShape {
  qmck::BatchVariant var;
  bool use_jit = false;
  qmcj::Kernel jk;
  uint64_t tile_points = 0;
  uint32_t ktiles = 0, groups = 0, rows = 0;
  uint32_t group_size = 0;  // shifts per thread group
};
int batch_job_shape(qmc_context* c, const BatchJob& b, BatchShape& sh);
// Points per tile of a batch job of n points: the variant's tuned minimum
// (0 = the default for real or complex jobs), at least n / batch_max_ktiles,
// rounded up to whole blocks.  A job's tiling depends only on this.
uint64_t batch_tile_points(const qmc_context* c, uint64_t tuned, bool cplx, uint64_t n);
// Most tiles any schedule can give a job of n points.
uint64_t batch_ktiles_bound(const qmc_context* c, uint64_t n);
// Upper bound of the batch scratch one job of `rows` rows and `ktiles` tiles takes.
size_t batch_job_bytes(size_t rows, uint64_t ktiles, uint32_t m, uint32_t dim, bool fp32);
// fp32_err_re/im of a result (its estimate already set) from the per-shift
// sampled sums of fp32 - fp64 contributions (dre, dim) and of fp64
// contributions (rre, rim) over `points` points.
void fp32_error(const double* dre, const double* dim, const double* rre, const double* rim, uint32_t m,
                uint64_t points, qmc_result& r);
// Evaluate all jobs with the persistent batch kernels (one round).
int run_batch(qmc_context* c, std::vector<BatchJob*>& jobs, double* kernel_seconds);
// Requests through rounds of run_batch (growth loop per request).
int run_requests(qmc_context* c, const qmc_request* reqs, uint32_t count, qmc_result* out, double* shift_sums);
// serving scheduler (qmc_serve.cpp)
void serve_shutdown(qmc_context* c);
int serve_inflight(qmc_context* c);
void free_context(qmc_context* c);
void load_tune_cache(qmc_context* c);
void batch_schedule_defaults(qmc_context* c);

}  // namespace qmch

#define HIPCHK(call)                                                                                  \
  do {                                                                                                \
    hipError_t e_ = (call);                                                                           \
    if (e_ != hipSuccess) return qmch::fail(QMC_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
  } while (0)
