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
#include <string>
#include <unordered_map>

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
  const uint64_t t0 = std::max<uint64_t>(tmin, (n + c->batch_max_ktiles - 1) / c->batch_max_ktiles);
  // as many tiles as tiles of t0 points need, made even (a short last tile
  // would leave its workgroup idle for most of a tile's time)
  const uint64_t kt = std::max<uint64_t>(1, (n + t0 - 1) / t0);
  const uint64_t tp = (n + kt - 1) / kt;
  return (tp + QMCD_BLOCK - 1) / QMCD_BLOCK * QMCD_BLOCK;
}

uint64_t batch_ktiles_bound(const qmc_context* c, uint64_t n) {
  // every tile holds a whole number (>= 1) of blocks and at least n / batch_max_ktiles points
  const uint64_t tp = batch_tile_points(c, QMCD_BLOCK, false, n);
  return (n + tp - 1) / tp;
}

size_t batch_job_bytes(size_t rows, uint64_t ktiles, uint32_t m, uint32_t dim, bool fp32) {
  // arena entries of one job (run_batch's layout) plus its share of the alignment padding
  size_t b = sizeof(qmcd::EvalArgs) + 4 + 8 + rows * (sizeof(qmck::RowRef) + 8 * ktiles + 8) + (size_t)m * dim * 8 +
             8 + 256;
  if (fp32)  // the fp64 twin over the first tiles, and the rows of the job's own first columns
    b += sizeof(qmcd::EvalArgs) + 4 + 8 + 8 +
         rows * (2 * (sizeof(qmck::RowRef) + 8) + 8 * (size_t)batch_fp32_sample_tiles((uint32_t)ktiles));
  return b;
}

namespace {

int run_batch_jobs(qmc_context* c, std::vector<BatchJob*>& jobs, double* kernel_seconds);

// Key of the jobs that can share one item: the integrand, the lattice and the
// transform (the shifts are what differs); generating vectors compare by their
// components mod n.
struct MergeKey {
  const BatchJob* b;
};
struct MergeHash {
  size_t operator()(const MergeKey& k) const {
    const BatchJob& b = *k.b;
    uint64_t h = (uint64_t)(uintptr_t)b.f * 0x9e3779b97f4a7c15ULL ^ b.n;
    h = h * 0x100000001b3ULL ^ (uint64_t)(uint32_t)b.t.kind ^ ((uint64_t)(uint32_t)b.t.r0 << 20) ^
        ((uint64_t)(uint32_t)b.t.r1 << 40);
    for (uint32_t j = 0; j < b.f->dim; ++j) h = (h ^ (b.z[j] % b.n)) * 0x100000001b3ULL;
    return (size_t)h;
  }
};
struct MergeEq {
  bool operator()(const MergeKey& x, const MergeKey& y) const {
    const BatchJob &a = *x.b, &b = *y.b;
    if (a.f != b.f || a.n != b.n || a.t.kind != b.t.kind || a.t.r0 != b.t.r0 || a.t.r1 != b.t.r1) return false;
    if (a.z == b.z) return true;
    for (uint32_t j = 0; j < a.f->dim; ++j)
      if (a.z[j] % a.n != b.z[j] % b.n) return false;
    return true;
  }
};

}  // namespace

int batch_job_shape(qmc_context* c, const BatchJob& b, BatchShape& sh) {
  const qmc_integrand* f = b.f;
  const bool cplx = (f->flags & QMC_DEFORM) != 0, fp32 = (f->flags & QMC_EVAL_FP32) != 0;
  qmcd::EvalArgs probe;
  int tsel = 0;
  int rc = set_transform(probe, b.t, tsel);
  if (rc) return rc;
  sh.var = qmck::BatchVariant{qmck::dim_class(f->dim, cplx), qmck::batch_tkc(tsel, f->has_vr), cplx, fp32};
  sh.use_jit = false;
  if (!fp32 && (f->flags & QMC_SPECIALISE) && c->jit &&
      specialised_kernel(c, const_cast<qmc_integrand*>(b.f), tsel, &sh.jk) == 0 && sh.jk.batch)
    sh.use_jit = true;
  const uint32_t S = cplx ? qmck::S_COMPLEX : qmck::S_REAL;
  const uint32_t tuned = sh.use_jit ? 0u : c->batch_group[sh.var.index()];
  sh.group_size = (tuned && tuned < S) ? tuned : S;
  sh.tile_points = batch_tile_points(c, sh.use_jit ? 0 : c->batch_tile[sh.var.index()], cplx, b.n);
  sh.ktiles = (uint32_t)((b.n + sh.tile_points - 1) / sh.tile_points);
  sh.groups = (b.m + sh.group_size - 1) / sh.group_size;
  sh.rows = cplx ? 2 * b.m : b.m;
  return QMC_OK;
}

// Real jobs of one integrand on one lattice with one transform (replicas
// with different shift seeds, or the requests of a served ticket that share a
// sector) run as one item whose shift table is the concatenation of theirs.
// A shift's sum depends only on the lattice, the tiling (a function of n and
// the kernel variant) and the shift itself, never on which shifts share its
// thread group, so every job's sums are bitwise those it gets alone; merged,
// the thread groups of S shifts are full instead of each job's last one
// being partly empty, and the item list is shorter.  Complex jobs are not
// merged: their count of points with Im F(z) > 0 is kept per job.
int run_batch(qmc_context* c, std::vector<BatchJob*>& jobs, double* kernel_seconds) {
  const uint32_t J = (uint32_t)jobs.size();
  if (kernel_seconds) *kernel_seconds = 0.0;
  if (J < 2) return run_batch_jobs(c, jobs, kernel_seconds);
  std::unordered_map<MergeKey, uint32_t, MergeHash, MergeEq> slot;  // key -> index into members
  std::vector<std::vector<uint32_t>> members;
  std::vector<BatchJob*> work;
  std::vector<uint32_t> owner(J, UINT32_MAX);
  for (uint32_t i = 0; i < J; ++i) {
    const BatchJob& b = *jobs[i];
    if ((b.f->flags & QMC_DEFORM) || b.ext_partial || b.tile_count) continue;
    auto ins = slot.emplace(MergeKey{&b}, (uint32_t)members.size());
    if (ins.second) members.emplace_back();
    members[ins.first->second].push_back(i);
  }
  bool any = false;
  for (const auto& g : members) any = any || g.size() > 1;
  if (!any) return run_batch_jobs(c, jobs, kernel_seconds);
  std::vector<BatchJob> merged;
  std::vector<std::vector<double>> tabs;
  merged.reserve(members.size());
  tabs.reserve(members.size());
  for (const auto& g : members) {
    if (g.size() == 1) continue;
    const BatchJob& first = *jobs[g.front()];
    const uint32_t dim = first.f->dim;
    BatchJob mj;
    mj.f = first.f;
    mj.n = first.n;
    mj.z = first.z;
    mj.t = first.t;
    std::vector<double> tab;
    for (uint32_t i : g) {
      tab.insert(tab.end(), jobs[i]->shifts, jobs[i]->shifts + (size_t)jobs[i]->m * dim);
      mj.m += jobs[i]->m;
      owner[i] = (uint32_t)merged.size();
    }
    tabs.push_back(std::move(tab));
    mj.shifts = tabs.back().data();
    merged.push_back(std::move(mj));
  }
  for (uint32_t i = 0; i < J; ++i)
    if (owner[i] == UINT32_MAX) work.push_back(jobs[i]);
  for (BatchJob& mj : merged) work.push_back(&mj);
  int rc = run_batch_jobs(c, work, kernel_seconds);
  if (rc) return rc;
  std::vector<uint32_t> at(merged.size(), 0);  // next shift of each merged job
  // the members read their rows in place from the merged job's (shared) rows
  std::vector<std::shared_ptr<const std::vector<double>>> rows_of(merged.size());
  for (size_t g = 0; g < merged.size(); ++g)
    rows_of[g] = std::make_shared<const std::vector<double>>(std::move(merged[g].sums));
  for (uint32_t i = 0; i < J; ++i) {
    if (owner[i] == UINT32_MAX) continue;
    const BatchJob& mj = merged[owner[i]];
    const uint32_t s0 = at[owner[i]];
    jobs[i]->sums.clear();
    jobs[i]->sums_keep = rows_of[owner[i]];
    jobs[i]->sums_at = rows_of[owner[i]]->data() + s0;
    jobs[i]->sign_points = 0;
    jobs[i]->fp32_dev.clear();
    jobs[i]->fp32_ref.clear();
    jobs[i]->fp32_dev_points = mj.fp32_dev_points;
    if (!mj.fp32_dev.empty()) {
      jobs[i]->fp32_dev.assign(mj.fp32_dev.begin() + s0, mj.fp32_dev.begin() + s0 + jobs[i]->m);
      jobs[i]->fp32_ref.assign(mj.fp32_ref.begin() + s0, mj.fp32_ref.begin() + s0 + jobs[i]->m);
    }
    at[owner[i]] = s0 + jobs[i]->m;
  }
  return QMC_OK;
}

namespace {

// Launch key of a table-driven job: its variant's index, made negative for a
// complex job with a general power (neither integer nor half-integer), which
// needs the kernels that hold the complex logarithm and exponential; the
// others run in the leaner integer-and-half-integer kernels.
int launch_key(const qmck::BatchVariant& v, const qmc_integrand* f) {
  const bool general = f->pu_mode == qmcd::PW_GEN || (f->n_f && f->pf_mode == qmcd::PW_GEN);
  return (v.cplx && general) ? -1 - v.index() : v.index();
}

int run_batch_jobs(qmc_context* c, std::vector<BatchJob*>& jobs, double* kernel_seconds) {
  const uint32_t J = (uint32_t)jobs.size();
  if (kernel_seconds) *kernel_seconds = 0.0;
  if (J == 0) return QMC_OK;
  struct Plan {
    qmck::BatchVariant var;
    int variant;  // launch key: launch_key(var, f), or past BATCH_VARIANTS for a specialised kernel
    uint32_t rows, ktiles, groups, group_size;
    uint64_t tile_points;
    size_t part_off, sh_off, row0;
    double cost;
    bool use_jit = false;  // the integrand's specialised batch kernel (QMC_SPECIALISE)
    qmcj::Kernel jk;
    uint32_t tiles = 0;    // tiles of the job this call evaluates
    bool finish = true;    // the job's sums are produced (all of its tiles are then evaluated)
    uint32_t job;          // the job evaluated (a twin evaluates its job's first columns in fp64)
    int twin = -1;         // fp32 job: index of its fp64 twin plan
    size_t pref_row0 = 0;  // fp32 job: rows summing its first twin-ktiles columns
  };
  std::vector<Plan> plan(J);
  std::vector<hipFunction_t> jit_fns;  // distinct specialised kernels in this call
  size_t n_part = 0, n_sh = 0, n_rows = 0;
  for (uint32_t i = 0; i < J; ++i) {
    BatchJob& b = *jobs[i];
    const qmc_integrand* f = b.f;
    Plan& p = plan[i];
    p.job = i;
    BatchShape sh;
    int trc = batch_job_shape(c, b, sh);
    if (trc) return trc;
    p.var = sh.var;
    p.variant = launch_key(p.var, f);
    if (sh.use_jit) {
      // jobs of one specialised kernel form a launch of their own
      p.use_jit = true;
      p.jk = sh.jk;
      auto it = std::find(jit_fns.begin(), jit_fns.end(), p.jk.batch);
      p.variant = qmck::BATCH_VARIANTS + (int)(it - jit_fns.begin());
      if (it == jit_fns.end()) jit_fns.push_back(p.jk.batch);
    }
    p.tile_points = sh.tile_points;
    p.ktiles = sh.ktiles;
    p.groups = sh.groups;
    p.group_size = sh.group_size;
    p.rows = sh.rows;
    const uint64_t all = (uint64_t)p.ktiles * p.groups;
    if (b.tile_count && (b.tile_first >= all || b.tile_count > all - b.tile_first))
      return fail(QMC_EINVAL, "tile range [%u, %u) outside the job's %llu tiles", b.tile_first,
                  b.tile_first + b.tile_count, (unsigned long long)all);
    p.tiles = b.tile_count ? b.tile_count : (uint32_t)all;
    p.finish = b.finish || !b.ext_partial;
    if (!b.ext_partial) {
      p.part_off = n_part;
      n_part += (size_t)p.rows * p.ktiles;
    }
    p.sh_off = n_sh;
    n_sh += (size_t)b.m * f->dim;
    if (p.finish) {
      p.row0 = n_rows;
      n_rows += p.rows;
    }
    p.cost = cost_per_eval(f) * (double)b.n * b.m * ((double)p.tiles / (double)all);
  }
  // FP32 jobs: an fp64 twin over every kFp32SampleEvery-th tile of the job
  // (same tiling, same shifts), and rows summing the fp32 job's own columns of
  // those tiles: their difference is the fp32 evaluation's error over that
  // strided sample of points
  for (uint32_t i = 0; i < J; ++i) {
    if (!(jobs[i]->f->flags & QMC_EVAL_FP32) || !plan[i].finish) continue;
    Plan t = plan[i];
    t.job = i;
    t.tiles = 0;
    t.var.fp32 = false;
    t.variant = launch_key(t.var, jobs[i]->f);
    t.use_jit = false;
    t.ktiles = batch_fp32_sample_tiles(plan[i].ktiles);
    t.tiles = t.ktiles * t.groups;
    t.part_off = n_part;
    n_part += (size_t)t.rows * t.ktiles;
    t.row0 = n_rows;
    n_rows += t.rows;
    t.cost = plan[i].cost * t.ktiles / plan[i].ktiles;
    plan[i].twin = (int)plan.size();
    plan[i].pref_row0 = n_rows;
    n_rows += plan[i].rows;
    plan.push_back(t);
  }
  const uint32_t JT = (uint32_t)plan.size();
  // variants present, items ordered heaviest first
  std::map<int, std::vector<uint32_t>> by_var;
  for (uint32_t i = 0; i < JT; ++i) by_var[plan[i].variant].push_back(i);
  for (auto& kv : by_var)
    std::stable_sort(kv.second.begin(), kv.second.end(), [&](uint32_t x, uint32_t y) { return plan[x].cost > plan[y].cost; });
  const uint32_t NV = (uint32_t)by_var.size();

  // device layout
  size_t off = 0;
  const size_t o_items = off;
  off = align256(off + (size_t)JT * sizeof(qmcd::EvalArgs));
  const size_t o_order = off;
  off = align256(off + (size_t)JT * 4);
  const size_t o_prefix = off;
  off = align256(off + (size_t)(JT + NV) * 4);
  const size_t o_rows = off;
  off = align256(off + n_rows * sizeof(qmck::RowRef));
  const size_t o_sh = off;
  off = align256(off + n_sh * 8);
  // the variants' tile counters and the jobs' sign counts start at zero: they
  // are part of the upload (zeros from the host), so a round needs no fill
  // kernel; the sign counts are followed directly by the row results, and one
  // copy returns both
  const size_t o_cnt = off;
  off = (off + (size_t)NV * 4 + 7) / 8 * 8;
  const size_t o_sign = off;
  off += (size_t)JT * 8;
  const size_t upload = off;  // everything above comes from the host
  const size_t o_out = off;
  off = align256(off + n_rows * 8);
  const size_t o_part = off;
  off = align256(off + n_part * 8);
  char* ws = nullptr;
  int rc = scratch(c, off, &ws);
  if (rc) return rc;
  rc = stage(c, std::max(upload, (size_t)JT * 8 + n_rows * 8));
  if (rc) return rc;
  char* h = (char*)c->h_stage;
  // zeros where the loop below writes only some fields (the argument table) and
  // for the counters and sign counts; every row reference and every shift is
  // written in full, so those (large) regions are not cleared first
  std::memset(h, 0, o_rows);
  std::memset(h + o_cnt, 0, upload - o_cnt);

  qmcd::EvalArgs* items = (qmcd::EvalArgs*)(h + o_items);
  qmck::RowRef* rows = (qmck::RowRef*)(h + o_rows);
  double* shifts = (double*)(h + o_sh);
  double* d_part = (double*)(ws + o_part);
  double* d_out = (double*)(ws + o_out);
  unsigned long long* d_sign = (unsigned long long*)(ws + o_sign);
  for (uint32_t i = 0; i < JT; ++i) {
    const Plan& p = plan[i];
    BatchJob& b = *jobs[p.job];
    qmcd::EvalArgs& a = items[i];
    if (i >= J) {  // fp64 twin: its job's arguments (already filled) on its own columns
      a = items[p.job];
      a.partial = d_part + p.part_off;
      a.nblocks = p.ktiles;
      a.ktiles = p.ktiles;
      a.tile_skip = kFp32SampleEvery - 1;
      a.tile_first = 0;
      a.sign_count = d_sign + i;
      a.item = i;
      const double* jp = jobs[p.job]->ext_partial ? jobs[p.job]->ext_partial : d_part + plan[p.job].part_off;
      for (uint32_t r = 0; r < p.rows; ++r) {
        rows[p.row0 + r].p = d_part + p.part_off + (size_t)r * p.ktiles;
        rows[p.row0 + r].ncols = p.ktiles;
        rows[p.row0 + r].skip = 0;
        rows[plan[p.job].pref_row0 + r].p = jp + (size_t)r * plan[p.job].ktiles;
        rows[plan[p.job].pref_row0 + r].ncols = p.ktiles;
        rows[plan[p.job].pref_row0 + r].skip = kFp32SampleEvery - 1;
      }
      continue;
    }
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
    double* part = b.ext_partial ? b.ext_partial : d_part + p.part_off;
    a.partial = part;
    a.nblocks = p.ktiles;
    a.sign_count = d_sign + i;
    a.tile_points = p.tile_points;
    a.ktiles = p.ktiles;
    a.tile_first = b.tile_count ? b.tile_first : 0;
    a.shift_group = p.group_size;
    a.item = i;
    std::memcpy(shifts + p.sh_off, b.shifts, (size_t)b.m * b.f->dim * 8);
    if (p.finish)  // a slice that does not finish its lattice owns no rows
      for (uint32_t r = 0; r < p.rows; ++r) {
        rows[p.row0 + r].p = part + (size_t)r * p.ktiles;
        rows[p.row0 + r].ncols = p.ktiles;
        rows[p.row0 + r].skip = 0;
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
      acc += plan[i].tiles;
    }
    if (acc >= 0xFFFFFFFFull) return fail(QMC_EINVAL, "batch has more than 2^32 tiles");
    prefix[ppos + L.count] = (uint32_t)acc;
    pos += L.count;
    ppos += L.count + 1;
    launches.push_back(L);
  }
  HIPCHK(hipMemcpyAsync(ws, h, upload, hipMemcpyHostToDevice, c->stream));

  // launch shapes; with the scratch address they fix every kernel argument of
  // the round (the tables the kernels read are uploaded before each launch)
  std::vector<uint64_t> sig = {(uint64_t)(uintptr_t)ws, o_items, o_order, o_prefix, o_rows, o_out, o_cnt, JT, NV,
                               n_rows};
  std::vector<uint32_t> blocks_of(launches.size());
  std::vector<int> sv_of(launches.size());
  for (uint32_t v = 0; v < (uint32_t)launches.size(); ++v) {
    const Launch& L = launches[v];
    if (L.jit) {
      sv_of[v] = 0;
      blocks_of[v] = (uint32_t)std::max(1, L.jk.occ_batch) * (uint32_t)c->cus;
    } else {
      sv_of[v] = !L.var.cplx ? c->batch_sv[L.variant]
                 : L.variant < 0 ? qmck::BATCH_SV_COMPLEX_ANY : qmck::BATCH_SV_COMPLEX_INT_HALF;
      blocks_of[v] = (uint32_t)std::max(1, qmck::occupancy_batch(L.var, sv_of[v])) * (uint32_t)c->cus;
    }
    sig.insert(sig.end(), {(uint64_t)L.variant, L.jit ? (uint64_t)(uintptr_t)L.jk.batch : 0, (uint64_t)sv_of[v],
                           L.first, L.count, L.prefix_off, blocks_of[v]});
  }
  auto enqueue = [&](hipStream_t st) -> int {
    for (uint32_t v = 0; v < (uint32_t)launches.size(); ++v) {
      const Launch& L = launches[v];
      if (L.jit) {
        HIPCHK(qmcj::launch_batch(L.jk, (const qmcd::EvalArgs*)(ws + o_items), (const uint32_t*)(ws + o_order) + L.first,
                                  (const uint32_t*)(ws + o_prefix) + L.prefix_off, L.count,
                                  (uint32_t*)(ws + o_cnt) + v, blocks_of[v], st));
        continue;
      }
      HIPCHK(qmck::launch_batch(L.var, sv_of[v], (const qmcd::EvalArgs*)(ws + o_items),
                                (const uint32_t*)(ws + o_order) + L.first,
                                (const uint32_t*)(ws + o_prefix) + L.prefix_off, L.count,
                                (uint32_t*)(ws + o_cnt) + v, blocks_of[v], st));
    }
    return QMC_OK;
  };
  // the evaluation kernels lie between the context's two events (the
  // reported device time, as for a single lattice); the row reduction follows
  auto finish = [&]() -> int {
    HIPCHK(hipEventRecord(c->ev1, c->stream));
    HIPCHK(qmck::launch_finalize_rows((const qmck::RowRef*)(ws + o_rows), (uint32_t)n_rows, d_out, c->stream));
    HIPCHK(hipMemcpyAsync(c->h_stage, d_sign, (size_t)JT * 8 + n_rows * 8, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return QMC_OK;
  };

  // a round of one evaluation kernel launches it directly: a graph of one node
  // only adds launch latency (4% of the round for 1024 replicas of a small job)
  if (c->batch_graph && launches.size() > 1) {
    // a round of the same shape as an earlier one replays that round's graph
    hipGraphExec_t ge = nullptr;
    for (auto& e : c->graphs)
      if (e.sig == sig) {
        ge = e.exec;
        e.last_use = ++c->graph_tick;
        break;
      }
    if (!ge) {
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
      hipError_t ei = hipGraphInstantiate(&ge, g, nullptr, nullptr, 0);
      (void)hipGraphDestroy(g);
      if (ei != hipSuccess) return fail(QMC_EDEVICE, "hipGraphInstantiate failed: %s", hipGetErrorString(ei));
      if (c->graphs.size() >= qmc_context::kGraphCache) {
        auto lru = std::min_element(c->graphs.begin(), c->graphs.end(),
                                    [](const qmc_context::CachedGraph& x, const qmc_context::CachedGraph& y) {
                                      return x.last_use < y.last_use;
                                    });
        HIPCHK(hipStreamSynchronize(c->stream));  // no replay of it may still be queued
        (void)hipGraphExecDestroy(lru->exec);
        c->graphs.erase(lru);
      }
      c->graphs.push_back({sig, ge, ++c->graph_tick});
    }
    // the device interval starts here, after the host has built the graph
    HIPCHK(hipEventRecord(c->ev0, c->stream));
    HIPCHK(hipGraphLaunch(ge, c->stream));
    rc = finish();
    if (rc) return rc;
  } else {
    HIPCHK(hipEventRecord(c->ev0, c->stream));
    rc = enqueue(c->stream);
    if (rc) return rc;
    rc = finish();
    if (rc) return rc;
  }
  float ms = 0;
  HIPCHK(hipEventElapsedTime(&ms, c->ev0, c->ev1));
  if (kernel_seconds) *kernel_seconds = ms * 1e-3;
  const unsigned long long* sg = (const unsigned long long*)c->h_stage;
  const double* hout = c->h_stage + JT;  // the rows follow the sign counts
  for (uint32_t i = 0; i < J; ++i) {
    const Plan& p = plan[i];
    if (p.finish)
      jobs[i]->sums.assign(hout + p.row0, hout + p.row0 + p.rows);
    else
      jobs[i]->sums.clear();
    jobs[i]->sums_at = jobs[i]->sums.data();
    jobs[i]->sums_keep.reset();
    jobs[i]->sign_points = sg[i];
    jobs[i]->fp32_dev.clear();
    jobs[i]->fp32_ref.clear();
    jobs[i]->fp32_dev_points = 0;
    if (p.twin >= 0) {
      const Plan& t = plan[p.twin];
      jobs[i]->fp32_dev.resize(p.rows);
      jobs[i]->fp32_ref.assign(hout + t.row0, hout + t.row0 + p.rows);
      for (uint32_t r = 0; r < p.rows; ++r)
        jobs[i]->fp32_dev[r] = hout[p.pref_row0 + r] - hout[t.row0 + r];
      uint64_t pts = 0;  // points of the sampled tiles (the last tile may be short)
      for (uint32_t q = 0; q < t.ktiles; ++q) {
        const uint64_t k0 = (uint64_t)q * kFp32SampleEvery * t.tile_points;
        pts += std::min<uint64_t>(t.tile_points, jobs[i]->n - k0);
      }
      jobs[i]->fp32_dev_points = pts;
    }
  }
  return QMC_OK;
}

}  // namespace

// The fp32 error is taken as relative to the integral: the sample's summed
// fp32 - fp64 difference over the sample's summed fp64 contribution (complex
// modulus), times the modulus of the estimate.  A bias of the fp32 polynomials
// that is a fraction of the integrand is then read off a sample that need not
// represent the whole cube in value; when the sample is the whole lattice the
// statement is |Q_fp32 - Q_fp64| up to a relative O(error).  A sample whose
// fp64 sum vanishes falls back to the mean difference per point.
void fp32_error(const double* dre, const double* dim, const double* rre, const double* rim, uint32_t m,
                uint64_t points, qmc_result& r) {
  double a = 0.0, b = 0.0, fr = 0.0, fi = 0.0;
  for (uint32_t s = 0; s < m; ++s) {
    a += dre[s];
    b += dim[s];
    fr += rre[s];
    fi += rim[s];
  }
  const double ref = std::hypot(fr, fi);
  if (ref > 0.0 && std::isfinite(ref)) {
    const double q = std::hypot(r.re, r.im);
    r.fp32_err_re = std::fabs(a) / ref * q;
    r.fp32_err_im = std::fabs(b) / ref * q;
  } else {
    const double scale = points ? 1.0 / ((double)m * (double)points) : 0.0;
    r.fp32_err_re = std::fabs(a) * scale;
    r.fp32_err_im = std::fabs(b) * scale;
  }
}

int run_requests(qmc_context* c, const qmc_request* reqs, uint32_t count, qmc_result* out, double* shift_sums) {
  auto t0 = std::chrono::steady_clock::now();
  struct St {
    qmc_integrand* f;
    const double* sh = nullptr;   // shift table: in the call's pool, or in shifts
    std::vector<double> shifts;   // a table grown by the Monte Carlo fallback
    const uint64_t* z = nullptr;  // the request's generating vector, or zown
    std::vector<uint64_t> zown;   // a registered or grown lattice's
    uint64_t n;
    uint32_t mcur = 0, first_new = 0;  // shifts [first_new, mcur) run next
    // per-shift sums at the current lattice: in job.sums when the round evaluated
    // all of its shifts, else in sre, sim (the earlier shifts' sums kept there)
    const double *re = nullptr, *im = nullptr;
    std::vector<double> sre, sim;
    std::vector<double> dre, dim_;     // fp32 evaluation: per-shift sampled fp32 - fp64 sums
    std::vector<double> rre, rim;      // ... and sampled fp64 sums
    uint64_t signs = 0;
    bool done = false;
    qmc_result r{};
    BatchJob job;
  };
  std::vector<St> st(count);
  size_t pool_size = 0;
  for (uint32_t i = 0; i < count; ++i)
    if (reqs[i].f && reqs[i].m <= QMC_MAX_SHIFTS) pool_size += (size_t)reqs[i].m * reqs[i].f->dim;
  std::vector<double> pool(pool_size);  // every request's first shift table
  size_t pool_off = 0;
  // requests usually share generating vectors: each (z, n, dim) is checked once
  const uint64_t* ok_z = nullptr;
  uint64_t ok_n = 0;
  uint32_t ok_dim = 0;
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
      if (!(q.z == ok_z && q.n == ok_n && dim <= ok_dim)) {
        int rc = check_lattice(q.n, dim, q.z);
        if (rc) return rc;
        ok_z = q.z;
        ok_n = q.n;
        ok_dim = dim;
      }
      s.n = q.n;
      s.z = q.z;  // the caller's array outlives the call
    } else {
      uint64_t nn = 0;
      if (next_registered(c, q.n, dim, &nn, true, &s.zown) != QMC_OK)
        return fail(QMC_ENOTFOUND, "request %u: no registered lattice with %u components", i, dim);
      s.n = nn;
      s.z = s.zown.data();
    }
    make_shifts(q.seed, q.m, dim, pool.data() + pool_off);
    s.sh = pool.data() + pool_off;
    pool_off += (size_t)q.m * dim;
    s.mcur = q.m;
    s.r.m = q.m;
    s.r.path = 2;
  }
  double dev = 0.0;
  std::vector<double> qs;  // one shift-mean buffer for every estimate
  for (;;) {
    std::vector<BatchJob*> jobs;
    std::vector<uint32_t> idx;
    for (uint32_t i = 0; i < count; ++i) {
      St& s = st[i];
      if (s.done) continue;
      s.job.f = s.f;
      s.job.n = s.n;
      s.job.z = s.z;
      s.job.m = s.mcur - s.first_new;
      s.job.shifts = s.sh + (size_t)s.first_new * s.f->dim;
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
      if (s.first_new == 0) {  // this round evaluated every shift of the lattice
        s.re = s.job.sums_at;
        s.im = cplx ? s.job.sums_at + madd : nullptr;
      } else {  // shifts added by the Monte Carlo fallback: append to the kept sums
        s.sre.resize(s.first_new);
        s.sre.insert(s.sre.end(), s.job.sums_at, s.job.sums_at + madd);
        s.re = s.sre.data();
        if (cplx) {
          s.sim.resize(s.first_new);
          s.sim.insert(s.sim.end(), s.job.sums_at + madd, s.job.sums_at + 2 * (size_t)madd);
          s.im = s.sim.data();
        }
      }
      s.signs = (s.first_new ? s.signs : 0) + s.job.sign_points;
      if (!s.job.fp32_dev.empty()) {
        auto keep = [&](std::vector<double>& re, std::vector<double>& im, const std::vector<double>& rows) {
          re.resize(s.first_new);
          im.resize(s.first_new);
          re.insert(re.end(), rows.begin(), rows.begin() + madd);
          if (cplx)
            im.insert(im.end(), rows.begin() + madd, rows.begin() + 2 * (size_t)madd);
          else
            im.resize(m, 0.0);
        };
        keep(s.dre, s.dim_, s.job.fp32_dev);
        keep(s.rre, s.rim, s.job.fp32_ref);
      }
      s.r.iterations += 1;
      s.r.evaluations += s.n * (uint64_t)madd;
      s.r.n = s.n;
      s.r.m = m;
      qs.resize(m);
      for (uint32_t k = 0; k < m; ++k) qs[k] = s.re[k] / (double)s.n;
      estimate(qs.data(), m, s.r.re, s.r.err_re);
      s.r.im = s.r.err_im = 0.0;
      if (cplx) {
        for (uint32_t k = 0; k < m; ++k) qs[k] = s.im[k] / (double)s.n;
        estimate(qs.data(), m, s.r.im, s.r.err_im);
      }
      if (!s.job.fp32_dev.empty())
        fp32_error(s.dre.data(), s.dim_.data(), s.rre.data(), s.rim.data(), m, s.job.fp32_dev_points, s.r);
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
        s.zown.swap(g.z);
        s.z = s.zown.data();
        s.first_new = 0;
      } else {
        // the next round overwrites job.sums: keep this lattice's sums
        if (s.re != s.sre.data()) s.sre.assign(s.re, s.re + m);
        if (cplx && s.im != s.sim.data()) s.sim.assign(s.im, s.im + m);
        s.first_new = m;
        s.mcur = g.m;
        s.shifts.resize((size_t)g.m * s.f->dim);
        make_shifts(q.seed, g.m, s.f->dim, s.shifts.data());
        s.sh = s.shifts.data();
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
      std::memcpy(shift_sums + off, s.re, (size_t)m * 8);
      off += m;
      if (s.f->flags & QMC_DEFORM) {
        std::memcpy(shift_sums + off, s.im, (size_t)m * 8);
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

// Default batch schedules of a new context, then the environment's overrides
// (QMC_BATCH_SV, QMC_BATCH_GROUP, QMC_BATCH_TILE, QMC_BATCH_TILE_COMPLEX) and
// the tune cache named by QMC_TUNE_CACHE.
void batch_schedule_defaults(qmc_context* c) {
  int force_sv = -1;
  if (const char* v = std::getenv("QMC_BATCH_SV")) force_sv = atoi(v);  // one points-per-decode variant for all
  for (int dc = 0; dc < 4; ++dc)
    for (int tkc = 0; tkc < qmck::TKC_COUNT; ++tkc)
      for (int f32 = 0; f32 < 2; ++f32) {
        const int v = qmck::BatchVariant{dc, tkc, false, f32 != 0}.index();
        // the autotuner's choices on MI355X: 4 points per decode (despite some
        // spilling), except 2 for fp32 evaluation of at most 4 variables
        c->batch_sv[v] = (f32 && dc == 0) ? 1 : 2;
        if (force_sv >= 0 && force_sv < qmck::BATCH_SV_VARIANTS) c->batch_sv[v] = force_sv;
      }
  if (const char* v = std::getenv("QMC_BATCH_GROUP")) {  // shifts per thread of the real batch kernels (0: all 8)
    const int g = atoi(v);
    if (g >= 0 && g <= qmck::S_REAL)
      for (int vi = 0; vi < qmck::BATCH_VARIANTS; ++vi) c->batch_group[vi] = (uint32_t)g;
  }
  if (const char* v = std::getenv("QMC_TUNE_CACHE")) {
    c->tune_cache = v;
    load_tune_cache(c);
  }
  if (const char* v = std::getenv("QMC_BATCH_TILE")) c->batch_tile_real = std::max(256ull, strtoull(v, nullptr, 10));
  if (const char* v = std::getenv("QMC_BATCH_TILE_COMPLEX"))
    c->batch_tile_complex = std::max(256ull, strtoull(v, nullptr, 10));
}

// Cache lines: "gfx950 <class's largest dimension> <tkc> <complex> <fp32> <sv index> <tile points>
// <shifts per group>".
void load_tune_cache(qmc_context* c) {
  if (c->tune_cache.empty()) return;
  FILE* fh = std::fopen(c->tune_cache.c_str(), "r");
  if (!fh) return;
  int dmax, tkc, cx, f32, sv;
  unsigned long long tile;
  unsigned group;
  char arch[64];
  while (std::fscanf(fh, "%63s %d %d %d %d %d %llu %u", arch, &dmax, &tkc, &cx, &f32, &sv, &tile, &group) == 8) {
    if (std::strcmp(arch, "gfx950") != 0 || tkc < 0 || tkc >= qmck::TKC_COUNT || cx < 0 || cx > 1 || f32 < 0 ||
        f32 > 1 || dmax < 1 || dmax > (int)QMC_MAX_DIM)
      continue;
    const int dc = qmck::dim_class((uint32_t)dmax, cx != 0);
    if (qmck::dim_class_max(dc, cx != 0) != dmax) continue;  // not a class boundary
    const int v = qmck::BatchVariant{dc, tkc, cx != 0, f32 != 0}.index();
    if (sv >= 0 && sv < qmck::BATCH_SV_VARIANTS) c->batch_sv[v] = sv;
    if (tile >= 256 && tile <= (1ull << 24)) c->batch_tile[v] = tile;
    if (group <= (unsigned)qmck::S_REAL) c->batch_group[v] = group;
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
    if (!v.fp32 && (reqs[i].f->flags & QMC_SPECIALISE) && c->jit) continue;
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
    // complex kernels: the jobs' power class, not a tuning choice, picks the sv index
    const int nsv = var.cplx ? 1 : qmck::BATCH_SV_VARIANTS;
    // shifts per thread: all the kernel holds (0), or groups of 4 or 2: more,
    // smaller tiles (a small batch spreads over more workgroups) for more
    // index work per evaluation; complex kernels hold one shift per thread
    const std::vector<uint32_t> groups = var.cplx ? std::vector<uint32_t>{0} : std::vector<uint32_t>{0, 4, 2};
    double best = 1e300;
    int best_sv = 0;
    uint64_t best_tile = tiles[0];
    uint32_t best_group = 0;
    for (int sv = 0; sv < nsv; ++sv) {
      if (!qmck::batch_kernel(var, sv)) continue;
      for (uint32_t group : groups) {
        for (uint64_t tile : tiles) {
          c->batch_sv[vi] = sv;
          c->batch_tile[vi] = tile;
          c->batch_group[vi] = group;
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
            best_group = group;
          }
        }
      }
    }
    c->batch_sv[vi] = best_sv;
    c->batch_tile[vi] = best_tile;
    c->batch_group[vi] = best_group;
    if (!c->tune_cache.empty()) {
      if (FILE* fh = std::fopen(c->tune_cache.c_str(), "a")) {
        std::fprintf(fh, "gfx950 %d %d %d %d %d %llu %u\n", qmck::dim_class_max(var.dclass, var.cplx), var.tkc,
                     var.cplx ? 1 : 0, var.fp32 ? 1 : 0,
                     best_sv, (unsigned long long)best_tile, best_group);
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
  CtxLock g(c);
  if (c->broken) return qmch::fail(QMC_EDEVICE, "context is unusable after a device error");
  HIPCHK(hipSetDevice(c->device));
  return qmch::autotune(c, reqs, count, configs_tried);
}
