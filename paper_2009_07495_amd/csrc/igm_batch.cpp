// C ABI of the batched solver: setup of many systems (host threads), one
// device arena per array kind, the job order of the persistent kernel, launch
// shapes and their autotuning, and per-system results.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <new>
#include <numeric>
#include <thread>
#include <vector>

#include "igm_batch.hpp"
#include "igm_team.hpp"

using namespace igm;

struct igm_batch {
  int device = 0;
  hipStream_t stream = nullptr;
  igm_policy pol{};
  int32_t nsys = 0;
  std::vector<int64_t> n, nnz;
  std::vector<int32_t> nterms;
  int64_t total_n = 0, total_nnz = 0;
  std::vector<BatchSys> sys;  // host copy of the device records
  std::vector<void *> bufs;
  int64_t device_bytes = 0;
  BatchSys *d_sys = nullptr;
  int32_t *d_jobs = nullptr;
  int32_t njobs = 0;
  int32_t *d_ctl = nullptr;  // [0] job queue, [1] timeout flag
  BatchResult *d_res = nullptr;
  std::vector<BatchResult> res;
  unsigned long long *d_words = nullptr;
  double *d_x = nullptr;  // solution buffer of igm_batch_solve and the autotuner
  int block = 0, rows = 0, grid = 0;
  std::vector<int32_t> team;
  igm_stats stats{};
  double wall_us_per_tick = 0.0;
  int last_error_line = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
};

namespace {

#define BT_HIP(call)                          \
  do {                                        \
    hipError_t e_ = (call);                   \
    if (e_ != hipSuccess) {                   \
      bt->last_error_line = __LINE__;         \
      return IGM_ERR_DEVICE;                  \
    }                                         \
  } while (0)

#define BT_TRY(call)               \
  do {                             \
    igm_status st_ = (call);       \
    if (st_ != IGM_OK) return st_; \
  } while (0)

constexpr int kMaxBatchM = 64;  // H lives in LDS: (m+1) m words
constexpr int64_t kAlign = 32;  // elements: every per-system segment starts 256-byte aligned (int64)

int64_t round_up(int64_t v, int64_t a) { return (v + a - 1) / a * a; }

double ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

template <class T>
igm_status arena(igm_batch *bt, T *&p, int64_t count) {
  const size_t bytes = sizeof(T) * (size_t)std::max<int64_t>(count, 1);
  void *q = nullptr;
  if (hipMalloc(&q, bytes) != hipSuccess) return IGM_ERR_OOM;
  bt->bufs.push_back(q);
  bt->device_bytes += (int64_t)bytes;
  p = (T *)q;
  return IGM_OK;
}

// Offsets of per-system segments of `len[s]` elements, each aligned.
int64_t layout(const std::vector<int64_t> &len, std::vector<int64_t> &off) {
  off.resize(len.size());
  int64_t t = 0;
  for (size_t s = 0; s < len.size(); ++s) {
    off[s] = t;
    t += round_up(len[s], kAlign);
  }
  return t;
}

void free_batch(igm_batch *bt) {
  for (void *p : bt->bufs) (void)hipFree(p);
  bt->bufs.clear();
  if (bt->ev0) (void)hipEventDestroy(bt->ev0);
  if (bt->ev1) (void)hipEventDestroy(bt->ev1);
  bt->ev0 = bt->ev1 = nullptr;
}

// Team sizes, job order (largest systems first, members consecutive), grid.
igm_status apply_shape(igm_batch *bt, int block, int rows) {
  const void *k = batch_kernel(block, rows, bt->pol.precond);
  if (!k) return IGM_ERR_ARG;
  hipDeviceProp_t prop;
  BT_HIP(hipGetDeviceProperties(&prop, bt->device));
  int nb = 0;
  BT_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k, block, batch_smem_bytes(bt->pol.m)));
  const int64_t cap = (int64_t)nb * prop.multiProcessorCount;
  if (cap < 1) return IGM_ERR_UNSUPPORTED;
  const int64_t per = (int64_t)block * rows;
  std::vector<int32_t> team(bt->nsys);
  int64_t njobs = 0;
  for (int32_t s = 0; s < bt->nsys; ++s) {
    const int64_t t = (bt->n[s] + per - 1) / per;
    if (t > kTeamMax || t > cap) return IGM_ERR_UNSUPPORTED;
    team[s] = (int32_t)t;
    njobs += t;
  }
  std::vector<int32_t> order(bt->nsys);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
    return bt->n[a] * (bt->nnz[a] / std::max<int64_t>(bt->n[a], 1) + bt->pol.m) >
           bt->n[b] * (bt->nnz[b] / std::max<int64_t>(bt->n[b], 1) + bt->pol.m);
  });
  std::vector<int32_t> jobs;
  jobs.reserve(2 * njobs);
  for (int32_t s : order)
    for (int32_t q = 0; q < team[s]; ++q) {
      jobs.push_back(s);
      jobs.push_back(q);
    }
  for (int32_t s = 0; s < bt->nsys; ++s) bt->sys[s].team = team[s];
  BT_HIP(hipMemcpy(bt->d_sys, bt->sys.data(), sizeof(BatchSys) * bt->nsys, hipMemcpyHostToDevice));
  BT_HIP(hipMemcpy(bt->d_jobs, jobs.data(), sizeof(int32_t) * jobs.size(), hipMemcpyHostToDevice));
  bt->team = team;
  bt->njobs = (int32_t)njobs;
  bt->grid = (int)std::min<int64_t>(cap, njobs);
  bt->block = block;
  bt->rows = rows;
  return IGM_OK;
}

igm_status run(igm_batch *bt, double *x_dev) {
  auto t0 = std::chrono::steady_clock::now();
  const igm_policy &p = bt->pol;
  BT_HIP(hipMemsetAsync(bt->d_ctl, 0, 2 * sizeof(int32_t), bt->stream));
  BT_HIP(hipMemsetAsync(bt->d_words, 0, sizeof(unsigned long long) * kTeamSlots * kTeamWords * (size_t)bt->nsys,
                        bt->stream));
  for (auto &r : bt->res) {
    memset(&r, 0, sizeof(r));
    r.status = IGM_ERR_DEVICE;  // overwritten by the system's first member
    r.first_ovf = kNoEvent;
    r.jstar = -1;
  }
  BT_HIP(hipMemcpyAsync(bt->d_res, bt->res.data(), sizeof(BatchResult) * bt->nsys, hipMemcpyHostToDevice,
                        bt->stream));
  BatchArgs a;
  memset(&a, 0, sizeof(a));
  a.sys = bt->d_sys;
  a.jobs = bt->d_jobs;
  a.njobs = bt->njobs;
  a.m = p.m;
  a.df = p.df;
  a.precond = p.precond;
  a.b_dot = p.b_dot; a.b_axpy = p.b_axpy; a.b_norm = p.b_norm;
  a.b_div_num = p.b_div_num; a.b_div_den = p.b_div_den; a.b_rot = p.b_rot; a.b_tmp = p.b_tmp;
  a.b_cs_num = p.b_cs_num; a.b_cs_den = p.b_cs_den;
  a.max_refine = p.max_refine;
  a.phase_clock = p.phase_clock;
  a.gtol = p.gtol;
  a.tol = p.tol;
  a.queue = bt->d_ctl;
  a.timeout = bt->d_ctl + 1;
  a.res = bt->d_res;
  a.x = x_dev;
  void *args[] = {(void *)&a};
  const void *k = batch_kernel(bt->block, bt->rows, p.precond);
  BT_HIP(hipEventRecord(bt->ev0, bt->stream));
  BT_HIP(hipLaunchCooperativeKernel(k, dim3(bt->grid), dim3(bt->block), args, batch_smem_bytes(p.m), bt->stream));
  BT_HIP(hipEventRecord(bt->ev1, bt->stream));
  int32_t ctl[2] = {0, 0};
  BT_HIP(hipMemcpyAsync(bt->res.data(), bt->d_res, sizeof(BatchResult) * bt->nsys, hipMemcpyDeviceToHost,
                        bt->stream));
  BT_HIP(hipMemcpyAsync(ctl, bt->d_ctl, sizeof(ctl), hipMemcpyDeviceToHost, bt->stream));
  BT_HIP(hipStreamSynchronize(bt->stream));
  float ms = 0.f;
  BT_HIP(hipEventElapsedTime(&ms, bt->ev0, bt->ev1));
  igm_status status = IGM_OK;
  int64_t refs = 0, iters = 0;
  for (const auto &r : bt->res) {
    refs += r.refinements;
    iters += r.iterations;
    if (status == IGM_OK && r.status != IGM_OK) status = (igm_status)r.status;
  }
  if (ctl[1]) status = IGM_ERR_DEVICE;
  igm_stats &st = bt->stats;
  st.status = status;
  st.refinements = (int32_t)std::min<int64_t>(refs, INT32_MAX);
  st.iterations = (int32_t)std::min<int64_t>(iters, INT32_MAX);
  st.time_kernel_ms = ms;
  st.time_cycle_ms = ms;
  st.time_solve_ms = ms_since(t0);
  return status;
}

igm_status setup(igm_batch *bt, const int64_t *n, const int64_t *row_ptr, const int32_t *col, const double *val,
                 const double *b, int32_t *failed) {
  const int32_t ns = bt->nsys;
  const igm_policy &p = bt->pol;
  // offsets of each system in the caller's arrays, validation
  std::vector<int64_t> rp_off(ns), nz_off(ns), b_off(ns);
  int64_t trp = 0, tnz = 0, tb = 0;
  bt->n.resize(ns);
  bt->nnz.resize(ns);
  for (int32_t s = 0; s < ns; ++s) {
    if (n[s] < 1 || n[s] >= ((int64_t)1 << 31)) { if (failed) *failed = s; return IGM_ERR_ARG; }
    rp_off[s] = trp;
    nz_off[s] = tnz;
    b_off[s] = tb;
    const int64_t *rp = row_ptr + trp;
    if (rp[0] != 0 || rp[n[s]] < 0) { if (failed) *failed = s; return IGM_ERR_ARG; }
    igm_status v = validate_csr(n[s], rp, col + tnz, val + tnz, b + tb);
    if (v != IGM_OK) { if (failed) *failed = s; return v; }
    bt->n[s] = n[s];
    bt->nnz[s] = rp[n[s]];
    trp += n[s] + 1;
    tnz += rp[n[s]];
    tb += n[s];
  }
  bt->total_n = tb;
  bt->total_nnz = tnz;
  // host setup of every system, in parallel
  std::vector<HostSetup> hs(ns);
  std::vector<igm_status> sst(ns, IGM_OK);
  std::atomic<int32_t> next(0);
  auto worker = [&] {
    for (;;) {
      const int32_t s = next.fetch_add(1);
      if (s >= ns) break;
      const int64_t *rp = row_ptr + rp_off[s];
      std::vector<int64_t> rpv(rp, rp + n[s] + 1);
      std::vector<int32_t> cv(col + nz_off[s], col + nz_off[s] + bt->nnz[s]);
      std::vector<double> av(val + nz_off[s], val + nz_off[s] + bt->nnz[s]);
      std::vector<double> bv(b + b_off[s], b + b_off[s] + n[s]);
      sst[s] = host_setup(n[s], rpv, cv, av, bv, p, hs[s]);
    }
  };
  const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<std::thread> pool;
  for (unsigned t = 1; t < std::min<unsigned>(hw, (unsigned)ns); ++t) pool.emplace_back(worker);
  worker();
  for (auto &t : pool) t.join();
  for (int32_t s = 0; s < ns; ++s)
    if (sst[s] != IGM_OK) { if (failed) *failed = s; return sst[s]; }

  // arenas
  const int m = p.m;
  bt->nterms.resize(ns);
  int max_terms = 1;
  std::vector<int64_t> L_rp(ns), L_nz(ns), L_n(ns), L_soff(ns), L_sw(ns), L_sent(ns), L_V(ns), L_W(ns);
  for (int32_t s = 0; s < ns; ++s) {
    bt->nterms[s] = std::min(p.s_terms + 1, hs[s].nterms);
    max_terms = std::max(max_terms, bt->nterms[s]);
    L_rp[s] = n[s] + 1;
    L_nz[s] = bt->nnz[s];
    L_n[s] = n[s];
    L_soff[s] = (int64_t)hs[s].sell_off.size();
    L_sw[s] = (int64_t)hs[s].sell_w.size();
    L_sent[s] = (int64_t)hs[s].sell_col.size();
    L_V[s] = (int64_t)(m + 1) * round_up(n[s], 16);
    L_W[s] = (int64_t)kTeamSlots * kTeamWords;
  }
  std::vector<int64_t> O_rp, O_nz, O_n, O_soff, O_sw, O_sent, O_V, O_W;
  int64_t *d_rp, *d_soff, *d_ld = nullptr, *d_ud = nullptr, *d_V;
  int64_t *d_sval[kMaxTerms] = {nullptr};
  int32_t *d_col, *d_sw, *d_scol;
  double *d_a, *d_ah, *d_b, *d_bh;
  BT_TRY(arena(bt, d_rp, layout(L_rp, O_rp)));
  const int64_t tot_nz = layout(L_nz, O_nz);
  BT_TRY(arena(bt, d_col, tot_nz));
  BT_TRY(arena(bt, d_a, tot_nz));
  BT_TRY(arena(bt, d_ah, tot_nz));
  const int64_t tot_n = layout(L_n, O_n);
  BT_TRY(arena(bt, d_b, tot_n));
  BT_TRY(arena(bt, d_bh, tot_n));
  if (p.precond == IGM_PRE_JACOBI) {
    BT_TRY(arena(bt, d_ld, tot_n));
    BT_TRY(arena(bt, d_ud, tot_n));
  }
  BT_TRY(arena(bt, d_soff, layout(L_soff, O_soff)));
  BT_TRY(arena(bt, d_sw, layout(L_sw, O_sw)));
  const int64_t tot_sent = layout(L_sent, O_sent);
  BT_TRY(arena(bt, d_scol, tot_sent));
  for (int l = 0; l < max_terms; ++l) BT_TRY(arena(bt, d_sval[l], tot_sent));
  BT_TRY(arena(bt, d_V, layout(L_V, O_V)));
  BT_TRY(arena(bt, bt->d_words, layout(L_W, O_W)));
  BT_TRY(arena(bt, bt->d_x, bt->total_n));
  BT_TRY(arena(bt, bt->d_sys, ns));
  int64_t max_jobs = (int64_t)ns * kTeamMax * 2;
  BT_TRY(arena(bt, bt->d_jobs, max_jobs));
  BT_TRY(arena(bt, bt->d_ctl, 2));
  BT_TRY(arena(bt, bt->d_res, ns));
  BT_HIP(hipMemset(d_V, 0, sizeof(int64_t) * (size_t)(O_V.back() + round_up(L_V.back(), kAlign))));
  bt->sys.resize(ns);
  bt->res.resize(ns);
  int64_t xo = 0;
  for (int32_t s = 0; s < ns; ++s) {
    const HostSetup &h = hs[s];
    BatchSys &S = bt->sys[s];
    memset(&S, 0, sizeof(S));
    S.n = n[s];
    S.ldv = round_up(n[s], 16);
    S.x_off = xo;
    xo += n[s];
    S.team = 1;
    S.nterms = bt->nterms[s];
    for (int l = 0; l < kMaxTerms; ++l) S.alpha[l] = h.alpha[l];
    const size_t nn = (size_t)n[s], nz = (size_t)bt->nnz[s];
    auto up = [&](void *dst, const void *src, size_t bytes) -> hipError_t {
      return bytes ? hipMemcpy(dst, src, bytes, hipMemcpyHostToDevice) : hipSuccess;
    };
    BT_HIP(up(d_rp + O_rp[s], row_ptr + rp_off[s], sizeof(int64_t) * (nn + 1)));
    BT_HIP(up(d_col + O_nz[s], col + nz_off[s], sizeof(int32_t) * nz));
    BT_HIP(up(d_a + O_nz[s], h.a.data(), sizeof(double) * nz));
    BT_HIP(up(d_ah + O_nz[s], val + nz_off[s], sizeof(double) * nz));
    BT_HIP(up(d_b + O_n[s], h.b.data(), sizeof(double) * nn));
    BT_HIP(up(d_bh + O_n[s], b + b_off[s], sizeof(double) * nn));
    BT_HIP(up(d_soff + O_soff[s], h.sell_off.data(), sizeof(int64_t) * h.sell_off.size()));
    BT_HIP(up(d_sw + O_sw[s], h.sell_w.data(), sizeof(int32_t) * h.sell_w.size()));
    BT_HIP(up(d_scol + O_sent[s], h.sell_col.data(), sizeof(int32_t) * h.sell_col.size()));
    for (int l = 0; l < S.nterms; ++l) {
      BT_HIP(up(d_sval[l] + O_sent[s], h.sell_val[l].data(), sizeof(int64_t) * h.sell_val[l].size()));
      S.sell_val[l] = d_sval[l] + O_sent[s];
    }
    if (p.precond == IGM_PRE_JACOBI) {
      BT_HIP(up(d_ld + O_n[s], h.ldiag.data(), sizeof(int64_t) * nn));
      BT_HIP(up(d_ud + O_n[s], h.udiag.data(), sizeof(int64_t) * nn));
      S.ldiag = d_ld + O_n[s];
      S.udiag = d_ud + O_n[s];
    }
    S.row_ptr = d_rp + O_rp[s];
    S.col = d_col + O_nz[s];
    S.a = d_a + O_nz[s];
    S.ahat = d_ah + O_nz[s];
    S.b = d_b + O_n[s];
    S.bhat = d_bh + O_n[s];
    S.sell_off = d_soff + O_soff[s];
    S.sell_w = d_sw + O_sw[s];
    S.sell_col = d_scol + O_sent[s];
    S.V = d_V + O_V[s];
    S.words = bt->d_words + O_W[s];
  }
  return IGM_OK;
}

// Shapes in order of preference: fewest rows per thread with the largest
// workgroup first.
igm_status default_shape(igm_batch *bt) {
  for (int i = 0; i < kNumBatchShapes; ++i) {
    igm_status st = apply_shape(bt, kBatchShapes[i][0], kBatchShapes[i][1]);
    if (st == IGM_OK) return IGM_OK;
    if (st != IGM_ERR_UNSUPPORTED) return st;
  }
  return IGM_ERR_UNSUPPORTED;
}

}  // namespace

extern "C" {

igm_status igm_batch_create(int32_t nsys, const int64_t *n, const int64_t *row_ptr, const int32_t *col,
                            const double *val, const double *b, const igm_policy *pol, int32_t *failed,
                            igm_batch **out) {
  if (failed) *failed = -1;
  if (!out) return IGM_ERR_ARG;
  *out = nullptr;
  if (nsys < 1 || !n || !row_ptr || !col || !val || !b || !pol) return IGM_ERR_ARG;
  if (pol->struct_size != (int32_t)sizeof(igm_policy)) return IGM_ERR_ARG;
  igm_status st = check_policy(*pol);
  if (st != IGM_OK) return st;
  if (pol->precond == IGM_PRE_ILU0 || pol->m > kMaxBatchM) return IGM_ERR_UNSUPPORTED;
  auto t0 = std::chrono::steady_clock::now();
  igm_batch *bt = new (std::nothrow) igm_batch();
  if (!bt) return IGM_ERR_OOM;
  bt->pol = *pol;
  bt->nsys = nsys;
  st = IGM_OK;
  if (hipGetDevice(&bt->device) != hipSuccess || hipEventCreate(&bt->ev0) != hipSuccess ||
      hipEventCreate(&bt->ev1) != hipSuccess)
    st = IGM_ERR_DEVICE;
  if (st == IGM_OK) st = setup(bt, n, row_ptr, col, val, b, failed);
  if (st == IGM_OK) st = default_shape(bt);
  if (st == IGM_OK) {
    int wall_khz = 0;
    if (hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, bt->device) != hipSuccess)
      st = IGM_ERR_DEVICE;
    bt->wall_us_per_tick = wall_khz > 0 ? 1000.0 / wall_khz : 0.0;
  }
  if (st != IGM_OK) {
    free_batch(bt);
    delete bt;
    return st;
  }
  bt->stats.time_setup_ms = ms_since(t0);
  *out = bt;
  return IGM_OK;
}

igm_status igm_batch_set_stream(igm_batch *bt, void *hip_stream) {
  if (!bt) return IGM_ERR_ARG;
  bt->stream = (hipStream_t)hip_stream;
  return IGM_OK;
}

igm_status igm_batch_set_shape(igm_batch *bt, int32_t block, int32_t rows_per_thread) {
  if (!bt) return IGM_ERR_ARG;
  const int ob = bt->block, orr = bt->rows;
  igm_status st = apply_shape(bt, block, rows_per_thread);
  if (st != IGM_OK && ob) (void)apply_shape(bt, ob, orr);
  return st;
}

igm_status igm_batch_set_phase_clock(igm_batch *bt, int32_t on) {
  if (!bt || on < 0 || on > 1) return IGM_ERR_ARG;
  bt->pol.phase_clock = on;
  return IGM_OK;
}

igm_status igm_batch_autotune(igm_batch *bt, int32_t *block, int32_t *rows_per_thread) {
  if (!bt) return IGM_ERR_ARG;
  int best_b = bt->block, best_r = bt->rows;
  double best = 1e300;
  for (int i = 0; i < kNumBatchShapes; ++i) {
    igm_status st = apply_shape(bt, kBatchShapes[i][0], kBatchShapes[i][1]);
    if (st == IGM_ERR_UNSUPPORTED) continue;
    if (st != IGM_OK) return st;
    double t = 1e300;
    for (int rep = 0; rep < 2; ++rep) {  // the first run warms caches and code
      BT_HIP(hipMemsetAsync(bt->d_x, 0, sizeof(double) * (size_t)bt->total_n, bt->stream));
      st = run(bt, bt->d_x);
      if (st == IGM_ERR_DEVICE) return st;
      t = std::min(t, (double)bt->stats.time_kernel_ms);
    }
    if (t < best) {
      best = t;
      best_b = kBatchShapes[i][0];
      best_r = kBatchShapes[i][1];
    }
  }
  BT_TRY(apply_shape(bt, best_b, best_r));
  if (block) *block = best_b;
  if (rows_per_thread) *rows_per_thread = best_r;
  return IGM_OK;
}

igm_status igm_batch_solve_device(igm_batch *bt, double *x_dev) {
  if (!bt || !x_dev) return IGM_ERR_ARG;
  return run(bt, x_dev);
}

igm_status igm_batch_solve(igm_batch *bt, double *x) {
  if (!bt || !x) return IGM_ERR_ARG;
  BT_HIP(hipMemcpyAsync(bt->d_x, x, sizeof(double) * (size_t)bt->total_n, hipMemcpyHostToDevice, bt->stream));
  igm_status st = run(bt, bt->d_x);
  if (st == IGM_ERR_DEVICE) return st;
  BT_HIP(hipMemcpyAsync(x, bt->d_x, sizeof(double) * (size_t)bt->total_n, hipMemcpyDeviceToHost, bt->stream));
  BT_HIP(hipStreamSynchronize(bt->stream));
  return st;
}

igm_status igm_batch_get_result(const igm_batch *bt, int32_t i, igm_stats *out) {
  if (!bt || !out || i < 0 || i >= bt->nsys) return IGM_ERR_ARG;
  memset(out, 0, sizeof(*out));
  const BatchResult &r = bt->res[i];
  out->struct_size = sizeof(igm_stats);
  out->status = r.status;
  out->refinements = r.refinements;
  out->iterations = r.iterations;
  out->first_ovf = r.first_ovf;
  out->relres_orig = r.relres_orig;
  out->relres_scaled = r.relres_scaled;
  out->time_solve_ms = r.t_end >= r.t_begin ? (double)(r.t_end - r.t_begin) * bt->wall_us_per_tick / 1000.0 : 0.0;
  out->n = bt->n[i];
  out->nnz = bt->nnz[i];
  out->nterms = bt->nterms[i];
  out->grid_blocks = bt->team.empty() ? 0 : bt->team[i];
  out->block_threads = bt->block;
  out->rows_per_thread = bt->rows;
  for (int k = 0; k < 8; ++k) out->phase_us[k] = (double)r.phase[k] * bt->wall_us_per_tick;
  return IGM_OK;
}

igm_status igm_batch_get_stats(const igm_batch *bt, igm_stats *out) {
  if (!bt || !out) return IGM_ERR_ARG;
  *out = bt->stats;
  out->struct_size = sizeof(igm_stats);
  out->n = bt->total_n;
  out->nnz = bt->total_nnz;
  out->grid_blocks = bt->grid;
  out->block_threads = bt->block;
  out->rows_per_thread = bt->rows;
  out->device_bytes = bt->device_bytes;
  out->last_error_line = bt->last_error_line;
  return IGM_OK;
}

void igm_batch_destroy(igm_batch *bt) {
  if (!bt) return;
  free_batch(bt);
  delete bt;
}

}  // extern "C"
