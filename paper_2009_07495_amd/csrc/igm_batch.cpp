// Batched solver (C ABI) and the host helpers it shares with the served
// solver: per-system preparation (validation and host setup, in parallel
// threads), one device region per system, the job order of the persistent
// kernel, launch shapes and their autotuning, and per-system results.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <new>
#include <numeric>
#include <string>
#include <thread>
#include <vector>

#include "igm_batch.hpp"
#include "igm_par.hpp"
#include "igm_trace.hpp"
#include "igm_team.hpp"

using namespace igm;

namespace igm {

namespace {

constexpr size_t kSegAlign = 256;  // every array of a region starts 256-byte aligned

size_t align_up(size_t v) { return (v + kSegAlign - 1) / kSegAlign * kSegAlign; }

// Walks the arrays of one system's region in a fixed order; used both to size
// the region and to place the arrays.
template <class F>
void walk_region(const HostSystem &hs, bool own_x, F &&f) {
  const HostSetup &h = hs.h;
  const size_t n = (size_t)hs.n, nz = (size_t)hs.nnz;
  const size_t ldv = (size_t)((hs.n + 15) / 16 * 16);
  const size_t sell = h.sell_off.empty() ? 0 : (size_t)h.sell_off.back();
  const bool pre = hs.pol.precond != IGM_PRE_NONE, ilu = hs.pol.precond == IGM_PRE_ILU0;
  // inputs and structure (always made by the host), x, exchange words
  f("row_ptr", sizeof(int64_t) * (n + 1));
  f("col", sizeof(int32_t) * nz);
  f("ahat", sizeof(double) * nz);
  f("bhat", sizeof(double) * n);
  f("sell_off", sizeof(int64_t) * h.sell_off.size());
  f("sell_w", sizeof(int32_t) * h.sell_w.size());
  f("sell_col", sizeof(int32_t) * h.sell_col.size());
  if (hs.device_setup) f("diag_pos", sizeof(int64_t) * n);
  if (ilu) {
    f("lptr", sizeof(int64_t) * h.lptr.size());
    f("uptr", sizeof(int64_t) * h.uptr.size());
    f("lcol", sizeof(int32_t) * h.lcol.size());
    f("ucol", sizeof(int32_t) * h.ucol.size());
    f("flev_ptr", sizeof(int32_t) * h.flev_ptr.size());
    f("flev_rows", sizeof(int32_t) * h.flev_rows.size());
    f("blev_ptr", sizeof(int32_t) * h.blev_ptr.size());
    f("blev_rows", sizeof(int32_t) * h.blev_rows.size());
  }
  if (own_x) f("x", sizeof(double) * n);
  f("words", sizeof(unsigned long long) * (size_t)kTeamSlots * kTeamWords);
  // values of the setup (made by the host, or by the kernel with device setup)
  f("a", sizeof(double) * nz);
  f("b", sizeof(double) * n);
  if (hs.pol.two_sided) f("cscale", sizeof(double) * n);
  for (int l = 0; l < hs.nterms; ++l) f("sell_val", sizeof(int64_t) * sell);
  if (pre) {
    f("ldiag", sizeof(int64_t) * n);
    f("udiag", sizeof(int64_t) * n);
  }
  if (ilu) {
    f("lval", sizeof(int64_t) * (size_t)h.lptr[n]);
    f("uval", sizeof(int64_t) * (size_t)h.uptr[n]);
    f("lvalf", sizeof(double) * (size_t)h.lptr[n]);
    f("uvalf", sizeof(double) * (size_t)h.uptr[n]);
  }
  // work arrays (written before they are read)
  if (ilu) {
    f("zbuf", sizeof(int64_t) * n);
    f("wbuf", sizeof(int64_t) * n);
    f("fbuf", sizeof(double) * n);
    f("lev_cnt", sizeof(unsigned) * (h.flev_ptr.size() - 1 + h.blev_ptr.size() - 1) * kLevStride);
  }
  f("V", sizeof(int64_t) * (size_t)(hs.pol.m + 1) * ldv);
}

// The first array of the setup's values (not part of a device setup's image).
bool is_value_array(const char *name) { return std::string(name) == "a"; }

bool is_work_array(const char *name) {
  const std::string nm(name);
  return nm == "zbuf" || nm == "wbuf" || nm == "fbuf" || nm == "lev_cnt" || nm == "V";
}

// Host source of a data array of the region (nullptr for x and words).
const void *array_source(const HostSystem &hs, const char *name, int &term) {
  const HostSetup &h = hs.h;
  const std::string nm(name);
  if (nm == "row_ptr") return hs.row_ptr.data();
  if (nm == "col") return hs.col.data();
  if (nm == "a") return h.a.data();
  if (nm == "ahat") return hs.ahat.data();
  if (nm == "b") return h.b.data();
  if (nm == "bhat") return hs.bhat.data();
  if (nm == "cscale") return h.cscale.data();
  if (nm == "diag_pos") return h.diag_pos.data();
  if (nm == "sell_off") return h.sell_off.data();
  if (nm == "sell_w") return h.sell_w.data();
  if (nm == "sell_col") return h.sell_col.data();
  if (nm == "sell_val") return h.sell_val[term++].data();
  if (nm == "ldiag") return h.ldiag.data();
  if (nm == "udiag") return h.udiag.data();
  if (nm == "lptr") return h.lptr.data();
  if (nm == "uptr") return h.uptr.data();
  if (nm == "lcol") return h.lcol.data();
  if (nm == "ucol") return h.ucol.data();
  if (nm == "lval") return h.lval.data();
  if (nm == "uval") return h.uval.data();
  if (nm == "lvalf") return hs.lvalf.data();
  if (nm == "uvalf") return hs.uvalf.data();
  if (nm == "flev_ptr") return h.flev_ptr.data();
  if (nm == "flev_rows") return h.flev_rows.data();
  if (nm == "blev_ptr") return h.blev_ptr.data();
  if (nm == "blev_rows") return h.blev_rows.data();
  return nullptr;
}

}  // namespace

igm_status prepare_system(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
                          const double *b, const igm_policy &pol, HostSystem &out, bool allow_device_setup) {
  if (pol.struct_size != (int32_t)sizeof(igm_policy)) return IGM_ERR_ARG;
  igm_status st = check_policy(pol);
  if (st != IGM_OK) return st;
  if (pol.m > kMaxBatchM) return IGM_ERR_UNSUPPORTED;
  st = validate_csr(n, row_ptr, col, val, b);
  if (st != IGM_OK) return st;
  out.n = n;
  out.nnz = row_ptr[n];
  out.pol = pol;
  par_assign(out.row_ptr, row_ptr, n + 1);
  par_assign(out.col, col, out.nnz);
  par_assign(out.ahat, val, out.nnz);
  par_assign(out.bhat, b, n);
  // device setup: the ILU(0) factors are built in the basis array, which must hold them
  const int64_t ldv = (n + 15) / 16 * 16;
  out.device_setup = allow_device_setup && pol.s_terms == 0 && !pol.gauss_seidel &&
                     (pol.precond != IGM_PRE_ILU0 || out.nnz <= (int64_t)(pol.m + 1) * ldv);
  if (out.device_setup) {
    st = host_structure(n, out.row_ptr, out.col, pol, out.h);
    out.nterms = 1;
    return st;
  }
  st = host_setup(n, out.row_ptr, out.col, out.ahat, out.bhat, pol, out.h);
  if (st != IGM_OK) return st;
  out.nterms = std::min(pol.s_terms + 1, out.h.nterms);
  if (pol.precond == IGM_PRE_ILU0) {
    par_assign(out.lvalf, out.h.lval.data(), (int64_t)out.h.lval.size());
    par_assign(out.uvalf, out.h.uval.data(), (int64_t)out.h.uval.size());
  }
  return IGM_OK;
}

size_t system_bytes(const HostSystem &hs, bool own_x) {
  size_t total = 0;
  walk_region(hs, own_x, [&](const char *, size_t bytes) { total += align_up(bytes); });
  return total;
}

void record_for(const HostSystem &hs, bool own_x, char *base, BatchSys &S) {
  const HostSetup &h = hs.h;
  const igm_policy &p = hs.pol;
  memset(&S, 0, sizeof(S));
  S.n = hs.n;
  S.ldv = (hs.n + 15) / 16 * 16;
  S.team = 1;
  S.nterms = hs.nterms;
  S.s_rule = p.s_rule;
  S.m = p.m; S.df = p.df; S.precond = p.precond; S.max_refine = p.max_refine;
  S.b_dot = p.b_dot; S.b_axpy = p.b_axpy; S.b_norm = p.b_norm;
  S.b_div_num = p.b_div_num; S.b_div_den = p.b_div_den; S.b_rot = p.b_rot; S.b_tmp = p.b_tmp;
  S.b_cs_num = p.b_cs_num; S.b_cs_den = p.b_cs_den;
  S.gtol = p.gtol;
  S.tol = p.tol;
  S.shift_retry = p.shift_retry;
  for (int l = 0; l < kMaxTerms; ++l) S.alpha[l] = h.alpha[l];
  S.device_setup = hs.device_setup ? 1 : 0;
  S.alpha_a = p.alpha_a;
  if (p.precond == IGM_PRE_ILU0) {
    S.nflev = h.flev_ptr.empty() ? 0 : (int32_t)h.flev_ptr.size() - 1;
    S.nblev = h.blev_ptr.empty() ? 0 : (int32_t)h.blev_ptr.size() - 1;
    S.max_level = max_level_rows(h);
  }
  size_t off = 0;
  int term = 0;
  walk_region(hs, own_x, [&](const char *name, size_t bytes) {
    char *d = base + off;
    off += align_up(bytes);
    const std::string nm(name);
    if (nm == "row_ptr") S.row_ptr = (const int64_t *)d;
    else if (nm == "col") S.col = (const int32_t *)d;
    else if (nm == "a") S.a = (const double *)d;
    else if (nm == "ahat") S.ahat = (const double *)d;
    else if (nm == "b") S.b = (const double *)d;
    else if (nm == "bhat") S.bhat = (const double *)d;
    else if (nm == "cscale") S.cscale = (const double *)d;
    else if (nm == "diag_pos") S.diag_pos = (const int64_t *)d;
    else if (nm == "sell_off") S.sell_off = (const int64_t *)d;
    else if (nm == "sell_w") S.sell_w = (const int32_t *)d;
    else if (nm == "sell_col") S.sell_col = (const int32_t *)d;
    else if (nm == "sell_val") S.sell_val[term++] = (const int64_t *)d;
    else if (nm == "ldiag") S.ldiag = (const int64_t *)d;
    else if (nm == "udiag") S.udiag = (const int64_t *)d;
    else if (nm == "lptr") S.lptr = (const int64_t *)d;
    else if (nm == "uptr") S.uptr = (const int64_t *)d;
    else if (nm == "lcol") S.lcol = (const int32_t *)d;
    else if (nm == "ucol") S.ucol = (const int32_t *)d;
    else if (nm == "lval") S.lval = (const int64_t *)d;
    else if (nm == "uval") S.uval = (const int64_t *)d;
    else if (nm == "lvalf") S.lvalf = (const double *)d;
    else if (nm == "uvalf") S.uvalf = (const double *)d;
    else if (nm == "flev_ptr") S.flev_ptr = (const int32_t *)d;
    else if (nm == "flev_rows") S.flev_rows = (const int32_t *)d;
    else if (nm == "blev_ptr") S.blev_ptr = (const int32_t *)d;
    else if (nm == "blev_rows") S.blev_rows = (const int32_t *)d;
    else if (nm == "zbuf") S.zbuf = (int64_t *)d;
    else if (nm == "wbuf") S.wbuf = (int64_t *)d;
    else if (nm == "fbuf") S.fbuf = (double *)d;
    else if (nm == "lev_cnt") S.lev_cnt = (unsigned *)d;
    else if (nm == "V") S.V = (int64_t *)d;
    else if (nm == "x") S.x = (double *)d;
    else if (nm == "words") S.words = (unsigned long long *)d;
  });
}

size_t image_bytes(const HostSystem &hs) {
  size_t total = 0;
  bool work = false;
  walk_region(hs, true, [&](const char *name, size_t bytes) {
    work = work || is_work_array(name) || (hs.device_setup && is_value_array(name));
    if (!work) total += align_up(bytes);
  });
  return total;
}

void build_image(const HostSystem &hs, char *img, const double *x0) {
  size_t off = 0;
  int term = 0;
  bool work = false;
  walk_region(hs, true, [&](const char *name, size_t bytes) {
    work = work || is_work_array(name) || (hs.device_setup && is_value_array(name));
    if (work) return;
    char *d = img + off;
    const size_t span = align_up(bytes);
    off += span;
    const std::string nm(name);
    if (nm == "x" && x0) {
      memcpy(d, x0, bytes);
      memset(d + bytes, 0, span - bytes);
      return;
    }
    const void *src = array_source(hs, name, term);
    if (src && bytes) memcpy(d, src, bytes);
    memset(d + (src ? bytes : 0), 0, src ? span - bytes : span);
  });
}

hipError_t place_system(const HostSystem &hs, char *base, bool own_x, hipStream_t st, BatchSys &S) {
  record_for(hs, own_x, base, S);
  size_t off = 0;
  int term = 0;
  hipError_t err = hipSuccess;
  walk_region(hs, own_x, [&](const char *name, size_t bytes) {
    char *d = base + off;
    off += align_up(bytes);
    if (err != hipSuccess || is_work_array(name) || !bytes) return;
    const std::string nm(name);
    if (nm == "x") return;  // the caller's
    if (nm == "words") {
      // cleared by a copy (a copy engine rather than a fill kernel)
      static const std::vector<unsigned long long> zeros((size_t)kTeamSlots * kTeamWords, 0ull);
      err = hipMemcpyAsync(d, zeros.data(), bytes, hipMemcpyHostToDevice, st);
      return;
    }
    const void *src = array_source(hs, name, term);
    if (src) err = hipMemcpyAsync(d, src, bytes, hipMemcpyHostToDevice, st);
  });
  return err;
}

}  // namespace igm

struct igm_batch {
  int device = 0;
  hipStream_t stream = nullptr;
  igm_policy pol{};
  int32_t nsys = 0;
  std::vector<int64_t> n, nnz, x_off;
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
  double *d_x = nullptr;      // solution buffer of igm_batch_solve and the autotuner
  double *x_bound = nullptr;  // solution vector the uploaded records point into
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

double ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

template <class T>
igm_status dev_alloc(igm_batch *bt, T *&p, size_t count) {
  const size_t bytes = sizeof(T) * std::max<size_t>(count, 1);
  void *q = nullptr;
  if (hipMalloc(&q, bytes) != hipSuccess) return IGM_ERR_OOM;
  bt->bufs.push_back(q);
  bt->device_bytes += (int64_t)bytes;
  p = (T *)q;
  return IGM_OK;
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
  const void *k = batch_kernel(block, rows);
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
  for (int32_t s = 0; s < bt->nsys; ++s) {
    bt->sys[s].team = team[s];
    bt->sys[s].sweep_threads = sweep_threads(block, team[s], bt->sys[s].max_level);
  }
  bt->x_bound = nullptr;  // records are re-uploaded before the next solve
  BT_HIP(hipMemcpy(bt->d_jobs, jobs.data(), sizeof(int32_t) * jobs.size(), hipMemcpyHostToDevice));
  bt->team = team;
  bt->njobs = (int32_t)njobs;
  bt->grid = (int)std::min<int64_t>(cap, njobs);
  bt->block = block;
  bt->rows = rows;
  return IGM_OK;
}

igm_status run(igm_batch *bt, double *x_dev) {
  TraceRange trace_run("igm batch solve");
  auto t0 = std::chrono::steady_clock::now();
  if (bt->x_bound != x_dev) {  // point the records at this solution vector
    for (int32_t s = 0; s < bt->nsys; ++s) bt->sys[s].x = x_dev + bt->x_off[s];
    BT_HIP(hipMemcpyAsync(bt->d_sys, bt->sys.data(), sizeof(BatchSys) * bt->nsys, hipMemcpyHostToDevice,
                          bt->stream));
    bt->x_bound = x_dev;
  }
  BT_HIP(hipMemsetAsync(bt->d_ctl, 0, 2 * sizeof(int32_t), bt->stream));
  for (int32_t s = 0; s < bt->nsys; ++s)
    BT_HIP(hipMemsetAsync(bt->sys[s].words, 0, sizeof(unsigned long long) * kTeamSlots * kTeamWords, bt->stream));
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
  a.phase_clock = bt->pol.phase_clock;
  a.queue = bt->d_ctl;
  a.timeout = bt->d_ctl + 1;
  a.ring = 0;
  void *args[] = {(void *)&a};
  const void *k = batch_kernel(bt->block, bt->rows);
  BT_HIP(hipEventRecord(bt->ev0, bt->stream));
  BT_HIP(hipLaunchCooperativeKernel(k, dim3(bt->grid), dim3(bt->block), args, batch_smem_bytes(bt->pol.m),
                                    bt->stream));
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
  // offsets of each system in the caller's arrays
  std::vector<int64_t> rp_off(ns), nz_off(ns), b_off(ns);
  int64_t trp = 0, tnz = 0, tb = 0;
  for (int32_t s = 0; s < ns; ++s) {
    if (n[s] < 1 || n[s] >= ((int64_t)1 << 31)) { if (failed) *failed = s; return IGM_ERR_ARG; }
    rp_off[s] = trp;
    nz_off[s] = tnz;
    b_off[s] = tb;
    const int64_t nz = row_ptr[trp + n[s]];
    if (nz < 0) { if (failed) *failed = s; return IGM_ERR_ARG; }
    trp += n[s] + 1;
    tnz += nz;
    tb += n[s];
  }
  // validation and host setup of every system, in parallel
  std::vector<HostSystem> hs(ns);
  std::vector<igm_status> sst(ns, IGM_OK);
  std::atomic<int32_t> next(0);
  auto worker = [&] {
    for (;;) {
      const int32_t s = next.fetch_add(1);
      if (s >= ns) break;
      sst[s] = prepare_system(n[s], row_ptr + rp_off[s], col + nz_off[s], val + nz_off[s], b + b_off[s], bt->pol,
                              hs[s]);
    }
  };
  const unsigned hw = std::max(1u, std::min(16u, std::thread::hardware_concurrency()));
  std::vector<std::thread> pool;
  for (unsigned t = 1; t < std::min<unsigned>(hw, (unsigned)ns); ++t) pool.emplace_back(worker);
  worker();
  for (auto &t : pool) t.join();
  for (int32_t s = 0; s < ns; ++s)
    if (sst[s] != IGM_OK) { if (failed) *failed = s; return sst[s]; }
  // one allocation holds every system's region
  std::vector<size_t> roff(ns);
  size_t total = 0;
  for (int32_t s = 0; s < ns; ++s) {
    roff[s] = total;
    total += system_bytes(hs[s], false);
  }
  char *d_all = nullptr;
  BT_TRY(dev_alloc(bt, d_all, total));
  bt->n.resize(ns);
  bt->nnz.resize(ns);
  bt->nterms.resize(ns);
  bt->x_off.resize(ns);
  bt->sys.resize(ns);
  bt->res.resize(ns);
  int64_t xo = 0;
  for (int32_t s = 0; s < ns; ++s) {
    BT_HIP(place_system(hs[s], d_all + roff[s], false, bt->stream, bt->sys[s]));
    bt->n[s] = hs[s].n;
    bt->nnz[s] = hs[s].nnz;
    bt->nterms[s] = hs[s].nterms;
    bt->x_off[s] = xo;
    xo += hs[s].n;
  }
  bt->total_n = xo;
  bt->total_nnz = tnz;
  BT_TRY(dev_alloc(bt, bt->d_x, (size_t)bt->total_n));
  BT_TRY(dev_alloc(bt, bt->d_sys, (size_t)ns));
  BT_TRY(dev_alloc(bt, bt->d_jobs, (size_t)ns * kTeamMax * 2));
  BT_TRY(dev_alloc(bt, bt->d_ctl, 2));
  BT_TRY(dev_alloc(bt, bt->d_res, (size_t)ns));
  for (int32_t s = 0; s < ns; ++s) bt->sys[s].res = bt->d_res + s;
  BT_HIP(hipStreamSynchronize(bt->stream));  // the host vectors die here
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
  if (pol->m > kMaxBatchM) return IGM_ERR_UNSUPPORTED;
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
  out->shift_retries = r.shift_retries;
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
