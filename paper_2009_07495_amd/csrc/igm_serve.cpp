// Served solver (C ABI): continuous batching of solve requests on one
// persistent kernel.
//
// Request life: submit (inputs copied) -> a setup thread validates it, runs
// the host setup and writes the data part of the request's device region
// (inputs, setup products, x0, zeroed exchange words) into a staging area of
// pinned host memory -> the driver thread admits it when a slot, a device
// region for its whole footprint and enough idle workgroups for its team are
// free (first-fit over the pool; requests behind one that does not fit may
// pass it), writes the slot's record (pinned), appends the team's jobs to the
// ring (pinned) and publishes them -> the persistent kernel's workgroups claim
// them, copy the staged data into the region, solve, copy x back into the
// staging area and write the result -> the first member stores the request's
// sequence number in the slot's done flag (pinned) -> the driver takes x and
// the result and frees the slot, the region and the staging space.
//
// While the kernel is resident the server makes no copy or memset call: the
// runtime performs some of those with kernels of its own on other queues,
// which need not make progress next to a kernel that holds the device.
// Admitting a request only when its team fits in the idle workgroups means
// every admitted team starts at once; no member ever waits for a workgroup
// that is busy with another request.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "igm_batch.hpp"
#include "igm_par.hpp"
#include "igm_trace.hpp"
#include "igm_team.hpp"

using namespace igm;

namespace {

using Clock = std::chrono::steady_clock;

constexpr int32_t kRing = 1 << 20;       // job ring capacity (pairs)
constexpr size_t kRegionAlign = 4096;
// records are first built against this made-up base, then moved to the region
constexpr uintptr_t kFakeBase = (uintptr_t)1 << 44;

double ms_between(Clock::time_point a, Clock::time_point b) {
  return std::chrono::duration<double, std::milli>(b - a).count();
}

size_t round_region(size_t b) { return (b + kRegionAlign - 1) / kRegionAlign * kRegionAlign; }

// First-fit allocator over an address range.
class Pool {
 public:
  size_t capacity = 0, used = 0, peak = 0;
  void init(size_t cap) {
    capacity = cap;
    free_.clear();
    free_[0] = cap;
  }
  bool alloc(size_t bytes, size_t &off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < bytes) continue;
      off = it->first;
      const size_t rest = it->second - bytes;
      free_.erase(it);
      if (rest) free_[off + bytes] = rest;
      used += bytes;
      peak = std::max(peak, used);
      return true;
    }
    return false;
  }
  void release(size_t off, size_t bytes) {
    used -= bytes;
    auto it = free_.emplace(off, bytes).first;
    auto nx = std::next(it);
    if (nx != free_.end() && it->first + it->second == nx->first) {
      it->second += nx->second;
      free_.erase(nx);
    }
    if (it != free_.begin()) {
      auto pv = std::prev(it);
      if (pv->first + pv->second == it->first) {
        pv->second += it->second;
        free_.erase(it);
      }
    }
  }

 private:
  std::map<size_t, size_t> free_;
};

struct Request {
  int64_t ticket = 0;
  int64_t n = 0, nnz = 0;
  igm_policy pol{};
  hvec<int64_t> rp;
  hvec<int32_t> col;
  hvec<double> val, b, x0;
  BatchSys rec{};  // record against kFakeBase
  size_t bytes = 0;  // device region
  size_t img = 0;    // staged data part
  size_t stage_off = 0, x_off = 0, region = 0;
  bool staged = false;
  int32_t team = 0, slot = -1, seq = 0;
  int state = 0;  // 0 submitted, 1 prepared, 2 resident, 3 finished
  igm_status status = IGM_OK;
  BatchResult res{};
  std::vector<double> x;
  Clock::time_point t_submit, t_prepared, t_admitted, t_done;
};

}  // namespace

struct igm_server {
  int device = 0;
  hipStream_t kstream = nullptr;
  int block = 0, rows = 0, grid = 0, max_slots = 0;
  bool host_setup = false;  // config: every request's whole setup on the host
  char *d_pool = nullptr;
  Pool pool, stage;
  unsigned long long *d_arrive = nullptr;  // per slot, monotonic
  std::vector<int64_t> arrive_base;
  int32_t *d_ctl = nullptr;  // [0] claim counter, [1] timeout flag
  // pinned host memory (h_*) and the device addresses of the same bytes (dh_*)
  char *h_stage = nullptr, *dh_stage = nullptr;
  BatchSys *h_recs = nullptr, *dh_recs = nullptr;
  BatchResult *h_res = nullptr, *dh_res = nullptr;
  int32_t *h_jobs = nullptr, *dh_jobs = nullptr;
  int32_t *h_stop = nullptr, *dh_stop = nullptr;
  int32_t *h_done = nullptr, *dh_done = nullptr;
  int64_t *h_published = nullptr, *dh_published = nullptr;
  int64_t published = 0;
  int32_t next_seq = 1;
  int busy_wg = 0;
  double wall_us_per_tick = 0.0;
  bool kernel_alive = false;
  // shared state
  std::mutex mu;
  std::condition_variable cv_setup, cv_done, cv_stage;
  std::deque<Request *> to_prepare, prepared;
  std::map<int64_t, std::unique_ptr<Request>> requests;
  std::vector<Request *> slot_req;
  std::vector<int32_t> free_slots;
  int64_t next_ticket = 0, submitted = 0, completed = 0;
  bool stopping = false, drained = false;
  std::vector<std::thread> setup_pool;
  std::thread driver;
};

namespace {

void finish(igm_server *sv, Request *r, igm_status st) {
  // caller holds sv->mu
  if (r->staged) {
    sv->stage.release(r->stage_off, r->img);
    r->staged = false;
    sv->cv_stage.notify_all();
  }
  r->status = st;
  r->state = 3;
  r->t_done = Clock::now();
  sv->completed += 1;
  sv->cv_done.notify_all();
}

template <class T>
T *rebase(T *p, char *base) {
  return p ? (T *)((const char *)p - kFakeBase + (uintptr_t)base) : nullptr;
}

void setup_worker(igm_server *sv) {
  for (;;) {
    Request *r = nullptr;
    {
      std::unique_lock<std::mutex> lk(sv->mu);
      sv->cv_setup.wait(lk, [&] { return sv->drained || !sv->to_prepare.empty(); });
      if (sv->to_prepare.empty()) return;
      r = sv->to_prepare.front();
      sv->to_prepare.pop_front();
    }
    TraceRange trace_setup("igm request setup");
    HostSystem hs;
    igm_status st =
        prepare_system(r->n, r->rp.data(), r->col.data(), r->val.data(), r->b.data(), r->pol, hs, !sv->host_setup);
    hvec<int64_t>().swap(r->rp);
    hvec<int32_t>().swap(r->col);
    hvec<double>().swap(r->val);
    hvec<double>().swap(r->b);
    if (st == IGM_OK) {
      r->bytes = round_region(system_bytes(hs, true));
      r->img = round_region(image_bytes(hs));
      const int64_t per = (int64_t)sv->block * sv->rows;
      const int64_t team = (r->n + per - 1) / per;
      if (r->bytes > sv->pool.capacity || r->img > sv->stage.capacity || team > kTeamMax || team > sv->grid)
        st = IGM_ERR_UNSUPPORTED;
      r->team = (int32_t)team;
    }
    if (st == IGM_OK) {  // staging space; waits while the area is full
      std::unique_lock<std::mutex> lk(sv->mu);
      size_t off = 0;
      sv->cv_stage.wait(lk, [&] { return sv->drained || sv->stage.alloc(r->img, off); });
      if (sv->drained && !sv->stage.alloc(r->img, off)) {
        st = IGM_ERR_DEVICE;  // shutting down with the area full
      } else {
        r->stage_off = off;
        r->staged = true;
      }
    }
    if (st == IGM_OK) {
      build_image(hs, sv->h_stage + r->stage_off, r->x0.empty() ? nullptr : r->x0.data());
      record_for(hs, true, (char *)kFakeBase, r->rec);
      r->x_off = (size_t)((const char *)r->rec.x - (const char *)kFakeBase);
      hvec<double>().swap(r->x0);
    }
    std::lock_guard<std::mutex> lk(sv->mu);
    r->t_prepared = Clock::now();
    if (st != IGM_OK) {
      finish(sv, r, st);
    } else {
      r->state = 1;
      sv->prepared.push_back(r);
    }
  }
}

// Writes the slot's record and publishes the team's jobs (caller holds sv->mu).
void publish(igm_server *sv, Request *r) {
  char *base = sv->d_pool + r->region;
  BatchSys S = r->rec;
  S.row_ptr = rebase(S.row_ptr, base);
  S.col = rebase(S.col, base);
  S.diag_pos = rebase(S.diag_pos, base);
  S.a = rebase(S.a, base);
  S.ahat = rebase(S.ahat, base);
  S.b = rebase(S.b, base);
  S.bhat = rebase(S.bhat, base);
  S.cscale = rebase(S.cscale, base);
  S.sell_off = rebase(S.sell_off, base);
  S.sell_w = rebase(S.sell_w, base);
  S.sell_col = rebase(S.sell_col, base);
  for (int l = 0; l < kMaxTerms; ++l) S.sell_val[l] = rebase(S.sell_val[l], base);
  S.ldiag = rebase(S.ldiag, base);
  S.udiag = rebase(S.udiag, base);
  S.lptr = rebase(S.lptr, base);
  S.uptr = rebase(S.uptr, base);
  S.lcol = rebase(S.lcol, base);
  S.ucol = rebase(S.ucol, base);
  S.lval = rebase(S.lval, base);
  S.uval = rebase(S.uval, base);
  S.lvalf = rebase(S.lvalf, base);
  S.uvalf = rebase(S.uvalf, base);
  S.flev_ptr = rebase(S.flev_ptr, base);
  S.flev_rows = rebase(S.flev_rows, base);
  S.blev_ptr = rebase(S.blev_ptr, base);
  S.blev_rows = rebase(S.blev_rows, base);
  S.V = rebase(S.V, base);
  S.zbuf = rebase(S.zbuf, base);
  S.wbuf = rebase(S.wbuf, base);
  S.fbuf = rebase(S.fbuf, base);
  S.lev_cnt = rebase(S.lev_cnt, base);
  S.x = rebase(S.x, base);
  S.words = rebase(S.words, base);
  S.team = r->team;
  S.sweep_threads = sweep_threads(sv->block, r->team, S.max_level);
  S.seq = r->seq;
  S.res = sv->dh_res + r->slot;
  S.src = sv->dh_stage + r->stage_off;
  S.dst = base;
  S.up_bytes = (int64_t)r->img;
  S.x_out = (double *)(sv->dh_stage + r->stage_off + r->x_off);
  S.arrive = sv->d_arrive + r->slot;
  sv->arrive_base[r->slot] += r->team;
  S.arrive_target = sv->arrive_base[r->slot];
  memcpy(sv->h_recs + r->slot, &S, sizeof(S));
  for (int32_t q = 0; q < r->team; ++q) {
    const int64_t e = 2 * ((sv->published + q) % kRing);
    sv->h_jobs[e] = r->slot;
    sv->h_jobs[e + 1] = q;
  }
  sv->published += r->team;
  std::atomic_thread_fence(std::memory_order_release);
  __atomic_store_n(sv->h_published, sv->published, __ATOMIC_RELEASE);
}

void driver_loop(igm_server *sv) {
  auto last_health = Clock::now();
  for (;;) {
    bool progress = false;
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      // completions
      for (int32_t slot = 0; slot < sv->max_slots; ++slot) {
        Request *r = sv->slot_req[slot];
        if (!r || __atomic_load_n(sv->h_done + slot, __ATOMIC_ACQUIRE) != r->seq) continue;
        memcpy(&r->res, sv->h_res + slot, sizeof(BatchResult));
        r->x.resize((size_t)r->n);
        memcpy(r->x.data(), sv->h_stage + r->stage_off + r->x_off, sizeof(double) * r->n);
        sv->pool.release(r->region, r->bytes);
        sv->busy_wg -= r->team;
        sv->slot_req[slot] = nullptr;
        sv->free_slots.push_back(slot);
        finish(sv, r, (igm_status)r->res.status);
        progress = true;
      }
      // admissions: among the first waiting requests, in arrival order, those that fit
      if (sv->kernel_alive) {
        int looked = 0;
        for (auto it = sv->prepared.begin(); it != sv->prepared.end() && looked < 16;) {
          Request *c = *it;
          ++looked;
          size_t off = 0;
          if (sv->free_slots.empty() || sv->busy_wg + c->team > sv->grid || !sv->pool.alloc(c->bytes, off)) {
            ++it;
            continue;
          }
          c->region = off;
          c->slot = sv->free_slots.back();
          sv->free_slots.pop_back();
          c->seq = sv->next_seq++;
          if (sv->next_seq == INT32_MAX) sv->next_seq = 1;
          sv->busy_wg += c->team;
          c->t_admitted = Clock::now();
          c->state = 2;
          sv->slot_req[c->slot] = c;
          publish(sv, c);
          it = sv->prepared.erase(it);
          progress = true;
        }
      }
    }
    // health of the persistent kernel
    const auto now = Clock::now();
    if (ms_between(last_health, now) > 2.0) {
      last_health = now;
      const bool running = hipStreamQuery(sv->kstream) == hipErrorNotReady;
      std::lock_guard<std::mutex> lk(sv->mu);
      if (sv->kernel_alive && !running) {
        sv->kernel_alive = false;  // it ended before the host stopped it (a failure): fail what it held
        for (int32_t slot = 0; slot < sv->max_slots; ++slot) {
          Request *r = sv->slot_req[slot];
          if (!r) continue;
          sv->slot_req[slot] = nullptr;
          finish(sv, r, IGM_ERR_DEVICE);
        }
      }
    }
    {
      // without the kernel nothing prepared can run: fail it as it arrives
      // (setup threads may still hand over requests submitted before the end)
      std::lock_guard<std::mutex> lk(sv->mu);
      if (!sv->kernel_alive && !sv->prepared.empty()) {
        for (Request *r : sv->prepared) finish(sv, r, IGM_ERR_DEVICE);
        sv->prepared.clear();
        progress = true;
      }
    }
    {
      std::lock_guard<std::mutex> lk(sv->mu);
      if (sv->stopping && sv->drained) break;
    }
    if (!progress) std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
}

igm_status launch(igm_server *sv) {
  BatchArgs a;
  memset(&a, 0, sizeof(a));
  a.sys = sv->dh_recs;
  a.phase_clock = 0;
  a.queue = sv->d_ctl;
  a.timeout = sv->d_ctl + 1;
  a.host_jobs = sv->dh_jobs;
  a.host_published = sv->dh_published;
  a.host_stop = sv->dh_stop;
  a.host_done = sv->dh_done;
  a.ring = kRing;
  void *args[] = {(void *)&a};
  const void *k = serve_kernel(sv->block, sv->rows);
  // an ordinary launch: the grid fits on the device at once, and admission
  // never gives a team more workgroups than are idle
  if (hipLaunchKernel(k, dim3(sv->grid), dim3(sv->block), args, batch_smem_bytes(kMaxBatchM), sv->kstream) !=
      hipSuccess)
    return IGM_ERR_DEVICE;
  sv->kernel_alive = true;
  return IGM_OK;
}

template <class T>
bool host_block(T *&h, T *&d, size_t count) {
  const size_t bytes = sizeof(T) * std::max<size_t>(count, 1);
  if (hipHostMalloc((void **)&h, bytes, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) return false;
  memset((void *)h, 0, bytes);
  return hipHostGetDevicePointer((void **)&d, h, 0) == hipSuccess;
}

void release_all(igm_server *sv) {
  if (sv->d_pool) (void)hipFree(sv->d_pool);
  if (sv->d_arrive) (void)hipFree(sv->d_arrive);
  if (sv->d_ctl) (void)hipFree(sv->d_ctl);
  void *hosts[] = {sv->h_stage, sv->h_recs, sv->h_res, sv->h_jobs, sv->h_stop, sv->h_done, sv->h_published};
  for (void *h : hosts)
    if (h) (void)hipHostFree(h);
  if (sv->kstream) (void)hipStreamDestroy(sv->kstream);
}

void fill_stats(const igm_server *sv, const Request *r, igm_stats *out) {
  memset(out, 0, sizeof(*out));
  out->struct_size = sizeof(igm_stats);
  out->status = r->status;
  out->refinements = r->res.refinements;
  out->iterations = r->res.iterations;
  out->first_ovf = r->res.first_ovf;
  out->shift_retries = r->res.shift_retries;
  out->relres_orig = r->res.relres_orig;
  out->relres_scaled = r->res.relres_scaled;
  out->time_solve_ms = ms_between(r->t_submit, r->t_done);
  out->time_setup_ms = ms_between(r->t_submit, r->t_prepared);
  out->time_cycle_ms = r->slot >= 0 ? ms_between(r->t_admitted, r->t_done) : 0.0;
  out->time_kernel_ms = r->res.t_end >= r->res.t_begin
                            ? (double)(r->res.t_end - r->res.t_begin) * sv->wall_us_per_tick / 1000.0
                            : 0.0;
  out->n = r->n;
  out->nnz = r->nnz;
  out->grid_blocks = r->team;
  out->block_threads = sv->block;
  out->rows_per_thread = sv->rows;
}

}  // namespace

extern "C" {

igm_status igm_server_create(const igm_server_config *cfg, igm_server **out) {
  if (!out) return IGM_ERR_ARG;
  *out = nullptr;
  igm_server_config c;
  memset(&c, 0, sizeof(c));
  if (cfg) {
    if (cfg->struct_size != (int32_t)sizeof(igm_server_config)) return IGM_ERR_ARG;
    c = *cfg;
  }
  if (c.block == 0 && c.rows_per_thread == 0) {  // 8192 rows per workgroup: 1M rows fit in 128
    c.block = 512;
    c.rows_per_thread = 16;
  }
  if (!serve_kernel(c.block, c.rows_per_thread)) return IGM_ERR_UNSUPPORTED;
  if (c.max_slots == 0) c.max_slots = 256;
  if (c.setup_threads == 0) c.setup_threads = 8;
  if (c.pool_bytes == 0) c.pool_bytes = (int64_t)16 << 30;
  if (c.stage_bytes == 0) c.stage_bytes = (int64_t)4 << 30;
  if (c.reserve_cus == 0) c.reserve_cus = 8;
  if (c.reserve_cus < 0) c.reserve_cus = 0;
  if (c.max_slots < 1 || c.max_slots > 65536 || c.setup_threads < 1 || c.setup_threads > 64 || c.pool_bytes < 0 ||
      c.stage_bytes < 0 || c.host_setup < 0 || c.host_setup > 1)
    return IGM_ERR_ARG;
  igm_server *sv = new (std::nothrow) igm_server();
  if (!sv) return IGM_ERR_OOM;
  sv->block = c.block;
  sv->rows = c.rows_per_thread;
  sv->max_slots = c.max_slots;
  sv->host_setup = c.host_setup != 0;
  igm_status st = IGM_OK;
  hipDeviceProp_t prop;
  int nb = 0, wall_khz = 0;
  if (hipGetDevice(&sv->device) != hipSuccess || hipGetDeviceProperties(&prop, sv->device) != hipSuccess ||
      hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, sv->device) != hipSuccess ||
      hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, serve_kernel(sv->block, sv->rows), sv->block,
                                                   batch_smem_bytes(kMaxBatchM)) != hipSuccess ||
      hipStreamCreateWithFlags(&sv->kstream, hipStreamNonBlocking) != hipSuccess)
    st = IGM_ERR_DEVICE;
  sv->wall_us_per_tick = wall_khz > 0 ? 1000.0 / wall_khz : 0.0;
  // the persistent kernel holds its compute units for its whole life; a few
  // stay free for other kernels (the runtime's own, the application's)
  sv->grid = nb * std::max(0, prop.multiProcessorCount - c.reserve_cus);
  if (st == IGM_OK && sv->grid < 1) st = IGM_ERR_UNSUPPORTED;
  if (st == IGM_OK && (hipMalloc((void **)&sv->d_pool, (size_t)c.pool_bytes) != hipSuccess ||
                       hipMalloc((void **)&sv->d_arrive, sizeof(unsigned long long) * sv->max_slots) != hipSuccess ||
                       hipMalloc((void **)&sv->d_ctl, 2 * sizeof(int32_t)) != hipSuccess))
    st = IGM_ERR_OOM;
  if (st == IGM_OK && (!host_block(sv->h_stage, sv->dh_stage, (size_t)c.stage_bytes) ||
                       !host_block(sv->h_recs, sv->dh_recs, (size_t)sv->max_slots) ||
                       !host_block(sv->h_res, sv->dh_res, (size_t)sv->max_slots) ||
                       !host_block(sv->h_jobs, sv->dh_jobs, 2 * (size_t)kRing) ||
                       !host_block(sv->h_published, sv->dh_published, 1) ||
                       !host_block(sv->h_stop, sv->dh_stop, 1) ||
                       !host_block(sv->h_done, sv->dh_done, (size_t)sv->max_slots)))
    st = IGM_ERR_OOM;
  // counters start at zero, before the kernel starts
  if (st == IGM_OK && (hipMemset(sv->d_ctl, 0, 2 * sizeof(int32_t)) != hipSuccess ||
                       hipMemset(sv->d_arrive, 0, sizeof(unsigned long long) * sv->max_slots) != hipSuccess ||
                       hipDeviceSynchronize() != hipSuccess))
    st = IGM_ERR_DEVICE;
  if (st == IGM_OK) st = launch(sv);
  if (st != IGM_OK) {
    if (sv->kernel_alive) {
      __atomic_store_n(sv->h_stop, 1, __ATOMIC_RELEASE);
      (void)hipStreamSynchronize(sv->kstream);
    }
    release_all(sv);
    delete sv;
    return st;
  }
  sv->pool.init((size_t)c.pool_bytes);
  sv->stage.init((size_t)c.stage_bytes);
  sv->arrive_base.assign(sv->max_slots, 0);
  sv->slot_req.assign(sv->max_slots, nullptr);
  for (int32_t s = sv->max_slots - 1; s >= 0; --s) sv->free_slots.push_back(s);
  for (int t = 0; t < c.setup_threads; ++t) sv->setup_pool.emplace_back(setup_worker, sv);
  sv->driver = std::thread(driver_loop, sv);
  *out = sv;
  return IGM_OK;
}

igm_status igm_server_submit(igm_server *sv, int64_t n, const int64_t *row_ptr, const int32_t *col,
                             const double *val, const double *b, const double *x0, const igm_policy *pol,
                             int64_t *ticket) {
  if (!sv || !ticket || !row_ptr || !col || !val || !b || !pol || n < 1 || n >= ((int64_t)1 << 31))
    return IGM_ERR_ARG;
  if (row_ptr[n] < 0) return IGM_ERR_ARG;
  auto r = std::make_unique<Request>();
  r->t_submit = Clock::now();
  r->res.first_ovf = kNoEvent;
  r->n = n;
  r->nnz = row_ptr[n];
  r->pol = *pol;
  par_assign(r->rp, row_ptr, n + 1);
  par_assign(r->col, col, r->nnz);
  par_assign(r->val, val, r->nnz);
  par_assign(r->b, b, n);
  if (x0) r->x0.assign(x0, x0 + n);
  std::lock_guard<std::mutex> lk(sv->mu);
  if (sv->stopping) return IGM_ERR_ARG;
  if (!sv->kernel_alive) return IGM_ERR_DEVICE;  // the persistent kernel has ended
  r->ticket = sv->next_ticket++;
  *ticket = r->ticket;
  sv->to_prepare.push_back(r.get());
  sv->requests[r->ticket] = std::move(r);
  sv->submitted += 1;
  sv->cv_setup.notify_one();
  return IGM_OK;
}

igm_status igm_server_poll(igm_server *sv, int64_t ticket, int32_t *done, double *x, igm_stats *stats) {
  if (!sv || !done) return IGM_ERR_ARG;
  std::lock_guard<std::mutex> lk(sv->mu);
  auto it = sv->requests.find(ticket);
  if (it == sv->requests.end()) return IGM_ERR_ARG;
  Request *r = it->second.get();
  *done = r->state == 3;
  if (!*done) return IGM_OK;
  if (x && !r->x.empty()) memcpy(x, r->x.data(), sizeof(double) * r->n);
  if (stats) fill_stats(sv, r, stats);
  sv->requests.erase(it);
  return IGM_OK;
}

igm_status igm_server_wait(igm_server *sv, int64_t ticket, double timeout_ms, double *x, igm_stats *stats) {
  if (!sv) return IGM_ERR_ARG;
  {
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->requests.find(ticket);
    if (it == sv->requests.end()) return IGM_ERR_ARG;
    Request *r = it->second.get();
    auto ready = [&] { return r->state == 3; };
    if (timeout_ms < 0) {
      sv->cv_done.wait(lk, ready);
    } else if (!sv->cv_done.wait_for(lk, std::chrono::duration<double, std::milli>(timeout_ms), ready)) {
      return IGM_PENDING;
    }
  }
  int32_t done = 0;
  igm_status st = igm_server_poll(sv, ticket, &done, x, stats);
  return st != IGM_OK ? st : (done ? IGM_OK : IGM_PENDING);
}

igm_status igm_server_get_stats(igm_server *sv, igm_server_stats *out) {
  if (!sv || !out) return IGM_ERR_ARG;
  std::lock_guard<std::mutex> lk(sv->mu);
  memset(out, 0, sizeof(*out));
  out->struct_size = sizeof(igm_server_stats);
  int32_t used = 0;
  for (Request *r : sv->slot_req) used += r != nullptr;
  out->slots_used = used;
  out->submitted = sv->submitted;
  out->completed = sv->completed;
  out->prepared_waiting = (int64_t)sv->prepared.size();
  out->setup_waiting = (int64_t)sv->to_prepare.size();
  out->resident = used;
  out->pool_bytes = (int64_t)sv->pool.capacity;
  out->pool_used = (int64_t)sv->pool.used;
  out->pool_peak = (int64_t)sv->pool.peak;
  out->workgroups = sv->grid;
  out->workgroups_busy = sv->busy_wg;
  out->block_threads = sv->block;
  out->rows_per_thread = sv->rows;
  out->jobs_published = sv->published;
  out->kernel_alive = sv->kernel_alive;
  return IGM_OK;
}

void igm_server_destroy(igm_server *sv, double timeout_ms) {
  if (!sv) return;
  {
    std::unique_lock<std::mutex> lk(sv->mu);
    sv->stopping = true;
    auto idle = [&] {
      if (!sv->to_prepare.empty() || !sv->prepared.empty()) return false;
      for (Request *r : sv->slot_req)
        if (r) return false;
      return true;
    };
    if (timeout_ms < 0) sv->cv_done.wait(lk, idle);
    else sv->cv_done.wait_for(lk, std::chrono::duration<double, std::milli>(timeout_ms), idle);
    sv->drained = true;
    sv->cv_setup.notify_all();
    sv->cv_stage.notify_all();
  }
  // the kernel leaves once no published job is left
  __atomic_store_n(sv->h_stop, 1, __ATOMIC_RELEASE);
  for (auto &t : sv->setup_pool) t.join();
  if (sv->driver.joinable()) sv->driver.join();
  (void)hipStreamSynchronize(sv->kstream);
  release_all(sv);
  delete sv;
}

}  // extern "C"
