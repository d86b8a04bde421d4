// C ABI of the igmres library: system setup and upload, the FP64 refinement
// driver of Fig. 1 around the persistent int-GMRES kernel, statistics, and
// the kernel-level entry points.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <new>

#include "igm_launch.hpp"
#include "igm_par.hpp"
#include "igm_trace.hpp"

using namespace igm;

namespace {

#define IGM_HIP(call)                                  \
  do {                                                 \
    hipError_t e_ = (call);                            \
    if (e_ != hipSuccess) {                            \
      if (s) s->last_error_line = __LINE__;            \
      return IGM_ERR_DEVICE;                           \
    }                                                  \
  } while (0)

#define IGM_TRY(call)                  \
  do {                                 \
    igm_status st_ = (call);           \
    if (st_ != IGM_OK) return st_;     \
  } while (0)

// Layout of the system's pinned host area (doubles): device scalars after the
// latest residual step and after the latest int-GMRES call, the call's state,
// and the constant initial state that every call starts from.
constexpr int kPinResidual = 0, kPinCall = 8, kPinState = 16, kPinInit = 32, kPinDoubles = 64;
static_assert(kScalWords <= 8, "scalar blocks");
static_assert(sizeof(CycleState) <= 16 * sizeof(double), "state blocks");

template <class T>
igm_status dalloc(igm_system *s, T *&p, size_t count) {
  size_t bytes = sizeof(T) * (count ? count : 1);
  void *q = nullptr;
  if (hipMalloc(&q, bytes) != hipSuccess) return IGM_ERR_OOM;
  if (hipMemset(q, 0, bytes) != hipSuccess) { (void)hipFree(q); return IGM_ERR_DEVICE; }
  s->bufs.push_back({q, bytes});
  s->device_bytes += (int64_t)bytes;
  p = (T *)q;
  return IGM_OK;
}

template <class T, class A>
igm_status upload(igm_system *s, T *&p, const std::vector<T, A> &v) {
  IGM_TRY(dalloc(s, p, v.size()));
  if (!v.empty()) IGM_HIP(hipMemcpy(p, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice));
  return IGM_OK;
}

// Device copy of a blocked sweep schedule (the progress words are set by
// alloc_work).
igm_status upload_schedule(igm_system *s, const BlockSchedule &h, BlockSweepArgs &d) {
  d = BlockSweepArgs{};
  d.S = h.S;
  d.nb = h.nb;
  d.narrow = h.narrow ? 1 : 0;
  d.max_levels = h.max_levels;
  d.max_width = h.max_width;
  int32_t *prow = nullptr, *plen = nullptr, *ecode = nullptr, *lvbase = nullptr, *lvoff = nullptr, *wbase = nullptr;
  int64_t *levent = nullptr, *eval = nullptr, *pdiag = nullptr;
  uint64_t *pmag = nullptr;
  int32_t *pshift = nullptr;
  double *evalf = nullptr;
  WaitRec *wrec = nullptr;
  IGM_TRY(upload(s, prow, h.prow));
  IGM_TRY(upload(s, plen, h.plen));
  IGM_TRY(upload(s, levent, h.levent));
  IGM_TRY(upload(s, ecode, h.ecode));
  IGM_TRY(upload(s, eval, h.eval));
  IGM_TRY(upload(s, evalf, h.evalf));
  IGM_TRY(upload(s, pdiag, h.pdiag));
  IGM_TRY(upload(s, pmag, h.pmag));
  IGM_TRY(upload(s, pshift, h.pshift));
  IGM_TRY(upload(s, lvbase, h.lvbase));
  IGM_TRY(upload(s, lvoff, h.lvoff));
  IGM_TRY(upload(s, wbase, h.wbase));
  IGM_TRY(upload(s, wrec, h.wrec));
  d.pad_slot = h.pad_slot;
  d.prow = prow; d.plen = plen; d.ecode = ecode; d.eval = eval; d.evalf = evalf; d.pdiag = pdiag;
  d.lvbase = lvbase; d.lvoff = lvoff; d.levent = levent; d.wbase = wbase; d.wrec = wrec;
  d.pmag = pmag; d.pshift = pshift;
  return IGM_OK;
}

void free_device(igm_system *s) {
  for (auto &b : s->bufs) (void)hipFree(b.p);
  s->bufs.clear();
  s->device_bytes = 0;
  if (s->h_pinned) { (void)hipHostFree(s->h_pinned); s->h_pinned = nullptr; }
}

// Integer matrix terms of refinement k (1, 2, ...): Abar^(k) of eq. (AA)
// holds Abar_0 and the first s(k) correction matrices, s(k) = S = s_terms
// (s_rule 0) or min(S, k - 1) (s_rule 1), at most what the setup built.
int32_t terms_for(const igm_policy &p, int32_t k, int32_t built) {
  const int32_t sk = p.s_rule == 0 ? p.s_terms : std::min(p.s_terms, k - 1);
  return std::min(sk + 1, built);
}

CycleArgs make_args(igm_system *s) {
  CycleArgs a;
  memset(&a, 0, sizeof(a));
  const igm_policy &p = s->pol;
  a.n = s->n;
  a.npad = s->npad;
  a.m = p.m;
  a.df = p.df;
  a.nterms = terms_for(p, 1, s->hs.nterms);
  a.precond = p.precond;
  a.b_dot = p.b_dot; a.b_axpy = p.b_axpy; a.b_norm = p.b_norm;
  a.b_div_num = p.b_div_num; a.b_div_den = p.b_div_den; a.b_rot = p.b_rot; a.b_tmp = p.b_tmp;
  a.b_cs_num = p.b_cs_num; a.b_cs_den = p.b_cs_den;
  a.gtol = p.gtol;
  a.sell_off = s->d_sell_off;
  a.sell_w = s->d_sell_w;
  a.sell_col = s->d_sell_col;
  for (int l = 0; l < kMaxTerms; ++l) {
    a.sell_val[l] = s->d_sell_val[l];
    a.alpha[l] = s->hs.alpha[l];
  }
  a.ldiag = s->d_ldiag; a.udiag = s->d_udiag;
  a.lptr = s->d_lptr; a.uptr = s->d_uptr; a.lcol = s->d_lcol; a.ucol = s->d_ucol;
  a.lval = s->d_lval; a.uval = s->d_uval;
  a.flev_ptr = s->d_flev_ptr; a.flev_rows = s->d_flev_rows;
  a.blev_ptr = s->d_blev_ptr; a.blev_rows = s->d_blev_rows;
  a.nflev = s->hs.flev_ptr.empty() ? 0 : (int32_t)s->hs.flev_ptr.size() - 1;
  a.nblev = s->hs.blev_ptr.empty() ? 0 : (int32_t)s->hs.blev_ptr.size() - 1;
  a.max_level = max_level_rows(s->hs);
  a.flev_host = s->hs.flev_ptr.data();
  a.blev_host = s->hs.blev_ptr.data();
  a.V = s->d_V;
  a.zbuf = s->d_z;
  a.wbuf = s->d_w;
  a.lev_cnt = s->d_levcnt;
  a.sweep_threads = sweep_threads(s->block, s->grid, a.max_level);
  a.bsf = s->bsf;
  a.bsb = s->bsb;
  a.sweep_lanes = s->sweep_lanes;
  a.sweep_lds_off = (int32_t)s->sweep_lds_off;
  a.spmv_lanes = s->spmv_lanes;
  a.spmv_lds_off = (int32_t)s->spmv_lds_off;
  a.crp = s->d_row_ptr;
  a.ccol = s->d_col;
  for (int l = 0; l < kMaxTerms; ++l) a.cval[l] = s->d_cval[l];
  a.H = s->d_H; a.c = s->d_c; a.s = s->d_s; a.g = s->d_g;
  a.state = s->d_state;
  a.sync = s->d_sync;
  a.sync_cap = s->sync_cap;
  a.update = 0;
  a.phase_clock = p.phase_clock;
  a.x = nullptr;
  a.scal = s->d_scal;
  a.cscale = s->d_cscale;
  return a;
}

// Choose the workgroup size B, rows per thread R and number of workgroups G
// of the cycle kernel: the first (B, R) in order of preference for which
// G = ceil(n / (B R)) fits both the target and the co-resident limit. Larger
// workgroups with fewer rows per thread keep the per-thread work of each
// inner product short; fewer workgroups make each grid reduction cheaper.
igm_status choose_launch(igm_system *s) {
  hipDeviceProp_t prop;
  IGM_HIP(hipGetDeviceProperties(&prop, s->device));
  int wall_khz = 0;
  IGM_HIP(hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, s->device));
  s->wall_us_per_tick = wall_khz > 0 ? 1000.0 / wall_khz : 0.0;
  int target = s->pol.grid_blocks > 0 ? s->pol.grid_blocks : 256;
  target = std::min(target, 1023);
  const size_t smem = s->cycle_lds;
  // ILU(0): the sweeps hold a row's structure in registers while they wait,
  // which the 512-thread shapes (256 registers per thread) keep without spills
  static const int kShapes[][2] = {{1024, 1}, {1024, 2}, {1024, 4}, {512, 8}, {512, 16}};
  static const int kShapesIlu[][2] = {{512, 1}, {512, 2}, {512, 4}, {512, 8}, {512, 16}};
  for (const auto &bs : s->pol.precond == IGM_PRE_ILU0 ? kShapesIlu : kShapes) {
    const int B = bs[0], R = bs[1];
    // co-resident workgroups of the kernel that will run (every mapping's
    // kernel when the mapping is measured after this choice)
    int nb = INT32_MAX;
    const bool tune = s->pol.spmv_lanes < 0;
    for (int32_t map : {1, 2, 4}) {
      if (tune ? (map == IGM_SPMV_MERGE && !s->spmv_merge_ok) : map != std::min(s->spmv_lanes, 4)) continue;
      int k = 0;
      IGM_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&k, cycle_kernel(B, R, s->pol.precond, map), B, smem));
      nb = std::min(nb, k);
    }
    const int64_t cap = std::min<int64_t>((int64_t)nb * prop.multiProcessorCount, target);
    const int64_t G = (s->n + (int64_t)B * R - 1) / ((int64_t)B * R);
    if (nb > 0 && G <= cap) {
      s->grid = (int)G;
      s->block = B;
      s->rows_per_thread = R;
      s->max_coresident = nb * prop.multiProcessorCount;
      return IGM_OK;
    }
  }
  return IGM_ERR_UNSUPPORTED;
}

igm_status alloc_work(igm_system *s) {
  const int m = s->pol.m;
  const int64_t np = s->npad;
  int64_t extra = 2;
  if (s->pol.precond == IGM_PRE_ILU0)
    extra += 3;  // barriers around the two sweeps
  const int64_t cap = (int64_t)m * (m + 1) / 2 + (int64_t)m * extra + 16;
  if (cap > (int64_t)1 << 30) return IGM_ERR_UNSUPPORTED;
  s->sync_cap = (int32_t)cap;
  IGM_TRY(dalloc(s, s->d_V, (size_t)(m + 1) * np));
  IGM_TRY(dalloc(s, s->d_z, np));
  IGM_TRY(dalloc(s, s->d_w, np));
  s->d_levcnt = nullptr;
  s->d_prog = nullptr;
  if (s->pol.precond == IGM_PRE_ILU0) {
    IGM_TRY(dalloc(s, s->d_levcnt, ((s->hs.flev_ptr.size() - 1) + (s->hs.blev_ptr.size() - 1)) * kLevStride));
    // the backward schedule's progress words follow the forward ones
    IGM_TRY(dalloc(s, s->d_prog, ((size_t)s->bsf.nb + s->bsb.nb) * kLevStride));
    s->bsf.prog = s->d_prog;
    s->bsb.prog = s->d_prog + (size_t)s->bsf.nb * kLevStride;
  }
  IGM_TRY(dalloc(s, s->d_r, np));
  IGM_TRY(dalloc(s, s->d_rhat, np));
  IGM_TRY(dalloc(s, s->d_bk, np));
  IGM_TRY(dalloc(s, s->d_r0, np));
  IGM_TRY(dalloc(s, s->d_x, np));
  IGM_TRY(dalloc(s, s->d_H, (size_t)(m + 1) * m));
  IGM_TRY(dalloc(s, s->d_c, m));
  IGM_TRY(dalloc(s, s->d_s, m));
  IGM_TRY(dalloc(s, s->d_g, m + 1));
  IGM_TRY(dalloc(s, s->d_state, 1));
  IGM_TRY(dalloc(s, s->d_sync, (size_t)2 * kSyncGroups * cap));
  IGM_TRY(dalloc(s, s->d_red, kRedTotal));
  IGM_TRY(dalloc(s, s->d_scal, kScalWords));
  IGM_TRY(dalloc(s, s->d_parts, kMaxReduceParts + 1));  // partials, then the ticket (zeroed here)
  if (hipHostMalloc((void **)&s->h_pinned, kPinDoubles * sizeof(double)) != hipSuccess) return IGM_ERR_OOM;
  memset(s->h_pinned, 0, kPinDoubles * sizeof(double));
  CycleState *init = (CycleState *)(s->h_pinned + kPinInit);  // constant from here on
  init->first_ovf = kNoEvent;
  return IGM_OK;
}

igm_status device_norm(igm_system *s, const double *x, int64_t len, double *out_dev) {
  IGM_HIP(hipMemsetAsync(s->d_red, 0, sizeof(unsigned long long) * kRedTotal, s->stream));
  IGM_HIP(launch_absmax(s->stream, len, x, s->d_red + kRedMuX));
  IGM_HIP(launch_dnrm_sum(s->stream, len, x, s->d_red + kRedMuX, s->d_red + kRedSumX));
  IGM_HIP(launch_fin_norm(s->stream, s->d_red, out_dev));
  return IGM_OK;
}

// Lanes per row of the integer SpMV and the FP64 residual when the policy
// leaves it open. SELL-64 (one lane per row) loads every slice padded to its
// longest row and walks a row's entries one after another; a group of G lanes
// per row loads no padding and cuts the walk G-fold, but reduces across the
// group and leaves lanes idle on short rows. Measured on stencils (mean row
// lengths 7 and 27, SELL-64 fill above 0.95) one lane per row is fastest by
// 1.5x or more; on heavy-tailed rows (fill 0.08) 16 lanes are fastest, 5x
// ahead of SELL-64. The rule follows the fill.
int32_t auto_spmv_lanes(int64_t n, const int64_t *row_ptr) {
  if (n <= 0) return 1;
  const int64_t nnz = row_ptr[n];
  int64_t padded = 0;
  for (int64_t q = 0; q < n; q += kSlice) {
    int64_t w = 0;
    const int64_t e = std::min<int64_t>(n, q + kSlice);
    for (int64_t i = q; i < e; ++i) w = std::max<int64_t>(w, row_ptr[i + 1] - row_ptr[i]);
    padded += w * kSlice;
  }
  return 2 * nnz >= padded ? IGM_SPMV_SELL : IGM_SPMV_MERGE;
}

// Largest entry count of an aligned window of 1024 rows (every chunk of the
// merge mapping lies inside one).
int64_t max_chunk_entries(int64_t n, const int64_t *row_ptr) {
  int64_t m = 0;
  for (int64_t q = 0; q < n; q += 1024) m = std::max(m, row_ptr[std::min<int64_t>(n, q + 1024)] - row_ptr[q]);
  return m;
}

igm_status tune_spmv_lanes(igm_system *s);

// Everything that depends on the policy or the right-hand side.
igm_status build(igm_system *s) {
  free_device(s);
  IGM_TRY(host_setup(s->n, s->row_ptr, s->col, s->ahat, s->bhat, s->pol, s->hs));
  HostSetup &h = s->hs;
  const bool tune = s->pol.spmv_lanes < 0;
  const bool merge_ok = max_chunk_entries(s->n, s->row_ptr.data()) < ((int64_t)1 << 30);
  s->spmv_lanes = s->pol.spmv_lanes > 0 ? s->pol.spmv_lanes : tune ? 4 : auto_spmv_lanes(s->n, s->row_ptr.data());
  if (s->spmv_lanes == IGM_SPMV_MERGE && !merge_ok) {
    if (s->pol.spmv_lanes == IGM_SPMV_MERGE) return IGM_ERR_UNSUPPORTED;
    s->spmv_lanes = 16;
  }
  s->spmv_merge_ok = merge_ok;
  // ILU(0): the blocked schedules of the two sweeps, sized by the LDS a
  // workgroup of the cycle kernel has left for the block's values
  BlockSchedule sf, sb;
  s->cycle_lds = cycle_smem_bytes(s->pol.m);
  s->spmv_lds_off = 0;
  if (s->spmv_lanes > 1) {  // sized for the largest workgroup and any mapping (measured: all are tried)
    s->spmv_lds_off = (s->cycle_lds + 255) / 256 * 256;
    s->cycle_lds = s->spmv_lds_off + std::max<size_t>((size_t)1024 * sizeof(int64_t), merge_lds_bytes(1024));
  }
  s->bsf = s->bsb = BlockSweepArgs{};
  s->sweep_lanes = 0;
  s->sweep_lds_off = 0;
  if (s->pol.precond == IGM_PRE_ILU0) {
    hipDeviceProp_t prop;
    IGM_HIP(hipGetDeviceProperties(&prop, s->device));
    s->sweep_lds_off = (s->cycle_lds + 255) / 256 * 256;
    const int64_t room = (int64_t)prop.sharedMemPerBlock - (int64_t)s->sweep_lds_off - kCycleStaticLds;
    int64_t S = s->pol.sweep_rows > 0 ? s->pol.sweep_rows : kSweepRowsAuto;
    S = std::min<int64_t>(S, (s->n + 63) / 64 * 64);
    // the largest S (halving from the request) whose values and level tables fit
    for (;;) {
      if (S < 64 || room < (int64_t)sweep_lds_bytes(64, 64)) return IGM_ERR_UNSUPPORTED;
      if ((int64_t)sweep_lds_bytes(S, 0) <= room) {
        block_schedule(s->n, true, (int32_t)S, h.lptr, h.lcol, h.lval, h.ldiag, sf);
        block_schedule(s->n, false, (int32_t)S, h.uptr, h.ucol, h.uval, h.udiag, sb);
        if ((int64_t)sweep_lds_bytes(S, std::max(sf.max_levels, sb.max_levels)) <= room) break;
      }
      S = S / 2 / 64 * 64;
    }
    if (sf.wrec.size() >= ((size_t)1 << 31) || sb.wrec.size() >= ((size_t)1 << 31)) return IGM_ERR_UNSUPPORTED;
    const int32_t ml = std::max(sf.max_levels, sb.max_levels);
    sf.max_levels = sb.max_levels = ml;
    s->cycle_lds = s->sweep_lds_off + sweep_lds_bytes(S, ml);
    s->sweep_lanes = s->pol.sweep_lanes > 0 ? s->pol.sweep_lanes : kSweepLanesAuto;
  }
  // Rows touched by the cycle kernel: every row r < grid * BLOCK * R. The basis,
  // the SELL slices (zero width) and the diagonals (value 1) are padded to that
  // many rows so the kernel needs no per-row bounds test; padded rows stay 0.
  IGM_TRY(choose_launch(s));
  const int64_t touched = (int64_t)s->grid * s->block * s->rows_per_thread;
  s->npad = (std::max(s->n, touched) + kSlice - 1) / kSlice * kSlice;
  {
    const int64_t ns = s->npad / kSlice;
    const int64_t end = h.sell_off.back();
    h.sell_off.resize(ns + 1, end);
    h.sell_w.resize(ns, 0);
    if (s->pol.precond != IGM_PRE_NONE) {
      h.ldiag.resize(s->npad, 1);
      h.udiag.resize(s->npad, 1);
    }
  }
  IGM_TRY(upload(s, s->d_row_ptr, s->row_ptr));
  IGM_TRY(upload(s, s->d_col, s->col));
  IGM_TRY(upload(s, s->d_a, h.a));
  IGM_TRY(upload(s, s->d_ahat, s->ahat));
  IGM_TRY(upload(s, s->d_b, h.b));
  IGM_TRY(upload(s, s->d_bhat, s->bhat));
  s->d_cscale = nullptr;
  if (s->pol.two_sided) IGM_TRY(upload(s, s->d_cscale, h.cscale));
  IGM_TRY(upload(s, s->d_sell_off, h.sell_off));
  IGM_TRY(upload(s, s->d_sell_w, h.sell_w));
  IGM_TRY(upload(s, s->d_sell_col, h.sell_col));
  for (int l = 0; l < kMaxTerms; ++l) s->d_sell_val[l] = s->d_cval[l] = nullptr;
  for (int l = 0; l < h.nterms; ++l) IGM_TRY(upload(s, s->d_sell_val[l], h.sell_val[l]));
  if (s->spmv_lanes > 1)  // the same matrices in CSR order, for the lane groups
    for (int l = 0; l < h.nterms; ++l) IGM_TRY(upload(s, s->d_cval[l], h.abar[l]));
  if (s->pol.precond != IGM_PRE_NONE) {
    IGM_TRY(upload(s, s->d_ldiag, h.ldiag));
    IGM_TRY(upload(s, s->d_udiag, h.udiag));
    IGM_TRY(upload(s, s->d_lptr, h.lptr));
    IGM_TRY(upload(s, s->d_uptr, h.uptr));
    IGM_TRY(upload(s, s->d_lcol, h.lcol));
    IGM_TRY(upload(s, s->d_ucol, h.ucol));
    IGM_TRY(upload(s, s->d_lval, h.lval));
    IGM_TRY(upload(s, s->d_uval, h.uval));
    hvec<double> lf, uf;
    par_assign(lf, h.lval.data(), (int64_t)h.lval.size());
    par_assign(uf, h.uval.data(), (int64_t)h.uval.size());
    IGM_TRY(upload(s, s->d_lvalf, lf));
    IGM_TRY(upload(s, s->d_uvalf, uf));
    IGM_TRY(upload(s, s->d_flev_ptr, h.flev_ptr));
    IGM_TRY(upload(s, s->d_flev_rows, h.flev_rows));
    IGM_TRY(upload(s, s->d_blev_ptr, h.blev_ptr));
    IGM_TRY(upload(s, s->d_blev_rows, h.blev_rows));
    IGM_TRY(upload_schedule(s, sf, s->bsf));
    IGM_TRY(upload_schedule(s, sb, s->bsb));
  } else {
    s->d_ldiag = s->d_udiag = s->d_lptr = s->d_uptr = s->d_lval = s->d_uval = nullptr;
    s->d_lcol = s->d_ucol = nullptr;
    s->d_lvalf = s->d_uvalf = nullptr;
    s->d_flev_ptr = s->d_flev_rows = s->d_blev_ptr = s->d_blev_rows = nullptr;
    h.flev_ptr.clear();
    h.blev_ptr.clear();
  }
  IGM_TRY(alloc_work(s));
  if (tune) IGM_TRY(tune_spmv_lanes(s));
  // norms of the scaled and original right-hand sides (denominators of relres)
  IGM_TRY(device_norm(s, s->d_b, s->n, s->d_scal + kScalNormB));
  IGM_TRY(device_norm(s, s->d_bhat, s->n, s->d_scal + kScalNormBhat));
  IGM_HIP(hipStreamSynchronize(s->stream));
  return IGM_OK;
}

igm_status launch_cycle(igm_system *s, const CycleArgs &a) {
  const void *k = cycle_kernel(s->block, s->rows_per_thread, s->pol.precond, s->spmv_lanes);
  void *args[] = {(void *)&a};
  IGM_HIP(hipLaunchCooperativeKernel(k, dim3(s->grid), dim3(s->block), args, s->cycle_lds, s->stream));
  return IGM_OK;
}

igm_status prepare_cycle(igm_system *s) {
  IGM_HIP(hipMemsetAsync(s->d_sync, 0, sizeof(unsigned long long) * 2 * kSyncGroups * (size_t)s->sync_cap,
                         s->stream));
  IGM_HIP(hipMemcpyAsync(s->d_state, s->h_pinned + kPinInit, sizeof(CycleState), hipMemcpyHostToDevice,
                         s->stream));
  return IGM_OK;
}

// Lanes per row of the FP64 residual: the SpMV's mapping, except that with
// SELL-64 (one thread per row over the CSR arrays, which the residual reads)
// rows of 16 or more entries on average go to groups of 8 lanes, whose loads
// of consecutive entries coalesce (1M-row 27-point matrix: 481 -> 239 us).
// The sums keep the CSR order of each row either way.
static int residual_lanes(const igm_system *s) {
  return s->spmv_lanes == 1 && s->nnz >= 16 * s->n ? 8 : s->spmv_lanes;
}

// The FP64 residual step of a refinement (eq. (b), both norms, relres and
// gamma of eq. (gammak)) for the iterate x, its scalars copied to dst (pinned
// host memory) at the end; everything is enqueued on the system's stream.
igm_status enqueue_residual(igm_system *s, const double *x, double *dst) {
  IGM_HIP(hipMemsetAsync(s->d_red, 0, sizeof(unsigned long long) * kRedTotal, s->stream));
  IGM_HIP(launch_residual(s->stream, s->n, s->d_row_ptr, s->d_col, s->d_a, s->d_ahat, s->d_b, s->d_bhat, x,
                          s->d_cscale, s->d_r, s->d_rhat, s->d_red, residual_lanes(s)));
  IGM_HIP(launch_dnrm_sum(s->stream, s->n, s->d_r, s->d_red + kRedMuR, s->d_red + kRedSumR));
  IGM_HIP(launch_dnrm_sum(s->stream, s->n, s->d_rhat, s->d_red + kRedMuRhat, s->d_red + kRedSumRhat));
  IGM_HIP(launch_fin_residual(s->stream, s->d_red, s->d_scal + kScalNormB, s->d_scal));
  IGM_HIP(hipMemcpyAsync(dst, s->d_scal, sizeof(double) * kScalWords, hipMemcpyDeviceToHost, s->stream));
  return IGM_OK;
}

double ms_since(std::chrono::steady_clock::time_point t0) {
  return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
}

// Two timing events, destroyed with the object.
struct EventPair {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  EventPair() = default;
  EventPair(const EventPair &) = delete;
  EventPair &operator=(const EventPair &) = delete;
  ~EventPair() {
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
  }
};

// igm_policy.spmv_lanes = -1: time the standalone SpMV (all terms, a zero
// vector: the traffic does not depend on the values) with each mapping and keep
// the fastest. The cycle kernel's SpMV reads the same arrays in the same way.
igm_status tune_spmv_lanes(igm_system *s) {
  IGM_HIP(hipMemsetAsync(s->d_V, 0, sizeof(int64_t) * (size_t)s->npad, s->stream));
  EventPair ev;
  IGM_HIP(hipEventCreate(&ev.e0));
  IGM_HIP(hipEventCreate(&ev.e1));
  float best = 0.0f;
  int32_t pick = 1;
  for (int32_t g : {1, 2, 4, 8, 16, 32, 64}) {
    if (g == IGM_SPMV_MERGE && !s->spmv_merge_ok) continue;
    s->spmv_lanes = g;
    const CycleArgs a = make_args(s);
    IGM_HIP(launch_spmv(s->stream, a, s->hs.nterms, s->d_V, s->d_z));
    IGM_HIP(hipEventRecord(ev.e0, s->stream));
    for (int r = 0; r < 5; ++r) IGM_HIP(launch_spmv(s->stream, a, s->hs.nterms, s->d_V, s->d_z));
    IGM_HIP(hipEventRecord(ev.e1, s->stream));
    IGM_HIP(hipEventSynchronize(ev.e1));
    float ms = 0.0f;
    IGM_HIP(hipEventElapsedTime(&ms, ev.e0, ev.e1));
    if (g == 1 || ms < best) best = ms, pick = g;
  }
  s->spmv_lanes = pick;
  return IGM_OK;
}

// Fig. 1 on the device; x is a device vector of n doubles.
igm_status solve_dev(igm_system *s, double *x) {
  TraceRange trace_solve("igm solve");
  auto t0 = std::chrono::steady_clock::now();
  const igm_policy &p = s->pol;
  s->hist_ro.clear(); s->hist_rs.clear(); s->hist_gamma.clear(); s->hist_rho.clear(); s->hist_jstar.clear();
  igm_stats &st = s->stats;
  st.refinements = 0;
  st.iterations = 0;
  st.first_ovf = kNoEvent;
  st.time_cycle_ms = 0.0;
  st.shift_retries = 0;
  igm_status status = IGM_NOT_CONVERGED;
  CycleArgs a = make_args(s);
  a.update = 1;
  a.x = x;
  EventPair ev;  // destroyed on every return path
  IGM_HIP(hipEventCreate(&ev.e0));
  IGM_HIP(hipEventCreate(&ev.e1));
  hipEvent_t e0 = ev.e0, e1 = ev.e1;
  double *res = s->h_pinned + kPinResidual;   // scalars of the latest residual step
  double *after = s->h_pinned + kPinCall;     // scalars after the latest call (rho)
  CycleState *hcs = (CycleState *)(s->h_pinned + kPinState);
  // The first residual step; every later one is enqueued right behind the
  // int-GMRES call that produced its iterate, so a refinement waits for the
  // device once. A call that fails leaves x unchanged, and the residual step
  // behind it then repeats the previous one bit for bit.
  IGM_TRY(enqueue_residual(s, x, res));
  IGM_HIP(hipStreamSynchronize(s->stream));
  for (int k = 0;; ++k) {
    TraceRange trace_refinement("igm refinement");
    // top of refinement k+1: residuals, relres, gamma
    const double gamma = res[kScalGamma], ro = res[kScalRelresOrig], rs = res[kScalRelresScaled];
    s->hist_ro.push_back(ro);
    s->hist_rs.push_back(rs);
    st.relres_orig = ro;
    st.relres_scaled = rs;
    if (!isfinite(ro)) { status = IGM_ERR_RANGE; break; }
    if (ro < p.tol) { status = IGM_OK; break; }
    if (k >= p.max_refine) { status = IGM_NOT_CONVERGED; break; }
    s->hist_gamma.push_back(gamma);
    if (gamma == 0.0) { s->hist_rho.push_back(0.0); status = IGM_OK; break; }
    // FP64 start step and cast of v1, then the int-GMRES call with the fused update
    a.nterms = terms_for(p, k + 1, s->hs.nterms);
    IGM_TRY(prepare_cycle(s));
    IGM_HIP(launch_start_vector(s->stream, a, s->d_r, s->d_scal, s->d_lvalf, s->d_uvalf, s->d_bk, s->d_r0, s->d_red));
    CycleState cs;
    for (;;) {  // the call, repeated from the same v1 while a retry can adjust a shift
      IGM_HIP(hipEventRecord(e0, s->stream));
      {
        TraceRange trace_call("igm int-GMRES call");
        IGM_TRY(launch_cycle(s, a));
      }
      IGM_HIP(hipEventRecord(e1, s->stream));
      IGM_HIP(hipMemcpyAsync(hcs, s->d_state, sizeof(CycleState), hipMemcpyDeviceToHost, s->stream));
      IGM_HIP(hipMemcpyAsync(after, s->d_scal, sizeof(double) * kScalWords, hipMemcpyDeviceToHost, s->stream));
      IGM_TRY(enqueue_residual(s, x, res));  // the next refinement's residual step
      IGM_HIP(hipStreamSynchronize(s->stream));
      cs = *hcs;
      float ms = 0.f;
      IGM_HIP(hipEventElapsedTime(&ms, e0, e1));
      st.time_cycle_ms += ms;
      if (cs.range_err || cs.timeout || cs.first_ovf == kNoEvent || st.shift_retries >= p.shift_retry) break;
      if (!adjust_shifts(s->pol, cs.first_ovf)) break;
      st.shift_retries += 1;
      a = make_args(s);  // the adjusted shifts; v1 (column 0 of V) is untouched by the call
      a.update = 1;
      a.x = x;
      a.nterms = terms_for(p, k + 1, s->hs.nterms);
      IGM_TRY(prepare_cycle(s));
    }
    s->hist_rho.push_back(after[kScalRho]);
    for (int k = 0; k < 8; ++k) st.phase_us[k] = (double)cs.phase[k] * s->wall_us_per_tick;
    if (cs.range_err) { status = IGM_ERR_RANGE; break; }
    if (cs.timeout) { status = IGM_ERR_DEVICE; s->last_error_line = __LINE__; break; }
    st.refinements += 1;
    st.iterations += cs.steps;
    s->hist_jstar.push_back(cs.jstar);
    if (cs.first_ovf != kNoEvent) { st.first_ovf = cs.first_ovf; status = IGM_ERR_OVERFLOW; break; }
    if (cs.jstar == 0) { status = IGM_ERR_BREAKDOWN; break; }
  }
  st.status = status;
  st.time_solve_ms = ms_since(t0);
  return status;
}

void fill_stats_static(igm_system *s) {
  igm_stats &st = s->stats;
  st.struct_size = sizeof(igm_stats);
  st.n = s->n;
  st.nnz = s->nnz;
  st.nterms = s->hs.nterms;
  st.grid_blocks = s->grid;
  st.rows_per_thread = s->rows_per_thread;
  st.block_threads = s->block;
  st.levels_fwd = s->hs.flev_ptr.empty() ? 0 : (int32_t)s->hs.flev_ptr.size() - 1;
  st.levels_bwd = s->hs.blev_ptr.empty() ? 0 : (int32_t)s->hs.blev_ptr.size() - 1;
  st.device_bytes = s->device_bytes;
  st.spmv_lanes = s->spmv_lanes;
  st.sweep_rows = s->bsf.S;
}

}  // namespace

extern "C" {

igm_status igm_policy_preset(int32_t preset, igm_policy *out) {
  if (!out) return IGM_ERR_ARG;
  igm_policy p;
  memset(&p, 0, sizeof(p));
  p.struct_size = sizeof(igm_policy);
  p.df = 30;
  p.s_terms = 0;
  p.m = 30;
  p.max_refine = 2000;
  p.gtol = -1;
  p.tol = 1e-10;
  p.grid_blocks = 0;
  switch (preset) {
    case IGM_PRESET_PAPER_NOPREC:  // Sec. VII-B, Table IV
      p.alpha_a = 16; p.precond = IGM_PRE_NONE;
      p.b_dot = 16; p.b_axpy = 16; p.b_norm = 16; p.b_div_num = 16; p.b_div_den = 14;
      p.b_rot = 16; p.b_tmp = 16; p.b_cs_num = 16; p.b_cs_den = 14;
      break;
    case IGM_PRESET_PAPER_ILU:  // Sec. VII-C, Table VI
    case IGM_PRESET_JACOBI:     // the ILU construction on the diagonal only
      p.alpha_a = 32; p.precond = preset == IGM_PRESET_PAPER_ILU ? IGM_PRE_ILU0 : IGM_PRE_JACOBI;
      p.b_dot = 0; p.b_axpy = 0; p.b_norm = 0; p.b_div_num = 30; p.b_div_den = 0;
      p.b_rot = 0; p.b_tmp = 0; p.b_cs_num = 30; p.b_cs_den = 0;
      break;
    default:
      return IGM_ERR_ARG;
  }
  *out = p;
  return IGM_OK;
}

igm_status igm_create_system(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
                             const double *b, const igm_policy *pol, igm_system **out) {
  if (!out) return IGM_ERR_ARG;
  *out = nullptr;
  if (!pol || pol->struct_size != (int32_t)sizeof(igm_policy)) return IGM_ERR_ARG;
  IGM_TRY(check_policy(*pol));
  IGM_TRY(validate_csr(n, row_ptr, col, val, b));
  auto t0 = std::chrono::steady_clock::now();
  igm_system *s = new (std::nothrow) igm_system();
  if (!s) return IGM_ERR_OOM;
  if (hipGetDevice(&s->device) != hipSuccess) { delete s; return IGM_ERR_DEVICE; }
  s->pol = *pol;
  s->n = n;
  s->nnz = row_ptr[n];
  par_assign(s->row_ptr, row_ptr, n + 1);
  par_assign(s->col, col, s->nnz);
  par_assign(s->ahat, val, s->nnz);
  par_assign(s->bhat, b, n);
  igm_status st = build(s);
  if (st != IGM_OK) {
    free_device(s);
    delete s;
    return st;
  }
  s->stats.time_setup_ms = ms_since(t0);
  fill_stats_static(s);
  *out = s;
  return IGM_OK;
}

igm_status igm_set_policy(igm_system *s, const igm_policy *pol) {
  if (!s || !pol || pol->struct_size != (int32_t)sizeof(igm_policy)) return IGM_ERR_ARG;
  IGM_TRY(check_policy(*pol));
  auto t0 = std::chrono::steady_clock::now();
  igm_policy old = s->pol;
  s->pol = *pol;
  igm_status st = build(s);
  if (st != IGM_OK) {
    s->pol = old;
    igm_status st2 = build(s);
    (void)st2;
    fill_stats_static(s);
    return st;
  }
  s->stats.time_setup_ms = ms_since(t0);
  fill_stats_static(s);
  return IGM_OK;
}

igm_status igm_set_rhs(igm_system *s, const double *b) {
  if (!s || !b) return IGM_ERR_ARG;
  for (int64_t i = 0; i < s->n; ++i)
    if (!isfinite(b[i])) return IGM_ERR_ARG;
  s->bhat.assign(b, b + s->n);
  for (int64_t i = 0; i < s->n; ++i) s->hs.b[i] = s->bhat[i] / s->hs.dhat[i];  // eq. (eq1)
  IGM_HIP(hipMemcpy(s->d_bhat, s->bhat.data(), sizeof(double) * s->n, hipMemcpyHostToDevice));
  IGM_HIP(hipMemcpy(s->d_b, s->hs.b.data(), sizeof(double) * s->n, hipMemcpyHostToDevice));
  IGM_TRY(device_norm(s, s->d_b, s->n, s->d_scal + kScalNormB));
  IGM_TRY(device_norm(s, s->d_bhat, s->n, s->d_scal + kScalNormBhat));
  IGM_HIP(hipStreamSynchronize(s->stream));
  return IGM_OK;
}

igm_status igm_set_stream(igm_system *s, void *hip_stream) {
  if (!s) return IGM_ERR_ARG;
  IGM_HIP(hipStreamSynchronize(s->stream));
  s->stream = (hipStream_t)hip_stream;
  return IGM_OK;
}

igm_status igm_solve_device(igm_system *s, double *x_dev) {
  if (!s || !x_dev) return IGM_ERR_ARG;
  return solve_dev(s, x_dev);
}

igm_status igm_solve(igm_system *s, double *x) {
  if (!s || !x) return IGM_ERR_ARG;
  IGM_HIP(hipMemcpyAsync(s->d_x, x, sizeof(double) * s->n, hipMemcpyHostToDevice, s->stream));
  igm_status st = solve_dev(s, s->d_x);
  if (st == IGM_ERR_DEVICE) return st;
  IGM_HIP(hipMemcpyAsync(x, s->d_x, sizeof(double) * s->n, hipMemcpyDeviceToHost, s->stream));
  IGM_HIP(hipStreamSynchronize(s->stream));
  return st;
}

igm_status igm_get_stats(const igm_system *s, igm_stats *out) {
  if (!s || !out) return IGM_ERR_ARG;
  *out = s->stats;
  out->struct_size = sizeof(igm_stats);
  out->last_error_line = s->last_error_line;
  return IGM_OK;
}

igm_status igm_get_policy(const igm_system *s, igm_policy *out) {
  if (!s || !out) return IGM_ERR_ARG;
  *out = s->pol;
  out->struct_size = sizeof(igm_policy);
  return IGM_OK;
}

igm_status igm_get_history(const igm_system *s, int32_t cap, double *relres_orig, double *relres_scaled,
                           double *gamma, double *rho, int32_t *jstar, int32_t *count) {
  if (!s || cap < 0) return IGM_ERR_ARG;
  int32_t k = std::min<int32_t>(cap, (int32_t)s->hist_ro.size());
  for (int32_t i = 0; i < k; ++i) {
    if (relres_orig) relres_orig[i] = s->hist_ro[i];
    if (relres_scaled) relres_scaled[i] = s->hist_rs[i];
    if (gamma) gamma[i] = i < (int32_t)s->hist_gamma.size() ? s->hist_gamma[i] : NAN;
    if (rho) rho[i] = i < (int32_t)s->hist_rho.size() ? s->hist_rho[i] : NAN;
    if (jstar) jstar[i] = i < (int32_t)s->hist_jstar.size() ? s->hist_jstar[i] : -1;
  }
  if (count) *count = k;
  return IGM_OK;
}

igm_status igm_int_cycle(igm_system *s, const int64_t *v1, int32_t k, igm_cycle_trace *t) {
  if (!s || !v1 || !t || k < 1 || t->m != s->pol.m || !t->H || !t->c || !t->s || !t->g) return IGM_ERR_ARG;
  const int m = s->pol.m;
  IGM_HIP(hipMemsetAsync(s->d_V, 0, sizeof(int64_t) * (size_t)(m + 1) * s->npad, s->stream));
  IGM_HIP(hipMemsetAsync(s->d_H, 0, sizeof(int64_t) * (size_t)(m + 1) * m, s->stream));
  IGM_HIP(hipMemsetAsync(s->d_c, 0, sizeof(int64_t) * m, s->stream));
  IGM_HIP(hipMemsetAsync(s->d_s, 0, sizeof(int64_t) * m, s->stream));
  IGM_HIP(hipMemsetAsync(s->d_g, 0, sizeof(int64_t) * (m + 1), s->stream));
  IGM_HIP(hipMemcpyAsync(s->d_V, v1, sizeof(int64_t) * s->n, hipMemcpyHostToDevice, s->stream));
  IGM_TRY(prepare_cycle(s));
  CycleArgs a = make_args(s);
  a.nterms = terms_for(s->pol, k, s->hs.nterms);
  IGM_TRY(launch_cycle(s, a));
  CycleState cs;
  IGM_HIP(hipMemcpyAsync(&cs, s->d_state, sizeof(cs), hipMemcpyDeviceToHost, s->stream));
  IGM_HIP(hipMemcpyAsync(t->H, s->d_H, sizeof(int64_t) * (size_t)(m + 1) * m, hipMemcpyDeviceToHost, s->stream));
  IGM_HIP(hipMemcpyAsync(t->c, s->d_c, sizeof(int64_t) * m, hipMemcpyDeviceToHost, s->stream));
  IGM_HIP(hipMemcpyAsync(t->s, s->d_s, sizeof(int64_t) * m, hipMemcpyDeviceToHost, s->stream));
  IGM_HIP(hipMemcpyAsync(t->g, s->d_g, sizeof(int64_t) * (m + 1), hipMemcpyDeviceToHost, s->stream));
  if (t->V)
    for (int j = 0; j <= m; ++j)
      IGM_HIP(hipMemcpyAsync(t->V + (size_t)j * s->n, s->d_V + (size_t)j * s->npad, sizeof(int64_t) * s->n,
                             hipMemcpyDeviceToHost, s->stream));
  IGM_HIP(hipStreamSynchronize(s->stream));
  if (cs.timeout) { s->last_error_line = __LINE__; return IGM_ERR_DEVICE; }
  for (int k = 0; k < 8; ++k) s->stats.phase_us[k] = (double)cs.phase[k] * s->wall_us_per_tick;
  t->jstar = cs.jstar;
  t->breakdown = cs.breakdown;
  t->steps = cs.steps;
  t->first_ovf = cs.first_ovf;
  return IGM_OK;
}

// ---- kernel-level entry points ---------------------------------------------

// Kernel-level calls: reset the overflow record, record an event pair around
// the kernels themselves, then read back the event code and the duration.
static igm_status reset_state(igm_system *s) {
  IGM_TRY(prepare_cycle(s));
  if (!s->ev0) {
    IGM_HIP(hipEventCreate(&s->ev0));
    IGM_HIP(hipEventCreate(&s->ev1));
  }
  IGM_HIP(hipEventRecord(s->ev0, s->stream));
  return IGM_OK;
}

static igm_status read_event(igm_system *s, int64_t *first_ovf) {
  IGM_HIP(hipEventRecord(s->ev1, s->stream));
  CycleState cs;
  IGM_HIP(hipMemcpyAsync(&cs, s->d_state, sizeof(cs), hipMemcpyDeviceToHost, s->stream));
  IGM_HIP(hipStreamSynchronize(s->stream));
  float ms = 0.f;
  IGM_HIP(hipEventElapsedTime(&ms, s->ev0, s->ev1));
  s->stats.time_kernel_ms = ms;
  if (first_ovf) *first_ovf = cs.first_ovf;
  return IGM_OK;
}

igm_status igm_spmv(igm_system *s, int32_t nterms, const int64_t *v, int64_t *z, int64_t *first_ovf) {
  if (!s || !v || !z) return IGM_ERR_ARG;
  IGM_TRY(reset_state(s));
  CycleArgs a = make_args(s);
  int nt = std::max(1, std::min<int>(nterms, s->hs.nterms));
  IGM_HIP(launch_spmv(s->stream, a, nt, v, z));
  return read_event(s, first_ovf);
}

igm_status igm_precond(igm_system *s, const int64_t *z, int64_t *w, int64_t *first_ovf) {
  if (!s || !z || !w) return IGM_ERR_ARG;
  IGM_TRY(reset_state(s));
  CycleArgs a = make_args(s);
  IGM_HIP(launch_precond(s->stream, a, z, w));
  return read_event(s, first_ovf);
}

igm_status igm_dot(igm_system *s, const int64_t *w, const int64_t *v, int64_t *h, int64_t *first_ovf) {
  if (!s || !w || !v || !h) return IGM_ERR_ARG;
  IGM_TRY(reset_state(s));
  int64_t *d_out = (int64_t *)(s->d_scal + kScalOut);
  IGM_HIP(launch_reduce(s->stream, s->n, w, v, s->pol.b_dot, s->pol.df, 0, s->d_parts, d_out, s->d_state,
                        ((int64_t)1 << 24) | (3 << 16)));
  IGM_TRY(read_event(s, first_ovf));
  IGM_HIP(hipMemcpy(h, d_out, sizeof(int64_t), hipMemcpyDeviceToHost));
  return IGM_OK;
}

igm_status igm_axpy(igm_system *s, int64_t h, int64_t *w, const int64_t *v, int64_t *first_ovf) {
  if (!s || !w || !v) return IGM_ERR_ARG;
  IGM_TRY(reset_state(s));
  IGM_HIP(launch_axpy(s->stream, s->n, h, s->pol.b_axpy, s->pol.df, w, v, s->d_state));
  return read_event(s, first_ovf);
}

igm_status igm_norm(igm_system *s, const int64_t *w, int64_t *h, int64_t *first_ovf) {
  if (!s || !w || !h) return IGM_ERR_ARG;
  IGM_TRY(reset_state(s));
  int64_t *d_out = (int64_t *)(s->d_scal + kScalOut);
  IGM_HIP(launch_reduce(s->stream, s->n, w, w, s->pol.b_norm, s->pol.df, 1, s->d_parts, d_out, s->d_state,
                        ((int64_t)1 << 24) | (4 << 16)));
  IGM_TRY(read_event(s, first_ovf));
  IGM_HIP(hipMemcpy(h, d_out, sizeof(int64_t), hipMemcpyDeviceToHost));
  return IGM_OK;
}

igm_status igm_normalize(igm_system *s, const int64_t *w, int64_t h, int64_t *v, int64_t *first_ovf) {
  if (!s || !w || !v) return IGM_ERR_ARG;
  const int64_t den = h >> s->pol.b_div_den;
  if (den == 0) return IGM_ERR_BREAKDOWN;
  IGM_TRY(reset_state(s));
  IGM_HIP(launch_normalize(s->stream, s->n, w, den, s->pol.b_div_num,
                           s->pol.df - s->pol.b_div_num - s->pol.b_div_den, v, s->d_state));
  return read_event(s, first_ovf);
}

igm_status igm_residual(igm_system *s, const double *x, double *r, double *rhat) {
  if (!s || !x || !r || !rhat) return IGM_ERR_ARG;
  IGM_HIP(hipMemsetAsync(s->d_red, 0, sizeof(unsigned long long) * kRedTotal, s->stream));
  IGM_HIP(launch_residual(s->stream, s->n, s->d_row_ptr, s->d_col, s->d_a, s->d_ahat, s->d_b, s->d_bhat, x,
                          s->d_cscale, r, rhat, s->d_red, residual_lanes(s)));
  IGM_HIP(hipStreamSynchronize(s->stream));
  return IGM_OK;
}

igm_status igm_fp_norm(igm_system *s, const double *x, int64_t len, double *norm) {
  if (!s || !x || !norm || len < 0 || len >= ((int64_t)1 << 31)) return IGM_ERR_ARG;
  IGM_TRY(device_norm(s, x, len, s->d_scal + kScalOut));
  IGM_HIP(hipMemcpyAsync(norm, s->d_scal + kScalOut, sizeof(double), hipMemcpyDeviceToHost, s->stream));
  IGM_HIP(hipStreamSynchronize(s->stream));
  return IGM_OK;
}

igm_status igm_start_vector(igm_system *s, const double *r, double *bk, double *r0, int64_t *v1, double *gamma,
                            double *rho) {
  if (!s || !r || !bk || !r0 || !v1 || !gamma || !rho) return IGM_ERR_ARG;
  IGM_TRY(reset_state(s));
  IGM_HIP(hipMemsetAsync(s->d_red, 0, sizeof(unsigned long long) * kRedTotal, s->stream));
  IGM_HIP(launch_absmax(s->stream, s->n, r, s->d_red + kRedMuR));
  IGM_HIP(launch_fin_max(s->stream, s->d_red + kRedMuR, s->d_scal + kScalGamma));
  IGM_HIP(hipMemcpyAsync(s->h_pinned, s->d_scal + kScalGamma, sizeof(double), hipMemcpyDeviceToHost, s->stream));
  IGM_HIP(hipStreamSynchronize(s->stream));
  const double g = s->h_pinned[0];
  *gamma = g;
  *rho = 0.0;
  if (g == 0.0) return IGM_OK;
  CycleArgs a = make_args(s);
  a.V = v1;  // the cast of v1 writes its output as the first basis vector
  IGM_HIP(launch_start_vector(s->stream, a, r, s->d_scal, s->d_lvalf, s->d_uvalf, bk, r0, s->d_red));
  CycleState cs;
  IGM_HIP(hipMemcpyAsync(&cs, s->d_state, sizeof(cs), hipMemcpyDeviceToHost, s->stream));
  IGM_HIP(hipMemcpyAsync(s->h_pinned, s->d_scal, sizeof(double) * kScalWords, hipMemcpyDeviceToHost, s->stream));
  IGM_HIP(hipStreamSynchronize(s->stream));
  *rho = s->h_pinned[kScalRho];
  return cs.range_err ? IGM_ERR_RANGE : IGM_OK;
}

void igm_destroy(igm_system *s) {
  if (!s) return;
  (void)hipStreamSynchronize(s->stream);
  if (s->ev0) { (void)hipEventDestroy(s->ev0); (void)hipEventDestroy(s->ev1); }
  free_device(s);
  delete s;
}

const char *igm_status_str(igm_status st) {
  switch (st) {
    case IGM_OK: return "ok";
    case IGM_NOT_CONVERGED: return "not converged";
    case IGM_PENDING: return "pending";
    case IGM_ERR_ARG: return "invalid argument";
    case IGM_ERR_SINGULAR_ROW: return "all-zero row";
    case IGM_ERR_ZERO_PIVOT: return "zero pivot";
    case IGM_ERR_OVERFLOW: return "fixed-point overflow";
    case IGM_ERR_RANGE: return "value out of range";
    case IGM_ERR_OOM: return "out of memory";
    case IGM_ERR_DEVICE: return "device error";
    case IGM_ERR_BREAKDOWN: return "breakdown";
    case IGM_ERR_UNSUPPORTED: return "unsupported size";
  }
  return "unknown status";
}

}  // extern "C"
