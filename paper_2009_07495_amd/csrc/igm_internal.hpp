// Internal structures of the igmres library (host side).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <memory>
#include <string>
#include <type_traits>
#include <utility>
#include <vector>

#include "../../include/igmres.h"

namespace igm {

// Allocator that leaves elements default-initialised (no zero fill for plain
// numbers), so the parallel pass that writes every element of a fresh setup
// array also takes its page faults in parallel.
template <class T>
struct NoInitAlloc : std::allocator<T> {
  template <class U>
  struct rebind {
    using other = NoInitAlloc<U>;
  };
  NoInitAlloc() = default;
  template <class U>
  NoInitAlloc(const NoInitAlloc<U> &) noexcept {}
  template <class U>
  void construct(U *p) noexcept(std::is_nothrow_default_constructible<U>::value) {
    ::new ((void *)p) U;
  }
  template <class U, class... Args>
  void construct(U *p, Args &&...args) {
    ::new ((void *)p) U(std::forward<Args>(args)...);
  }
};
// Host array of the setup: resize(n) leaves the new elements unset.
template <class T>
using hvec = std::vector<T, NoInitAlloc<T>>;

constexpr int kMaxTerms = 9;       // A_0 .. A_8
// LDS of the merge-based chunk SpMV of a workgroup of `block` threads: int32
// row offsets (block + 1, padded to 16 bytes), then two int64 limb sums per row.
constexpr size_t merge_rp_bytes(int block) { return ((size_t)(block + 1) * 4 + 15) / 16 * 16; }
constexpr size_t merge_lds_bytes(int block) { return merge_rp_bytes(block) + (size_t)block * 16; }
constexpr int kSlice = 64;         // SELL slice height = wavefront width
constexpr int kSyncGroups = 8;     // arrival words per grid reduction (K)
constexpr int kMaxRows = 16;       // largest rows-per-thread instantiation

// Device-side record of one int-GMRES call.
struct CycleState {
  int64_t first_ovf;     // smallest overflow event code (atomicMin)
  int32_t jstar, breakdown, steps, timeout;
  int32_t range_err, pad_;
  // wall-clock ticks spent by workgroup 0 in each phase of the call:
  // 0 SpMV + preconditioner, 1 inner products/updates (local work),
  // 2 inner products (grid reduction wait), 3 norm, 4 normalisation,
  // 5 Givens, 6 end-of-step barrier, 7 whole call
  uint64_t phase[8];
};

// One dependency wait of the blocked triangular sweep (igm_bsweep.hpp):
// before local level `level`, block `dep` must have finished `need` of its
// local levels; `slot` indexes the waiting block's cache of what it last saw
// of that block.
struct alignas(16) WaitRec {
  int32_t level, slot, need, dep;
};

// Blocked schedule of one triangular sweep of the integer ILU(0) factors
// (forward on the strict lower factor in increasing rows, backward on the
// strict upper factor in decreasing rows). Positions number the rows in
// processing order; block q holds positions [q S, (q + 1) S), and inside a
// block the rows are sorted by local level (a row's level counts only the
// dependencies inside its block). Every dependency outside the block is in an
// earlier block and becomes a wait on that block's progress.
struct BlockSchedule {
  int32_t S = 0, nb = 0;     // rows per block, blocks
  int32_t max_slots = 0;     // most dependency blocks of one block
  int32_t max_levels = 0;    // most local levels of one block
  int32_t max_width = 0;     // most rows of one local level
  bool narrow = false;       // every factor value fits in int32
  hvec<int32_t> prow;        // n: row of each sorted position
  hvec<int32_t> plen;        // n: entries of each sorted position's row
  hvec<int32_t> ecode;       // >= 0: sorted position inside the block of an in-block dependency; < 0: -(row + 1)
  hvec<int64_t> eval;        // the factor's value of each entry
  hvec<double> evalf;        // the same values as doubles (FP64 start step)
  hvec<int64_t> pdiag;       // n: the factor's diagonal of each sorted position's row
  // n: the diagonal as an invariant divisor (see div_magic): multiplier, and
  // the shift l = ceil(log2 |d|) with bit 8 set for a negative divisor
  hvec<uint64_t> pmag;
  hvec<int32_t> pshift;
  hvec<int32_t> lvbase;      // nb + 1: where each block's level offsets start in lvoff and levent
  hvec<int32_t> lvoff;       // per block, nl + 1 offsets of its levels (positions inside the block)
  // per block, nl + 1: where each level's entries start. Inside a level of c
  // rows the entries are column-major: entry k (CSR order) of the level's
  // i-th row is at levent[L] + k c + i, so a row's entries are addressed from
  // its position alone; slots past a row's length are padding.
  hvec<int64_t> levent;
  hvec<int32_t> wbase;       // nb + 1: where each block's wait records start in wrec
  hvec<WaitRec> wrec;        // per block, sorted by level
  int64_t pad_slot = 0;      // the slot after every block's entries (ecode, eval, evalf hold pad_slot + 1)
};

// Device view of one BlockSchedule.
struct BlockSweepArgs {
  int32_t S, nb;
  int32_t narrow;      // every factor value fits in int32
  int32_t max_levels;  // most local levels of one block (sizes the LDS copy of a block's level table)
  int32_t max_width;   // most rows of one local level (sizes the integer sweep's compute wavefronts)
  const int32_t *prow, *plen;
  const int32_t *ecode;
  const int64_t *eval;
  const double *evalf;
  const int64_t *pdiag;
  const uint64_t *pmag;
  const int32_t *pshift;
  const int32_t *lvbase, *lvoff, *wbase;
  const int64_t *levent;
  const WaitRec *wrec;
  // a slot past every block's entries (code 0, value 0): the integer sweep's
  // prefetch loads it for lanes and entries without one
  int64_t pad_slot;
  // nb progress words kLevStride apart, zero at the start of the sweep: the
  // block's helper wavefront adds one per finished level
  unsigned *prog;
};

// Dependency blocks per block whose progress a sweep caches in LDS, wait
// records held in LDS at a time, and the LDS a sweep needs: the block's S
// values, its level table (offsets and entry starts of max_levels + 1
// levels), the record window, that cache, 16 spare bytes and the ring of the
// rows of the last two levels (kRowRing each).
constexpr int kSeenSlots = 256;
constexpr int kRecWindow = 256;
constexpr int kRowRing = 1024;
inline size_t sweep_lds_bytes(int64_t S, int32_t max_levels) {
  const size_t lv = (size_t)max_levels + 1;
  return 8 * (size_t)S + 8 * lv + (4 * lv + 15) / 16 * 16 + 16 * (size_t)kRecWindow + 4 * (size_t)kSeenSlots + 16 +
         8 * (size_t)kRowRing;
}
// Rows per block and lanes per row of the blocked sweeps when the policy
// leaves them open, and the static LDS the cycle kernel keeps besides its
// dynamic part (reduction scratch and flags; an upper bound).
constexpr int kSweepRowsAuto = 16384;
constexpr int kSweepLanesAuto = 4;
constexpr int kCycleStaticLds = 4096;

// Truncating division by an invariant nonzero divisor d through one
// multiply-high (Granlund and Montgomery, "Division by invariant integers
// using multiplication", 1994, unsigned form): with l = ceil(log2 |d|) and
// m = floor(2^64 (2^l - |d|) / |d|) + 1, floor(u / |d|) = (t + ((u - t) >> min(l, 1))) >> max(l - 1, 0)
// for every u < 2^64, t = floor(m u / 2^64). The sign follows C division.
inline void div_magic(int64_t d, uint64_t &m, int32_t &shift) {
  const uint64_t a = d < 0 ? 0ull - (uint64_t)d : (uint64_t)d;
  int32_t l = 0;
  while (l < 64 && (((unsigned __int128)1) << l) < a) ++l;
  m = (uint64_t)((((unsigned __int128)((((unsigned __int128)1) << l) - a)) << 64) / a) + 1;
  shift = l | (d < 0 ? 256 : 0);
}

// Builds the schedule of one sweep from a strict triangular factor in CSR
// (ptr, col, val), its diagonal, and S rows per block (a multiple of 64).
void block_schedule(int64_t n, bool lower, int32_t S, const hvec<int64_t> &ptr, const hvec<int32_t> &col,
                    const hvec<int64_t> &val, const hvec<int64_t> &diag, BlockSchedule &out);

// Host-side setup products (all derived from the FP64 input).
struct HostSetup {
  hvec<double> dhat, a, b;                     // eq. (eq1)/(eq2), (eq3)
  hvec<double> cscale;                         // eq. (eq2): sqrt(dhat); empty for eq. (eq1)
  int nterms = 0;
  int32_t alpha[kMaxTerms] = {0};
  std::vector<hvec<int64_t>> abar;             // eq. (A), on the input pattern
  hvec<int64_t> diag_pos;
  hvec<double> lu;                             // FP64 ILU(0) of A
  hvec<int64_t> ldiag, udiag;                  // cast diagonals
  // strict triangles of the integer factors, CSR
  hvec<int64_t> lptr, uptr;
  hvec<int32_t> lcol, ucol;
  hvec<int64_t> lval, uval;
  // level sets of the triangular sweeps
  hvec<int32_t> flev_ptr, flev_rows, blev_ptr, blev_rows;
  // SELL-64 layout of the integer matrices
  int64_t nslices = 0;
  hvec<int64_t> sell_off;                      // nslices + 1, entries
  hvec<int32_t> sell_w;                        // nslices
  hvec<int32_t> sell_col;                      // padded
  std::vector<hvec<int64_t>> sell_val;         // per term
};

igm_status host_setup(int64_t n, const hvec<int64_t> &row_ptr, const hvec<int32_t> &col,
                      const hvec<double> &ahat, const hvec<double> &bhat, const igm_policy &pol,
                      HostSetup &out);
igm_status check_policy(const igm_policy &p);
// The structural part of host_setup only, for a setup whose values are
// computed on the device: diagonal positions (-1 where a row has none; the
// device reports that, after the errors the host setup finds first), the
// factor patterns and level sets, the SELL-64 offsets, widths and columns. One matrix term, no
// Gauss-Seidel splitting (else IGM_ERR_UNSUPPORTED).
igm_status host_structure(int64_t n, const hvec<int64_t> &row_ptr, const hvec<int32_t> &col, const igm_policy &pol,
                          HostSetup &out);
// Overflow-driven shift retry (igm_policy.shift_retry): adjusts the shift that
// the stage of overflow event `code` names, in any record with the shift
// fields of igm_policy (the policy on the host, a team's working copy on the
// device); false if none can change. A right shift taken before a product
// grows by 4, at most to df (more bits dropped, a smaller product); a
// division's exponents shrink by 4, the numerator's first (a smaller
// quotient). Event codes: stage in bits 16-23, sub-stage in bits 0-15.
template <class P>
__host__ __device__ inline bool adjust_shift_fields(P &p, int32_t df, int64_t code) {
  // each case names its field directly (no pointer chosen at run time, so a
  // device copy of the fields stays in registers)
  auto raise = [df](int32_t &b) {
    if (b >= df) return false;
    b = b + 4 < df ? b + 4 : df;
    return true;
  };
  auto lower = [](int32_t &num, int32_t &den) {
    if (num > 0) {
      num = num > 4 ? num - 4 : 0;
      return true;
    }
    if (den <= 0) return false;
    den = den > 4 ? den - 4 : 0;
    return true;
  };
  if (code == INT64_MAX) return false;
  switch ((int)((code >> 16) & 0xFF)) {
    case 3: return (code & 1) == 0 ? raise(p.b_dot) : raise(p.b_axpy);  // inner product (even sub) / update
    case 4: return raise(p.b_norm);                                      // norm of w
    case 5: return lower(p.b_div_num, p.b_div_den);                      // normalisation
    case 6: return raise(p.b_rot);                                       // earlier rotations
    case 7: return raise(p.b_tmp);                                       // rotation radius
    case 8: return lower(p.b_cs_num, p.b_cs_den);                        // new rotation
    default: return false;                                               // SpMV, preconditioner, rotation of g
  }
}
inline bool adjust_shifts(igm_policy &p, int64_t code) { return adjust_shift_fields(p, p.df, code); }
// Rows of the largest level set of the ILU sweeps (0 without ILU).
int32_t max_level_rows(const HostSetup &h);
// Threads per workgroup that take part in the counter-driven ILU sweeps of a
// grid of `grid` workgroups of `block` threads: whole wavefronts, enough that
// about four times the widest level is in flight, at most the workgroup. The
// environment variable IGM_SWEEP_THREADS (a multiple of 64) overrides it.
int32_t sweep_threads(int block, int grid, int32_t max_level);
igm_status validate_csr(int64_t n, const int64_t *rp, const int32_t *col, const double *val, const double *b);

// Host-visible layout of an exact device partial sum (value = hi * 2^40 + lo).
struct AccWords {
  int64_t lo, hi;
};

struct DevBuf {
  void *p = nullptr;
  size_t bytes = 0;
};

// Spacing (32-bit words) of the completion counters of the ILU sweeps.
#ifndef IGM_LEV_STRIDE
#define IGM_LEV_STRIDE 32
#endif
constexpr int kLevStride = IGM_LEV_STRIDE;

// Arguments of the persistent cycle kernel.
struct CycleArgs {
  int64_t n, npad;
  int32_t m, df, nterms, precond;
  int32_t b_dot, b_axpy, b_norm, b_div_num, b_div_den, b_rot, b_tmp, b_cs_num, b_cs_den;
  int32_t nflev, nblev;
  int32_t max_level;  // rows of the largest ILU level set
  int64_t gtol;
  const int64_t *sell_off;
  const int32_t *sell_w;
  const int32_t *sell_col;
  const int64_t *sell_val[kMaxTerms];
  int32_t alpha[kMaxTerms];
  const int64_t *ldiag, *udiag;
  const int64_t *lptr, *uptr;
  const int32_t *lcol, *ucol;
  const int64_t *lval, *uval;
  const int32_t *flev_ptr, *flev_rows, *blev_ptr, *blev_rows;
  const int32_t *flev_host, *blev_host;  // host copies of the level offsets (launchers only)
  int64_t *V;      // (m+1) x npad
  int64_t *zbuf;   // npad (preconditioner path)
  int64_t *wbuf;   // npad (preconditioner path)
  unsigned *lev_cnt;      // ILU: completion counters (igm_sweep.hpp), nflev forward then nblev backward
  int32_t sweep_threads;  // ILU: threads per workgroup taking part in the sweeps (multiple of 64)
  // integer SpMV with several lanes per row (spmv_lanes 4, 16, 64; 1 = SELL-64):
  // the integer matrices in CSR order, and the byte offset of the LDS that
  // passes each chunk's row sums to their owners
  int32_t spmv_lanes;
  int32_t spmv_lds_off;
  const int64_t *crp;
  const int32_t *ccol;
  const int64_t *cval[kMaxTerms];
  BlockSweepArgs bsf, bsb;  // ILU: blocked schedules of the forward and backward sweeps (igm_bsweep.hpp)
  int32_t sweep_lanes;      // ILU: the policy's lanes per row (the sweeps run 4 whatever the value)
  int32_t sweep_lds_off;    // ILU: byte offset of the sweeps' LDS (S values, then the seen cache)
  int64_t *H, *c, *s, *g;
  CycleState *state;
  unsigned long long *sync;  // 2 * kSyncGroups * sync_cap words
  int32_t sync_cap;
  int32_t update;            // apply the closing least-squares step of Fig. 2 and x += gamma x^(k)
  int32_t phase_clock;       // record the phase clocks of workgroup 0
  double *x;
  const double *scal;        // device: {gamma, rho}
  const double *cscale;      // eq. (eq2): the update adds gamma (x^(k)_i / s_i); null for eq. (eq1)
};

// SpMV mappings of the cycle kernel: one thread per row over SELL-64, lanes
// per row over CSR, chunks split evenly by entries over the workgroup.
constexpr int kMapSell = 0, kMapLanes = 1, kMapMerge = 2;
const void *cycle_kernel(int block, int R, int pre, int spmv_lanes);
size_t cycle_smem_bytes(int m);

}  // namespace igm

struct igm_system {
  int device = 0;
  hipStream_t stream = nullptr;
  igm_policy pol{};
  int64_t n = 0, nnz = 0, npad = 0;
  igm::hvec<int64_t> row_ptr;
  igm::hvec<int32_t> col;
  igm::hvec<double> ahat, bhat;
  igm::HostSetup hs;
  double bhat_norm = 0.0, b_norm = 0.0;
  // device memory
  std::vector<igm::DevBuf> bufs;
  int64_t *d_row_ptr = nullptr;
  int32_t *d_col = nullptr;
  double *d_a = nullptr, *d_ahat = nullptr, *d_b = nullptr, *d_bhat = nullptr;
  double *d_cscale = nullptr;  // eq. (eq2) only
  int64_t *d_sell_off = nullptr;
  int32_t *d_sell_w = nullptr, *d_sell_col = nullptr;
  int64_t *d_sell_val[igm::kMaxTerms] = {nullptr};
  int64_t *d_ldiag = nullptr, *d_udiag = nullptr;
  int64_t *d_lptr = nullptr, *d_uptr = nullptr;
  int32_t *d_lcol = nullptr, *d_ucol = nullptr;
  int64_t *d_lval = nullptr, *d_uval = nullptr;
  double *d_lvalf = nullptr, *d_uvalf = nullptr;
  int32_t *d_flev_ptr = nullptr, *d_flev_rows = nullptr, *d_blev_ptr = nullptr, *d_blev_rows = nullptr;
  // work vectors
  int64_t *d_V = nullptr, *d_z = nullptr, *d_w = nullptr;
  unsigned *d_levcnt = nullptr;
  double *d_r = nullptr, *d_rhat = nullptr, *d_bk = nullptr, *d_r0 = nullptr, *d_x = nullptr;
  int64_t *d_H = nullptr, *d_c = nullptr, *d_s = nullptr, *d_g = nullptr;
  igm::CycleState *d_state = nullptr;
  unsigned long long *d_sync = nullptr;
  int32_t sync_cap = 0;
  unsigned long long *d_red = nullptr;  // scratch words of the FP64 reductions
  double *d_scal = nullptr;             // device scalars (gamma, rho, relres, norms)
  igm::AccWords *d_parts = nullptr;     // per-workgroup partial sums of the standalone reductions
  double *h_pinned = nullptr;           // small pinned staging area
  int m_alloc = 0;
  // launch configuration of the cycle kernel
  int grid = 0, block = 0, rows_per_thread = 0, max_coresident = 0;
  // ILU(0): blocked schedules of the two sweeps (device copies), their
  // progress words, and the cycle kernel's dynamic LDS (cycle part + sweeps)
  igm::BlockSweepArgs bsf{}, bsb{};
  unsigned *d_prog = nullptr;
  // integer matrices in CSR order (spmv_lanes > 1) and the chosen lanes per row
  int64_t *d_cval[igm::kMaxTerms] = {nullptr};
  int32_t spmv_lanes = 1;
  bool spmv_merge_ok = true;  // every 1024-row window holds fewer than 2^30 entries
  size_t spmv_lds_off = 0;
  int32_t sweep_lanes = 0;
  size_t cycle_lds = 0, sweep_lds_off = 0;
  // statistics
  igm_stats stats{};
  std::vector<double> hist_ro, hist_rs, hist_gamma, hist_rho;
  std::vector<int32_t> hist_jstar;
  int64_t device_bytes = 0;
  int last_error_line = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;  // timing of kernel-level calls
  double wall_us_per_tick = 0.0;             // device wall clock period
};
