// Level-scheduled triangular sweeps of the integer ILU(0) preconditioner
// (the preconditioner apply of Sec. VI) without a barrier per level.
//
// The rows of a triangular factor are grouped into level sets (every row
// depends only on rows of lower levels) and stored level by level, so the
// concatenated row list is a topological order. Each level L has a
// completion counter (word L * kLevStride of `cnt`); a row of level L may
// start once the counter of level L - 1 shows that whole level done (by
// induction every lower level is then done too). The counters only grow: in
// the sweep numbered `round` (0, 1, ... since they were cleared) level L is
// done when its counter reaches (round + 1) * |L| (compared modulo 2^32).
//
// Position p of the row list is handled by thread `pos0 + k * stride` of the
// participants, in increasing k. A thread loads the row's structure, its
// right-hand side and its diagonal before it waits, so only the gather of the
// finished neighbours and the arithmetic lie on the chain of dependent levels.
// Finished rows are stored with device-coherent stores; after they complete,
// one lane per level present among them adds their count to the level's
// counter (relaxed agent-scope atomic). A waiting row reads the counter and
// then the neighbours with device-coherent loads, so no cache write-back or
// invalidation is needed.
//
// Progress: every participant is resident and handles its positions in
// increasing order, and a wavefront re-checks all of its unfinished lanes on
// every pass, so the smallest unfinished position (whose lower levels are all
// done) always completes on its owner's next pass. Every wait is bounded
// (kSpinLimit passes); on timeout `to` is set and the remaining rows are
// computed from whatever values are present, so the sweep always ends.
#pragma once

#include "igm_rows.hpp"
#include "igm_sync.hpp"

namespace igm {

// entries of a row loaded before the wait (default of PRE below)
#ifndef IGM_SWEEP_PRE
#define IGM_SWEEP_PRE 16
#endif
constexpr int kSweepPre = IGM_SWEEP_PRE;

// One sweep. Integer (FP = false): y = tdiv(src - Lbar_strict y, Lbar_ii)
// (LOWER, src = z) or u = tdiv(src - Ubar_strict u, Ubar_ii), the sums exact.
// FP64 (FP = true, the start step of Sec. VI): the same substitution with the factors' values
// in FP64, each row summed in CSR order and then divided by its diagonal.
// src == dst is allowed (in place): row i reads src only at i and dst only at
// its neighbours, which precede it in the order. `a` is any record with the
// ILU fields of CycleArgs (and lvalf/uvalf for FP). PRE entries of the row
// are loaded before the wait (more registers, fewer dependent loads after it).
// Must be called by whole wavefronts (every lane, the same pos0 - lane and
// stride).
template <bool LOWER, bool FP, int PRE = kSweepPre, class A, class TX>
__device__ __forceinline__ void level_sweep(const A &a, const int32_t *__restrict__ lev_ptr,
                                            const int32_t *__restrict__ lev_rows, int nlev, unsigned *cnt,
                                            unsigned round, int64_t pos0, int64_t stride, const TX *src, TX *dst,
                                            bool &ovf, bool &to) {
  const int64_t *__restrict__ ptr = LOWER ? a.lptr : a.uptr;
  const int32_t *__restrict__ colp = LOWER ? a.lcol : a.ucol;
  const TX *__restrict__ valp;
  if constexpr (FP) valp = LOWER ? a.lvalf : a.uvalf;
  else valp = LOWER ? a.lval : a.uval;
  const int64_t *__restrict__ diag = LOWER ? a.ldiag : a.udiag;
  const int lane = threadIdx.x & 63;
  const int64_t nrows = nlev > 0 ? lev_ptr[nlev] : 0;
  int L = 0;
  for (int64_t base = 0; base < nrows; base += stride) {
    const int64_t p = base + pos0;
    bool todo = p < nrows;
    int64_t row = 0, lo = 0, hi = 0, dg = 1;
    TX rhs = 0;
    unsigned need = 0;
    int32_t c[PRE];
    TX v[PRE];
    if (todo) {
      // level of p: lev_ptr[L] <= p < lev_ptr[L + 1]; L never decreases
      int l0 = L, l1 = nlev - 1;
      while (l0 < l1) {
        const int mid = (l0 + l1 + 1) >> 1;
        if (lev_ptr[mid] <= p) l0 = mid; else l1 = mid - 1;
      }
      L = l0;
      if (L > 0) need = (round + 1u) * (unsigned)(lev_ptr[L] - lev_ptr[L - 1]);
      row = lev_rows[p];
      lo = ptr[row];
      hi = ptr[row + 1];
      dg = diag[row];
#pragma unroll
      for (int k = 0; k < PRE; ++k)
        if (lo + k < hi) {
          c[k] = colp[lo + k];
          v[k] = valp[lo + k];
        }
      rhs = ld_coh(src + row);
    }
    for (int spin = 0;; ++spin) {
      bool done = false;
      if (todo && (L == 0 || to || (int)(ld_coh(cnt + (L - 1) * kLevStride) - need) >= 0)) {
        Acc acc;
        acc.zero();
        double facc = 0.0;
        if constexpr (!FP) acc.add(rhs);
        // chunks of PRE entries in CSR order; the first one was loaded
        // before the wait
        for (int64_t e0 = lo; e0 < hi; e0 += PRE) {
          if (e0 > lo) {
#pragma unroll
            for (int k = 0; k < PRE; ++k)
              if (e0 + k < hi) {
                c[k] = colp[e0 + k];
                v[k] = valp[e0 + k];
              }
          }
          TX xv[PRE];
#pragma unroll
          for (int k = 0; k < PRE; ++k)
            if (e0 + k < hi) xv[k] = ld_coh(dst + c[k]);
#pragma unroll
          for (int k = 0; k < PRE; ++k)
            if (e0 + k < hi) {
              if constexpr (FP) facc = facc + v[k] * xv[k];
              else acc.sub(mulw(xv[k], v[k], ovf));
            }
        }
        if constexpr (FP) st_coh(dst + row, (rhs - facc) / (double)dg);
        else st_coh(dst + row, tdiv(acc.value(ovf), dg, ovf));
        done = true;
      }
      unsigned long long fin = __ballot(done);
      if (fin) {
        wait_vm();
        while (fin) {
          const int first = __ffsll((long long)fin) - 1;
          const int Lf = __shfl(L, first, 64);
          const unsigned long long grp = __ballot(done && L == Lf);
          if (lane == first)
            __hip_atomic_fetch_add(cnt + Lf * kLevStride, (unsigned)__popcll(grp), __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
          fin &= ~grp;
        }
      }
      todo = todo && !done;
      if (!__any(todo)) break;
      if (spin >= kSpinLimit) to = true;
      __builtin_amdgcn_s_sleep(IGM_POLL_SLEEP);
    }
  }
}

}  // namespace igm
