// Blocked triangular sweeps of the ILU(0) preconditioner (the preconditioner
// apply of Sec. VI: y = tdiv(z - Lbar_strict y, Lbar_ii) in increasing rows,
// then u = tdiv(y - Ubar_strict u, Ubar_ii) in decreasing rows; and the same
// substitutions in FP64 for the start step).
//
// The rows are cut into blocks of S consecutive positions in processing
// order (igm_bsched.cpp). One workgroup runs a block: level by level (local
// levels: only dependencies inside the block count), the block's values kept
// in LDS, one workgroup barrier between levels. A dependency on another block
// (always an earlier one) is a wait on that block's progress word, the number
// of its local levels finished, which the block's workgroup publishes after
// every level once its stores of that level have completed. Progress words
// start at zero for every sweep. Workgroup b runs blocks b, b + G, b + 2G, ...
// in order, so the lowest unfinished block only waits for finished blocks and
// always progresses; every wait is bounded (kSpinLimit polls), after which
// `to` is set and the rows are computed from whatever values are present, so
// the sweep always ends.
//
// The waits of a level are taken by wavefront 0, one record per lane; what
// each dependency block was last seen to have finished is cached in LDS
// (`seen`), so a requirement already met costs no memory access. The values
// other blocks need go out with device-coherent stores and come in with
// device-coherent loads, so no cache write-back or invalidation is needed.
//
// Integer sweeps split each row's entries over G lanes (an exact sum: the
// order does not matter); the FP64 sweep sums each row in CSR order (G = 1).
#pragma once

#include "igm_rows.hpp"
#include "igm_sync.hpp"

namespace igm {

// Exact product of a wide word a and a value b in int32, reduced mod 2^64,
// with the overflow flag: a = ah 2^32 + al, both partial products fit in 64
// bits, and the result fits in int64 iff ah b + floor(al b / 2^32) fits in
// int32.
__device__ __forceinline__ int64_t mul_w32(int64_t a, int32_t b, bool &ovf) {
  const int64_t ah = a >> 32;
  const uint64_t al = (uint64_t)a & 0xFFFFFFFFull;
  const int64_t lo = (int64_t)al * (int64_t)b;
  const int64_t hi = ah * (int64_t)b;
  const int64_t t = hi + (lo >> 32);
  if (t != (int64_t)(int32_t)t) ovf = true;
  return (int64_t)(((uint64_t)hi << 32) + (uint64_t)lo);
}

// Sum of an int64 over each group of G consecutive lanes (G = 1, 2, 4, 8, 16),
// returned to every lane of the group; every lane of the wavefront active.
template <int G>
__device__ __forceinline__ int64_t group_sum64(int64_t v) {
  if constexpr (G >= 2) v += dpp64<0xB1>(v);   // quad_perm [1,0,3,2]
  if constexpr (G >= 4) v += dpp64<0x4E>(v);   // quad_perm [2,3,0,1]
  if constexpr (G >= 8) v += dpp64<0x141>(v);  // row_half_mirror
  if constexpr (G >= 16) v += dpp64<0x140>(v); // row_mirror
  return v;
}

// One sweep by the whole grid. FP = false: integer values (TX = int64_t),
// dst = tdiv(src - strict part, diagonal); FP = true: doubles, G must be 1.
// `vals` is LDS for S values, `seen` LDS for kSeenSlots words. Must be called
// by every thread of every workgroup (BLOCK threads each).
template <int BLOCK, int G, bool FP, class TX>
__device__ __forceinline__ void block_sweep(const BlockSweepArgs &b, const TX *src, TX *dst, TX *vals,
                                            unsigned *seen, bool &ovf, bool &to) {
  static_assert(BLOCK % 64 == 0 && G >= 1 && G <= 16 && (G & (G - 1)) == 0, "lanes per row");
  static_assert(!FP || G == 1, "the FP64 substitution sums each row in CSR order");
  constexpr int RPP = BLOCK / G;  // rows per pass
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int rs = tid / G, gl = tid % G;
  for (int q = blockIdx.x; q < b.nb; q += gridDim.x) {
    const int64_t q0 = (int64_t)q * b.S;
    const int lb = b.lvbase[q];
    const int nl = b.lvbase[q + 1] - lb - 1;
    int wr = b.wbase[q];
    const int we = b.wbase[q + 1];
    for (int s = tid; s < kSeenSlots; s += BLOCK) seen[s] = 0;
    __syncthreads();
    for (int L = 0; L < nl; ++L) {
      // ---- the waits of level L (wavefront 0, one record per lane)
      if (tid < 64) {
        for (;;) {
          const int r = wr + lane;
          WaitRec rec{0, 0, 0, 0};
          if (r < we) rec = b.wrec[r];
          const bool mine = r < we && rec.level == L;
          const unsigned long long got = __ballot(mine);
          if (mine) {
            const bool cached = rec.slot < kSeenSlots;
            unsigned v = cached ? seen[rec.slot] : 0u;
            for (int spin = 0; v < (unsigned)rec.need; ++spin) {
              v = ld_coh(b.prog + (int64_t)rec.dep * kLevStride);
              if (v >= (unsigned)rec.need) break;
              if (spin >= kSpinLimit || to) {
                to = true;
                break;
              }
              __builtin_amdgcn_s_sleep(IGM_POLL_SLEEP);
            }
            if (cached) seen[rec.slot] = v;
          }
          const int cnt = __popcll(got);  // the records of a level are consecutive
          wr += cnt;
          if (cnt < 64) break;
        }
      }
      __syncthreads();
      // ---- the rows of level L
      const int p0 = b.lvoff[lb + L], p1 = b.lvoff[lb + L + 1];
      for (int base = p0; base < p1; base += RPP) {
        const int lp = base + rs;
        const bool act = lp < p1;
        Acc acc;
        acc.zero();
        double facc = 0.0;
        int64_t row = 0;
        if (act) {
          const int64_t pos = q0 + lp;
          row = b.prow[pos];
          const int64_t e1 = b.eoff[pos + 1];
          for (int64_t e = b.eoff[pos] + gl; e < e1; e += G) {
            const int32_t c = b.ecode[e];
            const TX xv = c >= 0 ? vals[c] : ld_coh(dst + (-(int64_t)c - 1));
            if constexpr (FP) {
              facc = facc + b.evalf[e] * xv;
            } else {
              const int64_t v = b.eval[e];
              acc.sub(b.narrow ? mul_w32(xv, (int32_t)v, ovf) : mulw(xv, v, ovf));
            }
          }
        }
        if constexpr (!FP && G > 1) {
          acc.lo = group_sum64<G>(acc.lo);
          acc.hi = group_sum64<G>(acc.hi);
        }
        if (act && gl == 0) {
          const TX rhs = ld_coh(src + row);
          const int64_t dg = b.pdiag[q0 + lp];
          TX y;
          if constexpr (FP) {
            y = (rhs - facc) / (double)dg;
          } else {
            acc.add(rhs);
            y = tdiv(acc.value(ovf), dg, ovf);
          }
          vals[lp] = y;
          st_coh(dst + row, y);
        }
      }
      // publish level L once this workgroup's stores of it have completed
      wait_vm();
      __syncthreads();
      if (tid == 0)
        __hip_atomic_store(b.prog + (int64_t)q * kLevStride, (unsigned)(L + 1), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

}  // namespace igm
