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
// Wavefront 0 of the workgroup is a helper: it takes the waits of a level,
// one record per lane, stores the finished levels and publishes the
// progress; what each dependency block was last seen to have finished is
// cached in LDS
// (`seen`), so a requirement already met costs no memory access. The values
// other blocks need go out with device-coherent stores and come in with
// device-coherent loads, so no cache write-back or invalidation is needed.
//
// Integer sweeps split each row's entries over G lanes (an exact sum: the
// order does not matter); the FP64 sweep sums each row in CSR order (G = 1).
#pragma once

#include <type_traits>

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

// tdiv(a, d) (truncation toward zero, the flag for INT64_MIN / -1) through
// the multiplier and shift that div_magic made for d (shift 512: d == 0, the
// general division flags it).
__device__ __forceinline__ int64_t tdiv_magic(int64_t a, int64_t d, uint64_t m, int32_t sh, bool &ovf) {
  if (sh & 512) return tdiv(a, d, ovf);
  const int l = sh & 255;
  const bool neg_a = a < 0;
  const uint64_t u = neg_a ? 0ull - (uint64_t)a : (uint64_t)a;
  const uint64_t t = __umul64hi(m, u);
  const uint64_t q = (t + ((u - t) >> (l < 1 ? l : 1))) >> (l > 1 ? l - 1 : 0);
  const bool neg = neg_a != ((sh & 256) != 0);
  if (!neg && q > (uint64_t)INT64_MAX) ovf = true;
  return neg ? (int64_t)(0ull - q) : (int64_t)q;
}

// One row of the integer sweep held by a compute lane: stage 1 (loaded three
// levels ahead, addressed by the position alone; lanes and entries without a
// row or entry load the padding slot, so every compute lane issues the same
// loads) and stage 2 (loaded one level ahead: the right-hand side and the
// values of the entries from other blocks, whose waits the helper has taken by
// then; lanes and entries without one load a dummy word).
template <int PRE, class T>
struct IntRow {
  bool act;  // the lane has a row
  int lp;    // position inside the block (act)
  int32_t row;
  int32_t len;
  int64_t dg;
  uint64_t mag;  // integer sweep only
  int32_t sh;
  T rhs;
  int32_t c[PRE];
  T v[PRE];
  T x[PRE];
};

// One sweep by the whole grid with a helper wavefront (integer: dst =
// tdiv(src - strict part, diagonal)). Wavefront 0 of the workgroup is the helper: it takes the waits
// on other blocks two levels ahead, stores each finished level's values to
// global memory from LDS and publishes the block's progress (one add per
// level, after its stores of that level have completed). Wavefronts 1 .. W
// compute, G lanes per row, W as few as the widest level needs (the rest
// idle): they read the block's own values from LDS and everything else from
// registers loaded ahead, and issue no global store and no wait, so the loads
// in flight for the next levels are never drained by a step of this one.
// Per level L: the helper publishes level L - 2, stores level L - 1 and takes
// the waits of level L + 2; the compute lanes compute L and load stage 2 of
// L + 1 and stage 1 of L + 3; one workgroup barrier. The three rows in flight
// rotate through fixed registers (the loop is unrolled by three). A level
// wider than the row ring (kRowRing) is stored by the compute lanes themselves
// (waited before the barrier); a level wider than one pass takes more passes.
// `lds` holds sweep_lds_bytes(S, max_levels) bytes. Every thread of every
// workgroup calls it. FP = true: the FP64 substitution of the start step on
// the same schedule (doubles, the factor values converted to double, one lane
// per row summing its products in CSR order, then (rhs - sum) / diagonal;
// splitting the products over several lanes and adding them in order through
// shuffles measured slower).
template <int BLOCK, int G, bool FP = false, class TX = typename std::conditional<FP, double, int64_t>::type>
__device__ __forceinline__ void block_sweep_int(const BlockSweepArgs &b, const TX *src, TX *dst, char *lds,
                                                bool &ovf, bool &to) {
  static_assert(BLOCK % 64 == 0 && BLOCK >= 128 && G >= 1 && G <= 16 && (G & (G - 1)) == 0, "lanes per row");
  static_assert(!FP || G == 1, "the FP64 substitution sums each row in CSR order");
  constexpr int PRE = G >= 16 ? 1 : 16 / G;  // entries per lane held in registers
  using Row = IntRow<PRE, TX>;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const bool helper = wave == 0;
  // compute wavefronts: enough for the widest level in one pass, at most all but the helper
  const int nw = min(BLOCK / 64 - 1, max(1, (b.max_width * G + 63) / 64));
  const bool computing = wave >= 1 && wave <= nw;
  const int rpp = nw * 64 / G;  // rows per pass
  const int ct = computing ? tid - 64 : 0;
  const int rs = ct / G, gl = ct % G;
  const int klv = b.max_levels + 1;
  TX *vals = (TX *)lds;
  int64_t *levent = (int64_t *)(lds + 8 * (size_t)b.S);
  int32_t *lvoff = (int32_t *)(levent + klv);
  WaitRec *recs = (WaitRec *)((char *)lvoff + (4 * (size_t)klv + 15) / 16 * 16);
  unsigned *seen = (unsigned *)(recs + kRecWindow);
  int32_t *ring = (int32_t *)(seen + kSeenSlots + 4);  // rows of the last two levels: [L & 1][i]
  const int64_t pad = b.pad_slot;

  for (int q = blockIdx.x; q < b.nb; q += gridDim.x) {
    const int64_t q0 = (int64_t)q * b.S;
    const int lb = b.lvbase[q];
    const int nl = b.lvbase[q + 1] - lb - 1;
    unsigned *prog = b.prog + (int64_t)q * kLevStride;
    int wr = b.wbase[q], win_lo = wr, win_hi = wr;  // the helper's next wait record and its window
    const int we = b.wbase[q + 1];
    for (int i = tid; i <= nl; i += BLOCK) {
      lvoff[i] = b.lvoff[lb + i];
      levent[i] = b.levent[lb + i];
    }
    for (int i = tid; i < kSeenSlots; i += BLOCK) seen[i] = 0;

    // stage 1 of pass `pass` of level L (L clamped to the block's last level)
    auto stage1 = [&](int L, int pass, Row &r) {
      L = L < nl ? L : nl - 1;
      const int p0 = lvoff[L], cnt = lvoff[L + 1] - p0;
      const int i = pass * rpp + rs;
      r.act = i < cnt;
      r.lp = r.act ? p0 + i : p0;
      const int64_t lev0 = levent[L];
      const int width = (int)((levent[L + 1] - lev0) / cnt);
      const int64_t pos = q0 + r.lp;
      r.row = b.prow[pos];
      r.len = b.plen[pos];
      r.dg = b.pdiag[pos];
      if constexpr (!FP) {
        r.mag = b.pmag[pos];
        r.sh = b.pshift[pos];
      }
#pragma unroll
      for (int j = 0; j < PRE; ++j) {
        const int k = gl + j * G;
        const int64_t e = (r.act && k < width) ? lev0 + i + (int64_t)k * cnt : pad;
        r.c[j] = b.ecode[e];
        if constexpr (FP) r.v[j] = b.evalf[e];
        else r.v[j] = b.eval[e];
      }
    };
    // stage 2: the right-hand side and the other blocks' values (their waits are taken)
    auto stage2 = [&](Row &r) {
      r.rhs = ld_coh(src + r.row);
#pragma unroll
      for (int j = 0; j < PRE; ++j) {
        const int k = gl + j * G;
        const bool cross = k < r.len && r.c[j] < 0;
        r.x[j] = ld_coh(dst + (cross ? -(int64_t)r.c[j] - 1 : (int64_t)r.row));
      }
    };
    // the row's value (the group's lane 0 holds it); L = the row's level
    auto compute = [&](const Row &r, int L) -> TX {
      if constexpr (FP) {
        double facc = 0.0;  // entries in CSR order: registers, then the rest
#pragma unroll
        for (int j = 0; j < PRE; ++j) {
          const int32_t c = r.c[j];
          const double xl = vals[c >= 0 ? c : 0];
          const double xv = c >= 0 ? xl : r.x[j];
          if (r.act && j < r.len) facc = facc + r.v[j] * xv;
        }
        if (!r.act) return 0.0;
        const int cnt = lvoff[L + 1] - lvoff[L];
        const int64_t e0 = levent[L] + (r.lp - lvoff[L]);
        for (int k = PRE; k < r.len; ++k) {  // entries beyond the registers, in order
          const int64_t e = e0 + (int64_t)k * cnt;
          const int32_t c = b.ecode[e];
          const double xv = c >= 0 ? vals[c] : ld_coh(dst + (-(int64_t)c - 1));
          facc = facc + b.evalf[e] * xv;
        }
        return (r.rhs - facc) / (double)r.dg;
      } else {
        Acc acc;
        acc.zero();
#pragma unroll
        for (int j = 0; j < PRE; ++j) {
          const int k = gl + j * G;
          const int32_t c = r.c[j];
          const int64_t xl = vals[c >= 0 ? c : 0];
          const int64_t xv = c >= 0 ? xl : r.x[j];
          if (r.act && k < r.len) acc.sub(b.narrow ? mul_w32(xv, (int32_t)r.v[j], ovf) : mulw(xv, r.v[j], ovf));
        }
        if (r.act) {
          const int cnt = lvoff[L + 1] - lvoff[L];
          const int64_t e0 = levent[L] + (r.lp - lvoff[L]);
          for (int k = gl + PRE * G; k < r.len; k += G) {  // entries beyond the registers
            const int64_t e = e0 + (int64_t)k * cnt;
            const int32_t c = b.ecode[e];
            const int64_t v = b.eval[e];
            const int64_t xv = c >= 0 ? vals[c] : ld_coh(dst + (-(int64_t)c - 1));
            acc.sub(mulw(xv, v, ovf));
          }
        }
        if constexpr (G > 1) {
          acc.lo = group_sum64<G>(acc.lo);
          acc.hi = group_sum64<G>(acc.hi);
        }
        int64_t y = 0;
        if (r.act && gl == 0) {
          acc.add(r.rhs);
          y = tdiv_magic(acc.value(ovf), r.dg, r.mag, r.sh, ovf);
        }
        return y;
      }
    };
    // the row's value into LDS and its row into the ring (or, for a level
    // the ring does not hold, straight to global memory)
    auto keep = [&](const Row &r, TX y, int L) {
      if (r.act && gl == 0) {
        vals[r.lp] = y;
        if (lvoff[L + 1] - lvoff[L] <= kRowRing) ring[(L & 1) * kRowRing + (r.lp - lvoff[L])] = r.row;
        else st_coh(dst + r.row, y);
      }
    };
    // helper: take the waits of level L (blocking)
    auto waits = [&](int L) {
      for (;;) {
        if (wr + 64 > win_hi && win_hi < we) {  // refill the window from the next record on
          const int cnt = we - wr < kRecWindow ? we - wr : kRecWindow;
          for (int i = lane; i < cnt; i += 64) recs[i] = b.wrec[wr + i];
          win_lo = wr;
          win_hi = wr + cnt;
        }
        const int r = wr + lane;
        WaitRec rec{0, 0, 0, 0};
        if (r < win_hi) rec = recs[r - win_lo];
        const bool mine = r < win_hi && rec.level == L;
        const unsigned long long got = __ballot(mine);
        if (mine) {
          const unsigned target = (unsigned)rec.need;
          const bool cached = rec.slot < kSeenSlots;
          unsigned v = cached ? seen[rec.slot] : 0u;
          for (int spin = 0; v < target; ++spin) {
            v = ld_coh(b.prog + (int64_t)rec.dep * kLevStride);
            if (v >= target) break;
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
    };
    // helper: level L's values from LDS to global memory (levels the ring held)
    auto store_level = [&](int L) {
      const int p0 = lvoff[L], cnt = lvoff[L + 1] - p0;
      if (cnt > kRowRing) return;
      for (int i = lane; i < cnt; i += 64) st_coh(dst + ring[(L & 1) * kRowRing + i], vals[p0 + i]);
    };
    auto publish = [&]() {
      wait_vm();
      if (lane == 0) __hip_atomic_fetch_add(prog, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    };

    // The helper and the compute wavefronts run separate loops with one
    // workgroup barrier per level each (a barrier counts per wavefront; the
    // branch is the same in every lane of a wavefront), so the loads the
    // helper waits for never mix with the compute lanes' loads in flight.
    if (helper) {
      waits(0);
      waits(1);
      __syncthreads();
      for (int L = 0; L < nl; ++L) {
        if (L >= 2) publish();          // level L - 2: its stores were issued a level ago
        if (L >= 1) store_level(L - 1);
        if (L + 2 < nl) waits(L + 2);   // two levels ahead: level L + 2's stage 2 is loaded in step L + 1
        __syncthreads();
      }
      if (nl >= 2) publish();
      store_level(nl - 1);
      publish();
    } else {
      __syncthreads();
      Row R0, R1, R2;
      if (computing) {
        stage1(0, 0, R0);
        stage1(1, 0, R1);
        stage2(R0);
        stage1(2, 0, R2);
      }
      // level L with A = its row (both stages loaded), B = level L + 1's
      // (stage 1 loaded); A's registers take level L + 3's stage 1
      auto step = [&](int L, Row &A, Row &B) {
        if (computing) {
          const TX y = compute(A, L);
          keep(A, y, L);
          for (int pass = 1; pass * rpp < lvoff[L + 1] - lvoff[L]; ++pass) {  // wider levels, A's registers
            stage1(L, pass, A);
            stage2(A);
            const TX yp = compute(A, L);
            keep(A, yp, L);
          }
          if (lvoff[L + 1] - lvoff[L] > kRowRing) wait_vm();  // stored by the compute lanes themselves
          stage2(B);
          stage1(L + 3, 0, A);
        }
        __syncthreads();
      };
      int L = 0;
      for (; L + 3 <= nl; L += 3) {
        step(L, R0, R1);
        step(L + 1, R1, R2);
        step(L + 2, R2, R0);
      }
      if (L < nl) step(L, R0, R1);
      if (L + 1 < nl) step(L + 1, R1, R2);
    }
  }
}

}  // namespace igm
