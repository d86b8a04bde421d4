// Synchronisation inside a "team": the T workgroups (1 <= T <= kTeamMax) of
// the batched solver that share one system.
//
// T == 1 (the common case) never touches global memory: every reduction is a
// workgroup reduction through LDS and every barrier is __syncthreads().
//
// T > 1: member q publishes payload word p by one relaxed agent-scope atomic
// add of (payload << 10) + 1 to word [slot][p][q] of the system's exchange
// area; lane q of the first wavefront of every member then polls member q's
// words until each shows one new arrival, so every lane ends up holding one
// member's payload. The words are never cleared: every lane remembers the
// value it last saw in each slot (in LDS) and decodes the difference. A slot
// is reused kTeamSlots exchanges later; by then every member has finished
// reading it, because no member can start exchange e + 2 before all members
// arrived at exchange e + 1. The area must be zero when a system's first
// member starts (it is cleared before each launch). Barriers that publish
// vectors to other members wrap the exchange in agent-scope release/acquire
// fences. Every wait is bounded (kSpinLimit).
#pragma once

#include "igm_sync.hpp"

namespace igm {

constexpr int kTeamMax = 256;   // workgroups per system
constexpr int kTeamSlots = 2;   // exchanges before a slot is reused
constexpr int kTeamPay = 4;     // payload words per exchange
constexpr int kTeamWords = kTeamPay * kTeamMax;  // words per slot

struct TeamShared {
  Acc wave[16];                                             // per-wavefront partial sums
  unsigned long long part[4][16];                           // per-wavefront partials of team_reduce
  unsigned long long prev[kTeamSlots][kTeamPay][kTeamMax];  // last value seen per exchange word
  unsigned long long res[4];                                // team_reduce results
  int64_t value;                                            // broadcast result of team_sum
  int flag;                                                 // broadcast overflow flag of team_sum
  int abort;                                                // a wait timed out
};

struct Team {
  unsigned long long *words;  // [kTeamSlots][kTeamPay][kTeamMax]
  int T, member, e;
  int *timeout;               // device flag of the launch
};

__device__ __forceinline__ void team_init(TeamShared &sh) {
  for (int i = threadIdx.x; i < kTeamSlots * kTeamWords; i += blockDim.x) (&sh.prev[0][0][0])[i] = 0;
  if (threadIdx.x == 0) {
    sh.abort = 0;
    sh.flag = 0;
  }
}

// One exchange among the T > 1 members; wavefront 0 only (all 64 lanes).
// u[0..P) are this member's payload words (wave-uniform). SUM: each word
// |u| < 2^53, and on return lane q holds the sum of the words of members
// q, q + 64, q + 128, ... (< T). MAX: each word is any 64-bit value (sent as
// two 32-bit halves, 2P <= kTeamPay) and lane q receives the maximum over the
// same members. Sets `to` on timeout.
template <int P, bool MAX>
__device__ __forceinline__ void team_exchange(Team &tm, TeamShared &sh, unsigned long long (&u)[P], bool &to) {
  constexpr int W = MAX ? 2 * P : P;  // words per member
  static_assert(P >= 1 && W <= kTeamPay, "payload words");
  const int q = threadIdx.x & 63;
  const int slot = tm.e % kTeamSlots;
  tm.e += 1;
  unsigned long long *base = tm.words + slot * kTeamWords;
  unsigned long long wv[W];
#pragma unroll
  for (int p = 0; p < P; ++p) {
    if (MAX) {
      wv[2 * p] = u[p] & 0xFFFFFFFFull;
      wv[2 * p + 1] = u[p] >> 32;
    } else {
      wv[p] = u[p];
    }
  }
  if (q == (tm.member & 63)) {
#pragma unroll
    for (int w = 0; w < W; ++w)
      __hip_atomic_fetch_add(base + w * kTeamMax + tm.member, (wv[w] << 10) + 1ull, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
  }
  constexpr int G = kTeamMax / 64;  // member groups per lane
  unsigned long long d[G][W];
#pragma unroll
  for (int g = 0; g < G; ++g)
#pragma unroll
    for (int w = 0; w < W; ++w) d[g][w] = 0;
  for (int spin = 0;; ++spin) {
    bool ok = true;
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int mq = q + 64 * g;
      if (mq < tm.T) {
#pragma unroll
        for (int w = 0; w < W; ++w) {
          d[g][w] = __hip_atomic_load(base + w * kTeamMax + mq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) -
                    sh.prev[slot][w][mq];
          ok = ok && (d[g][w] & 1023ull) == 1ull;
        }
      }
    }
    if (__all(ok)) break;
    if (spin >= kSpinLimit) { to = true; break; }
    __builtin_amdgcn_s_sleep(IGM_POLL_SLEEP);
  }
#pragma unroll
  for (int p = 0; p < P; ++p) u[p] = 0;
#pragma unroll
  for (int g = 0; g < G; ++g) {
    const int mq = q + 64 * g;
    if (mq < tm.T) {
      unsigned long long pay[W];
#pragma unroll
      for (int w = 0; w < W; ++w) {
        sh.prev[slot][w][mq] += d[g][w];
        pay[w] = (unsigned long long)((int64_t)d[g][w] >> 10);
      }
#pragma unroll
      for (int p = 0; p < P; ++p) {
        if (MAX) {
          const unsigned long long v = pay[2 * p] | (pay[2 * p + 1] << 32);
          u[p] = v > u[p] ? v : u[p];
        } else {
          u[p] += pay[p];
        }
      }
    }
  }
}

__device__ __forceinline__ void team_abort(Team &tm, TeamShared &sh) {
  sh.abort = 1;
  __hip_atomic_store(tm.timeout, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sum over each 16-lane row of a wavefront, left in every lane of the row.
__device__ __forceinline__ int64_t row16_sum(int64_t v) {
  v += dpp64<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp64<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp64<0x141>(v);  // row_half_mirror
  v += dpp64<0x140>(v);  // row_mirror
  return v;
}

// Exact team sum of one Acc per thread, finished by fin(S, ovf) in one lane
// and broadcast (value and overflow flag) to every thread of the workgroup.
// Threads of wavefronts 1.. run `side` meanwhile.
template <int BLOCK, class Fin, class Side>
__device__ __forceinline__ int64_t team_sum(Team &tm, Acc a, TeamShared &sh, Fin fin, Side side, bool &ovf) {
  static_assert(BLOCK / 64 <= 16, "one 16-lane row holds the wavefront partials");
  a = wave_sum(a);
  if ((threadIdx.x & 63) == 0) sh.wave[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    Acc p;
    p.zero();
    if (lane < BLOCK / 64) p = sh.wave[lane];
    p.lo = readlane64(row16_sum(p.lo), 0);
    p.hi = readlane64(row16_sum(p.hi), 0);
    bool to = false;
    if (tm.T > 1 && !sh.abort) {
      p.normalize();  // lo in [0, 2^40)
      unsigned long long u[2] = {(unsigned long long)p.lo, (unsigned long long)p.hi};
      team_exchange<2, false>(tm, sh, u, to);  // lane q: limbs of members q, q + 64, ...
      p.lo = wave_sum64((int64_t)u[0]);
      p.hi = wave_sum64((int64_t)u[1]);
    }
    if (lane == 0) {
      bool o = false;
      const int64_t S = p.value(o);
      sh.value = fin(S, o);
      sh.flag = o;
      if (to) team_abort(tm, sh);
    }
  } else {
    side();
  }
  __syncthreads();
  if (sh.flag) ovf = true;
  return sh.value;
}

// Barrier of the team that also publishes global-memory writes to the other
// members. Threads of wavefronts 1.. run `side` while wavefront 0 waits.
template <class Side>
__device__ __forceinline__ void team_barrier(Team &tm, TeamShared &sh, Side side) {
  __syncthreads();
  if (threadIdx.x < 64) {
    if (tm.T > 1 && !sh.abort) {
      bool to = false;
      unsigned long long u[1] = {0};
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      team_exchange<1, false>(tm, sh, u, to);
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      if (threadIdx.x == 0 && to) team_abort(tm, sh);
    }
  } else {
    side();
  }
  __syncthreads();
}

__device__ __forceinline__ void team_barrier(Team &tm, TeamShared &sh) {
  team_barrier(tm, sh, [] {});
}

// Team barrier for data exchanged only through device-coherent stores and
// loads (ld_coh / st_coh): each wavefront waits for its own stores to
// complete, then the members meet; no cache write-back or invalidation.
__device__ __forceinline__ void team_barrier_coh(Team &tm, TeamShared &sh) {
  wait_vm();
  __syncthreads();
  if (threadIdx.x < 64 && tm.T > 1 && !sh.abort) {
    bool to = false;
    unsigned long long u[1] = {0};
    team_exchange<1, false>(tm, sh, u, to);
    if (threadIdx.x == 0 && to) team_abort(tm, sh);
  }
  __syncthreads();
}

template <bool MAX>
__device__ __forceinline__ unsigned long long op_u64(unsigned long long a, unsigned long long b) {
  return MAX ? (a > b ? a : b) : a + b;
}

// Reduction over `width` consecutive lanes (a power of two <= 64) with xor
// shuffles; every lane of each group ends with its group's result.
template <bool MAX>
__device__ __forceinline__ unsigned long long lanes_reduce(unsigned long long v, int width) {
  for (int o = width >> 1; o > 0; o >>= 1)
    v = op_u64<MAX>(v, (unsigned long long)__shfl_xor((long long)v, o, 64));
  return v;
}

// Team reduction of P unsigned words per thread (sum, or max), result in every
// thread. Sums: each workgroup's partial of each word must stay below 2^53.
// Maxima: any 64-bit value (sent as two 32-bit halves), P <= 2.
template <int BLOCK, int P, bool MAX>
__device__ __forceinline__ void team_reduce(Team &tm, TeamShared &sh, unsigned long long (&v)[P]) {
  static_assert(P >= 1 && P <= (MAX ? 2 : 4), "payload words");
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int p = 0; p < P; ++p) {
    v[p] = lanes_reduce<MAX>(v[p], 64);
    if (lane == 0) sh.part[p][threadIdx.x >> 6] = v[p];
  }
  __syncthreads();
  if (threadIdx.x < 64) {
    unsigned long long r[P];
#pragma unroll
    for (int p = 0; p < P; ++p) r[p] = lanes_reduce<MAX>(lane < BLOCK / 64 ? sh.part[p][lane] : 0ull, 64);
    if (tm.T > 1 && !sh.abort) {
      bool to = false;
      team_exchange<P, MAX>(tm, sh, r, to);
#pragma unroll
      for (int p = 0; p < P; ++p) r[p] = lanes_reduce<MAX>(r[p], 64);
      if (lane == 0 && to) team_abort(tm, sh);
    }
    if (lane == 0) {
#pragma unroll
      for (int p = 0; p < P; ++p) sh.res[p] = r[p];
    }
  }
  __syncthreads();
#pragma unroll
  for (int p = 0; p < P; ++p) v[p] = sh.res[p];
  __syncthreads();
}

}  // namespace igm
