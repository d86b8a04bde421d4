// Grid-wide synchronisation for the persistent (cooperative) cycle kernel.
//
// A grid reduction adds, per workgroup, two 64-bit words with one relaxed
// agent-scope atomic each: (lo << 10) + 1 and (hi << 10) + 1 where lo/hi are
// the workgroup's exact partial sum split at bit 40. The low 10 bits of every
// word count its arrivals, so a word is complete when its count equals the
// number of workgroups mapped to it; no separate counter and no memory fence
// is needed. Arrivals are spread over kSyncGroups words per limb in separate
// cache lines (workgroup b uses word b % kSyncGroups) so the memory-side
// atomics do not serialise on one line; the first wavefront of every
// workgroup polls all words with one load per lane.
//
// A plain barrier (needed when workgroups read vectors other workgroups wrote)
// adds only to the lo words and wraps the arrival in agent-scope
// release/acquire fences.
//
// Every wait is bounded: after kSpinLimit polls the workgroup records a
// timeout and the kernel unwinds, so a launch can never hang.
#pragma once

#include "igm_device.hpp"

namespace igm {

#ifndef IGM_POLL_SLEEP
#define IGM_POLL_SLEEP 1  // s_sleep units (64 clocks) between polls
#endif

constexpr int kSpinLimit = 1 << 22;
static_assert(kSyncGroups == 8, "the sum decode reads one 8-lane half-row per limb");

struct GridSync {
  unsigned long long *words;  // [2 * kSyncGroups][cap]
  int cap;
  int nblocks;
  int next;
  int *timeout;  // device flag
};

// Workgroup-shared scratch of the reductions.
struct SyncShared {
  Acc wave[16];      // per-wavefront partial sums
  int64_t value;     // broadcast result
  int flag;          // broadcast overflow flag
  int abort;         // set on a timed-out wait
};

__device__ __forceinline__ unsigned expected_arrivals(int nblocks, int group) {
  return group < nblocks ? (unsigned)((nblocks - group + kSyncGroups - 1) / kSyncGroups) : 0u;
}

// Polls the words of sync slot s (lanes < nwords) until every word holds its
// expected count. Must be called by all 64 lanes of wavefront 0. Returns the
// word read by this lane (0 for lanes >= nwords) and sets *to on timeout.
__device__ __forceinline__ unsigned long long poll_words(const GridSync &gs, int s, int nwords, bool &to) {
  const int lane = threadIdx.x & 63;
  unsigned long long x = 0;
  unsigned expect = lane < nwords ? expected_arrivals(gs.nblocks, lane % kSyncGroups) : 0u;
  unsigned long long *p = gs.words + (size_t)lane * gs.cap + s;
  // one poll in flight, a short sleep between polls: more polling traffic
  // slows the arriving atomics down
  for (int spin = 0;; ++spin) {
    if (lane < nwords) x = __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const bool ok = (unsigned)(x & 1023ull) == expect;
    if (__all(ok)) break;
    if (spin >= kSpinLimit) { to = true; break; }
    __builtin_amdgcn_s_sleep(IGM_POLL_SLEEP);
  }
  return x;
}

__device__ __forceinline__ void record_timeout(const GridSync &gs, SyncShared &sh) {
  sh.abort = 1;
  __hip_atomic_store(gs.timeout, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Sum of one int64 over lanes 0..15 of a wavefront, returned to every lane
// (lanes 16..63 must hold 0).
__device__ __forceinline__ int64_t row0_sum(int64_t v) {
  v += dpp64<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp64<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp64<0x141>(v);  // row_half_mirror
  v += dpp64<0x140>(v);  // row_mirror
  return readlane64(v, 0);
}

// Exact grid sum of one Acc per thread, finished by `fin(S, ovf)` in wavefront
// 0 (S = the exact sum reduced to int64, ovf set if it left int64); the
// finished value and the overflow flag are broadcast to every thread.
// Threads of wavefronts 1.. run `side` while wavefront 0 waits.
template <int BLOCK, class Fin, class Side>
__device__ __forceinline__ int64_t grid_sum(GridSync &gs, Acc a, SyncShared &sh, Fin fin, Side side, bool &ovf) {
  static_assert(BLOCK / 64 <= 16, "one 16-lane row holds the wavefront partials");
  const int s = gs.next++;
  a = wave_sum(a);
  if ((threadIdx.x & 63) == 0) sh.wave[threadIdx.x >> 6] = a;
  __syncthreads();
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    Acc p;
    p.zero();
    if (lane < BLOCK / 64) p = sh.wave[lane];
    p.lo = row0_sum(p.lo);
    p.hi = row0_sum(p.hi);
    bool to = false;
    unsigned long long x = 0;
    if (!sh.abort) {
      if (lane == 0) {
        p.normalize();
        const int grp = blockIdx.x % kSyncGroups;
        __hip_atomic_fetch_add(gs.words + (size_t)grp * gs.cap + s, ((unsigned long long)p.lo << 10) + 1ull,
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(gs.words + (size_t)(kSyncGroups + grp) * gs.cap + s,
                               ((unsigned long long)p.hi << 10) + 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      x = poll_words(gs, s, 2 * kSyncGroups, to);
    }
    // lanes 0-7 hold the lo words, lanes 8-15 the hi words: three DPP steps
    // leave each 8-lane half-row's sum in its lanes (read from lanes 0 and 8)
    int64_t v = lane < kSyncGroups ? (int64_t)(x >> 10) : ((int64_t)x >> 10);
    v += dpp64<0xB1>(v);
    v += dpp64<0x4E>(v);
    v += dpp64<0x141>(v);
    Acc r;
    r.lo = readlane64(v, 0);
    r.hi = readlane64(v, kSyncGroups);
    if (lane == 0) {
      bool o = false;
      const int64_t S = r.value(o);
      sh.value = fin(S, o);
      sh.flag = o;
      if (to) record_timeout(gs, sh);
    }
  } else {
    side();
  }
  __syncthreads();
  if (sh.flag) ovf = true;
  return sh.value;
}

// Barrier that also publishes global-memory writes of every workgroup to
// every other workgroup (release before arriving, acquire after the wait).
// Threads of wavefronts 1.. run `side` while wavefront 0 waits; writes made by
// `side` are published by the next barrier.
template <class Side>
__device__ __forceinline__ void grid_barrier(GridSync &gs, SyncShared &sh, Side side) {
  const int s = gs.next++;
  __syncthreads();
  if (threadIdx.x < 64) {
    if (threadIdx.x == 0 && !sh.abort) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __hip_atomic_fetch_add(gs.words + (size_t)(blockIdx.x % kSyncGroups) * gs.cap + s, 1ull, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    }
    bool to = false;
    if (!sh.abort) poll_words(gs, s, kSyncGroups, to);
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (threadIdx.x == 0 && to) record_timeout(gs, sh);
  } else {
    side();
  }
  __syncthreads();
}

__device__ __forceinline__ void grid_barrier(GridSync &gs, SyncShared &sh) {
  grid_barrier(gs, sh, [] {});
}

// Barrier for data exchanged only through device-coherent stores and loads
// (ld_coh / st_coh): each wavefront waits for its own stores to complete,
// then the workgroups meet; no cache write-back or invalidation, so cached
// read-only data stays cached.
// Threads of wavefronts 1.. run `side` while wavefront 0 waits.
template <class Side>
__device__ __forceinline__ void grid_barrier_coh(GridSync &gs, SyncShared &sh, Side side) {
  const int s = gs.next++;
  wait_vm();
  __syncthreads();
  if (threadIdx.x < 64) {
    if (threadIdx.x == 0 && !sh.abort)
      __hip_atomic_fetch_add(gs.words + (size_t)(blockIdx.x % kSyncGroups) * gs.cap + s, 1ull, __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    bool to = false;
    if (!sh.abort) poll_words(gs, s, kSyncGroups, to);
    if (threadIdx.x == 0 && to) record_timeout(gs, sh);
  } else {
    side();
  }
  __syncthreads();
}

__device__ __forceinline__ void grid_barrier_coh(GridSync &gs, SyncShared &sh) {
  grid_barrier_coh(gs, sh, [] {});
}

// Workgroup sum of one Acc per thread; result valid in thread 0 only.
template <int BLOCK>
__device__ __forceinline__ Acc block_sum(Acc a, Acc *sh_wave) {
  a = wave_sum(a);
  const int wid = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0) sh_wave[wid] = a;
  __syncthreads();
  Acc t;
  t.zero();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < BLOCK / 64; ++k) t.add(sh_wave[k]);
  }
  return t;
}

}  // namespace igm
