// Device-side fixed-point arithmetic for the integer GMRES kernels (gfx950).
//
// Word semantics (Sec. II and V-B of the paper): int64 two's complement
// Q(63-df).df numbers. Right shifts are arithmetic (floor), divisions truncate
// toward zero, casts from double truncate toward zero. Every operation reports
// whether its exact result left int64 ("overflow"); the stored word is the
// exact result mod 2^64, so results after an overflow are still a pure
// function of the inputs. Sums of products are exact (the order of the terms
// does not matter), which is what lets any reduction tree give the same bits.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace igm {

constexpr int64_t kNoEvent = INT64_MAX;
constexpr int kLimbBits = 40;
constexpr uint64_t kLimbMask = (1ull << kLimbBits) - 1;

__device__ __forceinline__ int64_t ev_code(int j, int stage, int sub) {
  return ((int64_t)j << 24) | ((int64_t)stage << 16) | (int64_t)sub;
}

// floor(x / 2^b), 0 <= b <= 63
__device__ __forceinline__ int64_t asr(int64_t x, int b) { return x >> b; }

// x * 2^b with overflow flag, 0 <= b <= 63
__device__ __forceinline__ int64_t shl(int64_t x, int b, bool &ovf) {
  int64_t r = (int64_t)((uint64_t)x << b);
  if ((r >> b) != x) ovf = true;
  return r;
}

__device__ __forceinline__ int64_t scale2(int64_t x, int e, bool &ovf) {
  return e >= 0 ? shl(x, e, ovf) : asr(x, -e);
}

// exact product reduced mod 2^64, flag if it leaves int64
__device__ __forceinline__ int64_t mulc(int64_t a, int64_t b, bool &ovf) {
  int64_t p;  // the builtins store the product reduced mod 2^64
  if (__builtin_mul_overflow(a, b, &p)) ovf = true;
  return p;
}

// Same result as mulc for a "wide" operand a and a "narrow" operand b (a basis
// vector element or a rotation coefficient): when a is in [-2^32+1, 2^32] and
// b in [-2^31, 2^31) the product cannot leave int64 (|a b| <= 2^63 with
// equality only at -2^63), so a plain 64-bit multiply is exact; otherwise the
// full 128-bit check runs.
__device__ __forceinline__ int64_t mulw(int64_t a, int64_t b, bool &ovf) {
  const bool fits = ((uint64_t)(a + 0xFFFFFFFFll) >> 33) == 0 && ((uint64_t)(b + 0x80000000ll) >> 32) == 0;
  if (__builtin_expect(fits, 1)) return (int64_t)((uint64_t)a * (uint64_t)b);
  return mulc(a, b, ovf);
}

// t * t with the overflow check: exact iff |t| <= floor(sqrt(2^63 - 1)).
__device__ __forceinline__ int64_t sqrc(int64_t t, bool &ovf) {
  if ((uint64_t)(t + 3037000499ll) > 6074000998ull) ovf = true;
  return (int64_t)((uint64_t)t * (uint64_t)t);
}

__device__ __forceinline__ int64_t addc(int64_t a, int64_t b, bool &ovf) {
  int64_t r;
  if (__builtin_add_overflow(a, b, &r)) ovf = true;
  return r;
}

__device__ __forceinline__ int64_t subc(int64_t a, int64_t b, bool &ovf) {
  int64_t r;
  if (__builtin_sub_overflow(a, b, &r)) ovf = true;
  return r;
}

// C division (truncation toward zero); d == 0 gives 0 with the flag set,
// INT64_MIN / -1 wraps with the flag set.
__device__ __forceinline__ int64_t tdiv(int64_t a, int64_t d, bool &ovf) {
  if (d == 0) { ovf = true; return 0; }
  if (d == -1) {
    if (a == INT64_MIN) ovf = true;
    return (int64_t)(0ull - (uint64_t)a);
  }
  return a / d;
}

// tdiv for a divisor that is usually a power of two (the cast Jacobi
// diagonals of diagonally dominant stencil matrices): for d = 2^k > 0 the
// truncating quotient is (a + (d - 1 if a < 0)) >> k, exactly; other divisors
// take the general division.
__device__ __forceinline__ int64_t tdiv_diag(int64_t a, int64_t d, bool &ovf) {
  if (d > 0 && (d & (d - 1)) == 0) return (a + ((a >> 63) & (d - 1))) >> __builtin_ctzll((uint64_t)d);
  return tdiv(a, d, ovf);
}

// floor(sqrt(x)); x <= 0 gives 0. A double-precision estimate (within one of
// the root, which is below 2^31.5) corrected with exact integer squares,
// which fit in 64 bits; the correction makes the result exact whatever the
// estimate.
__device__ __forceinline__ int64_t isqrt64(int64_t xs) {
  if (xs <= 0) return 0;
  const uint64_t x = (uint64_t)xs;
  uint64_t r = (uint64_t)sqrt((double)x);
  if (r > 3037000499ull) r = 3037000499ull;  // floor(sqrt(2^63 - 1))
  while (r * r > x) --r;
  while ((r + 1) * (r + 1) <= x) ++r;
  return (int64_t)r;
}

// Exact signed accumulator for sums of int64 words: value = hi * 2^40 + lo
// with lo summing 40-bit non-negative limbs. Thousands of terms per thread or
// workgroup stay far inside int64 for both parts.
struct Acc {
  int64_t lo, hi;
  __device__ __forceinline__ void zero() { lo = 0; hi = 0; }
  __device__ __forceinline__ void add(int64_t p) {
    lo += (int64_t)((uint64_t)p & kLimbMask);
    hi += p >> kLimbBits;
  }
  __device__ __forceinline__ void sub(int64_t p) {
    lo -= (int64_t)((uint64_t)p & kLimbMask);
    hi -= p >> kLimbBits;
  }
  __device__ __forceinline__ void add(const Acc &o) { lo += o.lo; hi += o.hi; }
  __device__ __forceinline__ void normalize() {
    hi += lo >> kLimbBits;
    lo &= (int64_t)kLimbMask;
  }
  // exact value; returns the word mod 2^64 and flags values outside int64
  __device__ __forceinline__ int64_t value(bool &ovf) const {
    __int128 v = (__int128)hi * ((__int128)1 << kLimbBits) + (__int128)lo;
    if (v != (__int128)(int64_t)v) ovf = true;
    return (int64_t)v;
  }
};

// 64-bit DPP lane move (both 32-bit halves), all lanes active.
template <int CTRL>
__device__ __forceinline__ int64_t dpp64(int64_t v) {
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)(uint64_t)v, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(uint32_t)((uint64_t)v >> 32), CTRL, 0xF, 0xF, false);
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
}

__device__ __forceinline__ int64_t readlane64(int64_t v, int lane) {
  const int lo = __builtin_amdgcn_readlane((int)(uint32_t)(uint64_t)v, lane);
  const int hi = __builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), lane);
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint64_t)(uint32_t)lo);
}

// Sum of an int64 over the 64 lanes of a wavefront (every lane active; the
// result is wave-uniform). DPP quad xor-1, quad xor-2, half-row mirror and row
// mirror leave each 16-lane row's sum in all its lanes; the four row sums are
// then read out with v_readlane. Integer addition is exact and associative, so
// the order of the partial sums does not matter.
__device__ __forceinline__ int64_t wave_sum64(int64_t v) {
  v += dpp64<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp64<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp64<0x141>(v);  // row_half_mirror
  v += dpp64<0x140>(v);  // row_mirror
  return readlane64(v, 0) + readlane64(v, 16) + readlane64(v, 32) + readlane64(v, 48);
}

// Sum of an int64 over each group of G consecutive lanes (G = 1, 2, 4, 8, 16,
// 64), returned to every lane of the group; every lane of the wavefront active.
template <int G>
__device__ __forceinline__ int64_t group_sum64(int64_t v) {
  static_assert(G == 1 || G == 2 || G == 4 || G == 8 || G == 16 || G == 64, "lane groups");
  if constexpr (G == 64) return wave_sum64(v);
  if constexpr (G >= 2) v += dpp64<0xB1>(v);   // quad_perm [1,0,3,2]
  if constexpr (G >= 4) v += dpp64<0x4E>(v);   // quad_perm [2,3,0,1]
  if constexpr (G >= 8) v += dpp64<0x141>(v);  // row_half_mirror
  if constexpr (G >= 16) v += dpp64<0x140>(v); // row_mirror
  return v;
}

__device__ __forceinline__ Acc wave_sum(Acc a) {
  a.lo = wave_sum64(a.lo);
  a.hi = wave_sum64(a.hi);
  return a;
}

__device__ __forceinline__ unsigned long long dbits(double d) { return (unsigned long long)__double_as_longlong(d); }

// Device-coherent accesses (agent scope): they bypass the caches that are
// private to one chiplet, so values written by one workgroup are seen by all
// others once the writer's stores have completed, without cache write-back
// or invalidation. Used for the vectors the level-scheduled triangular
// sweeps exchange between workgroups.
__device__ __forceinline__ int64_t ld_coh(const int64_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_coh(int64_t *p, int64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_coh(const double *p) {
  return __longlong_as_double(__hip_atomic_load((const long long *)p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT));
}
__device__ __forceinline__ void st_coh(double *p, double v) {
  __hip_atomic_store((long long *)p, __double_as_longlong(v), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned ld_coh(const unsigned *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_coh(unsigned *p, unsigned v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// Records overflow event `code` in *first (the smallest code wins) once per
// wavefront in which any active lane saw an overflow, so a kernel whose rows
// all overflow does not serialise on one atomic word. `code` must be the same
// in every lane.
__device__ __forceinline__ void note_event(bool o, int64_t *first, int64_t code) {
  const unsigned long long m = __ballot(o);
  if (m && (int)(threadIdx.x & 63) == __ffsll((long long)m) - 1) atomicMin((long long *)first, (long long)code);
}

// Waits until this wavefront's outstanding memory operations have completed
// (s_waitcnt vmcnt(0); the other counters are left at their maxima).
__device__ __forceinline__ void wait_vm() { __builtin_amdgcn_s_waitcnt(0x0F70); }

// floor(q * 2^96) for 0 <= q <= 1 as a 128-bit integer (q a double).
__device__ __forceinline__ unsigned __int128 fix96(double q) {
  uint64_t b = dbits(q);
  int e = (int)((b >> 52) & 0x7ff);
  if (e == 0) return 0;  // zero or subnormal: below 2^-1022, contributes 0
  uint64_t mant = (b & ((1ull << 52) - 1)) | (1ull << 52);
  int sh = e - 1075 + 96;  // q = mant * 2^(e-1075)
  if (sh >= 0) return (unsigned __int128)mant << sh;
  if (sh <= -64) return 0;
  return (unsigned __int128)(mant >> (-sh));
}

// Round a 128-bit unsigned integer to the nearest double (ties to even).
__device__ __forceinline__ double u128_to_double_rn(unsigned __int128 v) {
  uint64_t hi = (uint64_t)(v >> 64), lo = (uint64_t)v;
  if (hi == 0 && lo < (1ull << 53)) return (double)lo;
  int p = hi ? 127 - __clzll(hi) : 63 - __clzll(lo);  // index of the leading bit
  int sh = p - 52;
  uint64_t mant = (uint64_t)(v >> sh);
  unsigned __int128 rest = v & ((((unsigned __int128)1) << sh) - 1);
  unsigned __int128 half = ((unsigned __int128)1) << (sh - 1);
  if (rest > half || (rest == half && (mant & 1))) {
    mant += 1;
    if (mant == (1ull << 53)) { mant >>= 1; sh += 1; }
  }
  return ldexp((double)mant, sh);
}

}  // namespace igm
