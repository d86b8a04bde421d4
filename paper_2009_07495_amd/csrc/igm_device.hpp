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

// floor(sqrt(x)) by the bitwise (digit-by-digit) method, integers only;
// x <= 0 gives 0.
__device__ __forceinline__ int64_t isqrt64(int64_t xs) {
  if (xs <= 0) return 0;
  uint64_t x = (uint64_t)xs, r = 0, bit = 1ull << 62;
  while (bit > x) bit >>= 2;
  while (bit) {
    if (x >= r + bit) { x -= r + bit; r = (r >> 1) + bit; }
    else r >>= 1;
    bit >>= 2;
  }
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

__device__ __forceinline__ int64_t shfl_xor64(int64_t v, int o) { return __shfl_xor(v, o, 64); }

// Sum of an Acc over the 64 lanes of a wavefront (result valid in every lane).
__device__ __forceinline__ Acc wave_sum(Acc a) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    a.lo += shfl_xor64(a.lo, o);
    a.hi += shfl_xor64(a.hi, o);
  }
  return a;
}

__device__ __forceinline__ unsigned long long dbits(double d) { return (unsigned long long)__double_as_longlong(d); }

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
