/*
 * Fixed-point primitives of the integer GMRES solver (Sec. V-B of the paper).
 * TEST INFRASTRUCTURE ONLY (see orc.h).
 *
 * Every operation is computed exactly in __int128 and then reduced to int64.
 */
#include <math.h>
#include "orc.h"

typedef __int128 i128;

static int fits64(i128 x) { return x >= (i128)INT64_MIN && x <= (i128)INT64_MAX; }

/* Exact value mod 2^64 as a two's complement int64 (the hardware result). */
static int64_t wrap64(i128 x) { return (int64_t)(uint64_t)(unsigned __int128)x; }

/* Right shift by b bits = division by 2^b rounded toward minus infinity
 * (Sec. V-A: shifts are multiplications/divisions by powers of two; the
 * paper's C code on x86 shifts signed words arithmetically). */
int64_t orc_asr(int64_t x, int32_t b) {
  if (b <= 0) return x;
  if (b > 63) b = 63;
  i128 d = (i128)1 << b;
  i128 q = (i128)x / d; /* truncates toward zero */
  if ((i128)x % d != 0 && x < 0) q -= 1;
  return (int64_t)q;
}

int64_t orc_shl(int64_t x, int32_t b, int32_t *ovf) {
  if (b <= 0) return x;
  if (b > 63) b = 63;
  i128 r = (i128)x * ((i128)1 << b);
  if (!fits64(r)) *ovf = 1;
  return wrap64(r);
}

int64_t orc_sc(int64_t x, int32_t e, int32_t *ovf) {
  return e >= 0 ? orc_shl(x, e, ovf) : orc_asr(x, -e);
}

/* Integer division instruction of C: quotient truncated toward zero. */
int64_t orc_tdiv(int64_t a, int64_t d, int32_t *ovf) {
  if (d == 0) { *ovf = 1; return 0; }
  i128 q = (i128)a / (i128)d;
  if (!fits64(q)) *ovf = 1; /* only INT64_MIN / -1 */
  return wrap64(q);
}

/* Babylonian (Newton) iteration on integers, started above the root: the
 * iterates decrease strictly until they reach floor(sqrt(x)). A negative
 * argument (only possible after an overflow) gives 0. */
int64_t orc_isqrt(int64_t x) {
  if (x <= 0) return 0;
  unsigned __int128 X = (unsigned __int128)x;
  unsigned __int128 r = X; /* any start >= sqrt(x) works */
  if (r > ((unsigned __int128)1 << 32)) r = (unsigned __int128)1 << 32; /* sqrt(2^63) < 2^32 */
  for (;;) {
    unsigned __int128 nr = (r + X / r) / 2;
    if (nr >= r) break;
    r = nr;
  }
  return (int64_t)r;
}

/* C cast double -> int64 (truncation toward zero); |y| must be < 2^63. */
int64_t orc_trunc(double y, int32_t *range_err) {
  if (!(y >= -9223372036854775808.0 && y < 9223372036854775808.0)) {
    *range_err = 1;
    return 0;
  }
  return (int64_t)y;
}

static int64_t mul_exact(int64_t a, int64_t b, int32_t *ovf) {
  i128 p = (i128)a * (i128)b;
  if (!fits64(p)) *ovf = 1;
  return wrap64(p);
}

/* Fixed-point multiplication, eq. (c1c2): both operands shifted right by their
 * beta, multiplied, and the Q(2df - b1 - b2) product brought back to Q df. */
int64_t orc_mul(int64_t t1, int64_t t2, int32_t b1, int32_t b2, int32_t df, int32_t *ovf) {
  int64_t p = mul_exact(orc_asr(t1, b1), orc_asr(t2, b2), ovf);
  return orc_asr(p, df - b1 - b2);
}

/* Fixed-point division (Sec. V-B.3): t1 * 2^b1 divided (C division) by
 * t2 / 2^b2, then scaled by 2^(df - b1 - b2). *zero is set when the shifted
 * denominator is 0. */
int64_t orc_div(int64_t t1, int64_t t2, int32_t b1, int32_t b2, int32_t df, int32_t *ovf, int32_t *zero) {
  int64_t den = orc_asr(t2, b2);
  if (den == 0) { *zero = 1; return 0; }
  int64_t num = orc_shl(t1, b1, ovf);
  int64_t q = orc_tdiv(num, den, ovf);
  return orc_sc(q, df - b1 - b2, ovf);
}

/* Exact sum of the wrapped int64 products; overflow if the sum leaves int64. */
static int64_t finish_sum(i128 s, int32_t *ovf) {
  if (!fits64(s)) *ovf = 1;
  return wrap64(s);
}

/* Inner product (Sec. V-C.1, Table II): only the first operand w is
 * shifted (beta_2 = 0), products are summed in Q(2df - b), and the sum is
 * shifted once by df - b to return to Q df. */
int64_t orc_dot(int64_t n, const int64_t *w, const int64_t *v, int32_t b, int32_t df, int32_t *ovf) {
  i128 s = 0;
  for (int64_t l = 0; l < n; ++l) s += mul_exact(orc_asr(w[l], b), v[l], ovf);
  return orc_asr(finish_sum(s, ovf), df - b);
}

/* Norm (Sec. V-C.2, Table II): sum of asr(w, b)^2 in Q(2df - 2b),
 * integer square root (Q(df - b)), then times 2^b (= 2^(df - (2df-2b)/2)). */
int64_t orc_norm(int64_t n, const int64_t *w, int32_t b, int32_t df, int32_t *ovf) {
  (void)df;
  i128 s = 0;
  for (int64_t l = 0; l < n; ++l) {
    int64_t t = orc_asr(w[l], b);
    s += mul_exact(t, t, ovf);
  }
  int64_t sq = finish_sum(s, ovf);
  return orc_shl(orc_isqrt(sq), b, ovf);
}

/* Gram-Schmidt update (Table II): w_l -= asr(asr(h, b) * v_l, df - b) for every l, in
 * place; only h is shifted (Sec. V-D.2). */
void orc_axpy(int64_t n, int64_t *w, const int64_t *v, int64_t h, int32_t b, int32_t df, int32_t *ovf) {
  int64_t hs = orc_asr(h, b);
  for (int64_t l = 0; l < n; ++l) {
    int64_t q = orc_asr(mul_exact(hs, v[l], ovf), df - b);
    i128 d = (i128)w[l] - q;
    if (!fits64(d)) *ovf = 1;
    w[l] = wrap64(d);
  }
}

/* Normalisation (Sec. V-B.3): v_l = sc(tdiv(shl(w_l, b1), den), df - b1 - b2) with
 * den = asr(h, b2) != 0 (the caller checks for 0). */
void orc_normalize(int64_t n, const int64_t *w, int64_t den, int32_t b1, int32_t b2, int32_t df, int64_t *v,
                   int32_t *ovf) {
  for (int64_t l = 0; l < n; ++l) {
    int64_t q = orc_tdiv(orc_shl(w[l], b1, ovf), den, ovf);
    v[l] = orc_sc(q, df - b1 - b2, ovf);
  }
}
