// Per-row pieces of the integer kernels shared by the persistent cycle kernel
// and the standalone kernels.
#pragma once

#include "igm_device.hpp"
#include "igm_internal.hpp"

namespace igm {

// Line 5 for one row (Sec. V-C.3, eq. (matvec)): z = A_0 v + sum_l
// asr(A_l v, alpha_l), the matrices in SELL-64 layout (slice = 64 rows stored
// column-major, so the 64 lanes of a wavefront read consecutive words). Every
// sum is exact; `ovf` is set if a product, a term or the total leaves int64.
// `a` is any record with the SELL fields of CycleArgs.
template <class A>
__device__ __forceinline__ int64_t spmv_row(const A &a, int64_t row, const int64_t *__restrict__ v,
                                            int nterms, bool &ovf) {
  const int64_t slice = row >> 6;
  const int64_t base = a.sell_off[slice] + (row & 63);
  const int wdt = a.sell_w[slice];
  Acc tot;
  tot.zero();
  for (int l = 0; l < nterms; ++l) {
    const int64_t *__restrict__ val = a.sell_val[l];
    Acc acc;
    acc.zero();
    for (int e = 0; e < wdt; ++e) {
      const int64_t pos = base + (int64_t)e * 64;
      acc.add(mulw(val[pos], v[a.sell_col[pos]], ovf));
    }
    int64_t t = acc.value(ovf);
    if (l > 0) t = asr(t, a.alpha[l]);
    tot.add(t);
  }
  return tot.value(ovf);
}

// Line 5' forward substitution for one row: y_i = tdiv(z_i - sum_{j<i}
// Lbar_ij y_j, Lbar_ii).
template <class A>
__device__ __forceinline__ int64_t lower_row(const A &a, int64_t row, int64_t zi,
                                             const int64_t *__restrict__ y, bool &ovf) {
  Acc acc;
  acc.zero();
  acc.add(zi);
  for (int64_t e = a.lptr[row]; e < a.lptr[row + 1]; ++e) acc.sub(mulw(y[a.lcol[e]], a.lval[e], ovf));
  return tdiv(acc.value(ovf), a.ldiag[row], ovf);
}

// Line 5' backward substitution for one row: u_i = tdiv(y_i - sum_{j>i}
// Ubar_ij u_j, Ubar_ii).
template <class A>
__device__ __forceinline__ int64_t upper_row(const A &a, int64_t row, int64_t yi,
                                             const int64_t *__restrict__ u, bool &ovf) {
  Acc acc;
  acc.zero();
  acc.add(yi);
  for (int64_t e = a.uptr[row]; e < a.uptr[row + 1]; ++e) acc.sub(mulw(u[a.ucol[e]], a.uval[e], ovf));
  return tdiv(acc.value(ovf), a.udiag[row], ovf);
}

// Line 11 for one element: sc(tdiv(shl(w, b1), den), df - b1 - b2).
__device__ __forceinline__ int64_t normalize_elem(int64_t w, int64_t den, int b1, int sc_exp, bool &ovf) {
  return scale2(tdiv(shl(w, b1, ovf), den, ovf), sc_exp, ovf);
}

}  // namespace igm
