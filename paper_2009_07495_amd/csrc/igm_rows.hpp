// Per-row pieces of the integer kernels shared by the persistent cycle kernel
// and the standalone kernels.
#pragma once

#include "igm_device.hpp"
#include "igm_internal.hpp"

namespace igm {

// Entries of one sparse row are visited in chunks: the column indices and
// values of a chunk are loaded together, then its gathered operands, then
// the chunk is consumed in ascending entry order. One row thus waits for two
// memory round trips per chunk instead of one per entry, and every sum keeps
// the order of the row (FP64 sums round exactly as the plain loop).
constexpr int kRowChunk = 8;

// op(val[e], x[col[e]]) for e = lo .. hi-1 in increasing order; COH: the
// gathered x are read with device-coherent loads.
template <bool COH = false, class TV, class TX, class Op>
__device__ __forceinline__ void row_visit(int64_t lo, int64_t hi, const int32_t *__restrict__ col,
                                          const TV *__restrict__ val, const TX *x, Op op) {
  for (int64_t e0 = lo; e0 < hi; e0 += kRowChunk) {
    int32_t c[kRowChunk];
    TV v[kRowChunk];
    TX xv[kRowChunk];
#pragma unroll
    for (int k = 0; k < kRowChunk; ++k)
      if (e0 + k < hi) {
        c[k] = col[e0 + k];
        v[k] = val[e0 + k];
      }
#pragma unroll
    for (int k = 0; k < kRowChunk; ++k)
      if (e0 + k < hi) xv[k] = COH ? ld_coh(x + c[k]) : x[c[k]];
#pragma unroll
    for (int k = 0; k < kRowChunk; ++k)
      if (e0 + k < hi) op(v[k], xv[k]);
  }
}

// Integer SpMV for one row (Fig. 2; Sec. V-C.3, eq. (matvec)): z = A_0 v + sum_l
// asr(A_l v, alpha_l), the matrices in SELL-64 layout (slice = 64 rows stored
// column-major, so the 64 lanes of a wavefront read consecutive words). Every
// sum is exact; `ovf` is set if a product, a term or the total leaves int64.
// `a` is any record with the SELL fields of CycleArgs. CH entries are in
// flight per chunk; NT loads the values and column indices as streaming
// (non-temporal) data, which leaves the caches to the gathered v: faster once
// the matrix is far larger than the last-level cache and read once per pass.
template <int CH = kRowChunk, bool NT = false, class A>
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
    for (int e0 = 0; e0 < wdt; e0 += CH) {
      int64_t vv[CH], xv[CH];
      int32_t c[CH];
#pragma unroll
      for (int k = 0; k < CH; ++k)
        if (e0 + k < wdt) {
          const int64_t pos = base + (int64_t)(e0 + k) * 64;
          if (NT) {
            vv[k] = __builtin_nontemporal_load(val + pos);
            c[k] = __builtin_nontemporal_load(a.sell_col + pos);
          } else {
            vv[k] = val[pos];
            c[k] = a.sell_col[pos];
          }
        }
#pragma unroll
      for (int k = 0; k < CH; ++k)
        if (e0 + k < wdt) xv[k] = v[c[k]];
#pragma unroll
      for (int k = 0; k < CH; ++k)
        if (e0 + k < wdt) acc.add(mulw(vv[k], xv[k], ovf));
    }
    int64_t t = acc.value(ovf);
    if (l > 0) t = asr(t, a.alpha[l]);
    tot.add(t);
  }
  return tot.value(ovf);
}

// The same SpMV row by g lanes (g = 4, 8, 16, 32 or 64, the same in every lane:
// aligned groups of consecutive lanes of one wavefront) over the CSR layout of
// the integer matrices (crp, ccol, cval): lane l of the group takes entries l,
// l + g, ...; the exact partial sums are combined over the group, so every
// lane of the group returns the row's z and sets the overflow flag exactly
// when spmv_row would. Rows with act == false give 0. Every lane of the
// wavefront must call it (the combination reads all lanes).
constexpr int kLaneChunk = 2;

__device__ __forceinline__ int64_t group_sum64_rt(int64_t v, int g) {
  for (int off = 1; off < g; off <<= 1) v += __shfl_xor(v, off, 64);
  return v;
}

template <class A>
__device__ __forceinline__ int64_t spmv_row_lanes(const A &a, int64_t row, bool act, const int64_t *__restrict__ v,
                                                  int nterms, int g, bool &ovf) {
  const int gl = (int)(threadIdx.x & (g - 1));
  const int64_t lo = act ? a.crp[row] : 0, hi = act ? a.crp[row + 1] : 0;
  Acc tot;
  tot.zero();
  for (int l = 0; l < nterms; ++l) {
    const int64_t *__restrict__ val = a.cval[l];
    Acc acc;
    acc.zero();
    for (int64_t e0 = lo + gl; e0 < hi; e0 += (int64_t)g * kLaneChunk) {
      int32_t c[kLaneChunk];
      int64_t vv[kLaneChunk], xv[kLaneChunk];
#pragma unroll
      for (int k = 0; k < kLaneChunk; ++k)
        if (e0 + k * g < hi) {
          c[k] = a.ccol[e0 + k * g];
          vv[k] = val[e0 + k * g];
        }
#pragma unroll
      for (int k = 0; k < kLaneChunk; ++k)
        if (e0 + k * g < hi) xv[k] = v[c[k]];
#pragma unroll
      for (int k = 0; k < kLaneChunk; ++k)
        if (e0 + k * g < hi) acc.add(mulw(vv[k], xv[k], ovf));
    }
    acc.lo = group_sum64_rt(acc.lo, g);
    acc.hi = group_sum64_rt(acc.hi, g);
    int64_t t = acc.value(ovf);
    if (l > 0) t = asr(t, a.alpha[l]);
    tot.add(t);
  }
  return tot.value(ovf);
}

// The SpMV of BLOCK consecutive rows row0 .. row0 + BLOCK - 1 (rows >= a.n
// give 0) by one workgroup with g lanes per row; row row0 + i's z is left in
// zl[i] (LDS). Called by every thread of the workgroup.
template <int BLOCK, class A>
__device__ __forceinline__ void spmv_chunk_lanes(const A &a, int64_t row0, const int64_t *__restrict__ v, int nterms,
                                                 int g, int64_t *zl, bool &ovf) {
  const int sh = __builtin_ctz((unsigned)g);
  const int rs = (int)(threadIdx.x >> sh), gl = (int)(threadIdx.x & (g - 1));
  for (int p = 0; p < g; ++p) {
    const int i = (p << (__builtin_ctz((unsigned)BLOCK) - sh)) + rs;
    const int64_t z = spmv_row_lanes(a, row0 + i, row0 + i < a.n, v, nterms, g, ovf);
    if (gl == 0) zl[i] = z;
  }
}

// The SpMV of BLOCK consecutive rows row0 .. row0 + BLOCK - 1 (rows >= a.n
// give 0) by one workgroup, its entries split evenly over the threads whatever
// the row lengths: the merge-based partition of Merrill and Garland (SC16). The
// chunk's BLOCK row ends and E entries form one merged sequence of BLOCK + E
// items; thread t takes items [t p, (t + 1) p), p = ceil((BLOCK + E) / BLOCK),
// so it walks a contiguous run of entries and crosses at most p row ends. The
// exact partial sums of one row from different threads meet in LDS through
// 64-bit atomic adds of the two limbs: integer addition is exact, so the row's
// term sum, the overflow flag and z equal spmv_row's whatever the split.
// Returns row row0 + threadIdx.x's z. LDS: merge_lds_bytes(BLOCK) at lds.
// Called by every thread of the workgroup; chunk entries below 2^31.
constexpr int kMergeBatch = 4;

template <int BLOCK, class A>
__device__ __forceinline__ int64_t spmv_chunk_merge(const A &a, int64_t row0, const int64_t *__restrict__ v,
                                                    int nterms, char *lds, bool &ovf) {
  int32_t *rp = (int32_t *)lds;  // rp[i]: first entry of row i relative to the chunk; rp[BLOCK] = E
  unsigned long long *slo = (unsigned long long *)(lds + merge_rp_bytes(BLOCK));
  unsigned long long *shi = slo + BLOCK;
  const int t = (int)threadIdx.x;
  const int64_t left = a.n - row0;
  const int nrows = left <= 0 ? 0 : left >= BLOCK ? BLOCK : (int)left;
  const int64_t base = nrows > 0 ? a.crp[row0] : 0;
  const int E = nrows > 0 ? (int)(a.crp[row0 + nrows] - base) : 0;
  if (t == 0) rp[0] = 0;
  rp[t + 1] = t < nrows ? (int32_t)(a.crp[row0 + t + 1] - base) : E;  // padded rows: empty
  __syncthreads();
  // thread t's first item: i row ends and j entries before it (merge-path
  // search: row end i precedes entry j exactly when rp[i + 1] <= j)
  const int total = BLOCK + E;
  const int per = (total + BLOCK - 1) / BLOCK;
  const int d0 = min(t * per, total), d1 = min(d0 + per, total);
  int lo = max(0, d0 - E), hi = min(d0, BLOCK);
  while (lo < hi) {
    const int mid = (lo + hi) >> 1;
    if (rp[mid + 1] <= d0 - mid - 1) lo = mid + 1;
    else hi = mid;
  }
  const int i0 = lo, j0 = d0 - lo;
  const int32_t *__restrict__ col = a.ccol + base;
  Acc tot;
  tot.zero();
  for (int l = 0; l < nterms; ++l) {
    const int64_t *__restrict__ val = a.cval[l] + base;
    slo[t] = 0;
    shi[t] = 0;
    __syncthreads();
    int i = i0, j = j0;
    Acc acc;
    acc.zero();
    for (int d = d0; d < d1;) {
      // the next batch of this thread's entries (loads issued together), then
      // the merged walk over them and the row ends between them
      int32_t c[kMergeBatch];
      int64_t vv[kMergeBatch], xv[kMergeBatch];
#pragma unroll
      for (int u = 0; u < kMergeBatch; ++u)
        if (j + u < E) {
          c[u] = col[j + u];
          vv[u] = val[j + u];
        }
#pragma unroll
      for (int u = 0; u < kMergeBatch; ++u)
        if (j + u < E) xv[u] = v[c[u]];
      // products of the entries this batch may consume (an entry whose product
      // is formed but which another thread consumes is in the same chunk, so
      // the overflow flag of the SpMV is unchanged)
      int64_t pr[kMergeBatch];
#pragma unroll
      for (int u = 0; u < kMergeBatch; ++u) pr[u] = (j + u < E && d + u < d1) ? mulw(vv[u], xv[u], ovf) : 0;
      int u = 0;
      while (d < d1 && u < kMergeBatch) {
        if (i < BLOCK && rp[i + 1] <= j) {  // row i ends here
          atomicAdd(slo + i, (unsigned long long)acc.lo);
          atomicAdd(shi + i, (unsigned long long)acc.hi);
          acc.zero();
          ++i;
        } else {
          int64_t pu = pr[0];
#pragma unroll
          for (int q = 1; q < kMergeBatch; ++q)
            if (q == u) pu = pr[q];
          acc.add(pu);
          ++j;
          ++u;
        }
        ++d;
      }
    }
    if (i < BLOCK) {  // the row this thread's items end inside
      atomicAdd(slo + i, (unsigned long long)acc.lo);
      atomicAdd(shi + i, (unsigned long long)acc.hi);
    }
    __syncthreads();
    Acc rs;
    rs.lo = (int64_t)slo[t];
    rs.hi = (int64_t)shi[t];
    int64_t tl = rs.value(ovf);
    if (l > 0) tl = asr(tl, a.alpha[l]);
    tot.add(tl);
    __syncthreads();
  }
  return tot.value(ovf);
}

// Preconditioner apply (Sec. VI), forward substitution for one row: y_i = tdiv(z_i - sum_{j<i}
// Lbar_ij y_j, Lbar_ii) (COH: y read with device-coherent loads).
template <bool COH = false, class A>
__device__ __forceinline__ int64_t lower_row(const A &a, int64_t row, int64_t zi, const int64_t *y, bool &ovf) {
  Acc acc;
  acc.zero();
  acc.add(zi);
  row_visit<COH>(a.lptr[row], a.lptr[row + 1], a.lcol, a.lval, y,
                 [&](int64_t l, int64_t yj) { acc.sub(mulw(yj, l, ovf)); });
  return tdiv(acc.value(ovf), a.ldiag[row], ovf);
}

// Preconditioner apply (Sec. VI), backward substitution for one row: u_i = tdiv(y_i - sum_{j>i}
// Ubar_ij u_j, Ubar_ii).
template <bool COH = false, class A>
__device__ __forceinline__ int64_t upper_row(const A &a, int64_t row, int64_t yi, const int64_t *u, bool &ovf) {
  Acc acc;
  acc.zero();
  acc.add(yi);
  row_visit<COH>(a.uptr[row], a.uptr[row + 1], a.ucol, a.uval, u,
                 [&](int64_t uv, int64_t uj) { acc.sub(mulw(uj, uv, ovf)); });
  return tdiv(acc.value(ovf), a.udiag[row], ovf);
}

// FP64 row of the triangular substitution of the start step (Sec. VI): (b - sum_e f_e x_col) /
// d, the sum in CSR order.
template <bool COH = false>
__device__ __forceinline__ double fp_sub_row(int64_t lo, int64_t hi, const int32_t *__restrict__ col,
                                             const double *__restrict__ f, const double *x, double b, double d) {
  double acc = 0.0;
  row_visit<COH>(lo, hi, col, f, x, [&](double fv, double xv) { acc = acc + fv * xv; });
  return (b - acc) / d;
}

// FP64 residual row of eq. (b): r = b - A x and rhat = bhat - Ahat x with the
// same gathered x, each sum in CSR order.
__device__ __forceinline__ void residual_row(int64_t lo, int64_t hi, const int32_t *__restrict__ col,
                                             const double *__restrict__ a, const double *__restrict__ ahat,
                                             const double *__restrict__ x, double b, double bhat, double &r,
                                             double &rhat) {
  double acc = 0.0, acch = 0.0;
  for (int64_t e0 = lo; e0 < hi; e0 += kRowChunk) {
    int32_t c[kRowChunk];
    double av[kRowChunk], hv[kRowChunk], xv[kRowChunk];
#pragma unroll
    for (int k = 0; k < kRowChunk; ++k)
      if (e0 + k < hi) {
        c[k] = col[e0 + k];
        av[k] = a[e0 + k];
        hv[k] = ahat[e0 + k];
      }
#pragma unroll
    for (int k = 0; k < kRowChunk; ++k)
      if (e0 + k < hi) xv[k] = x[c[k]];
#pragma unroll
    for (int k = 0; k < kRowChunk; ++k)
      if (e0 + k < hi) {
        acc = acc + av[k] * xv[k];
        acch = acch + hv[k] * xv[k];
      }
  }
  r = b - acc;
  rhat = bhat - acch;
}

// Normalisation v = w / h (Fig. 2) for one element: sc(tdiv(shl(w, b1), den), df - b1 - b2).
__device__ __forceinline__ int64_t normalize_elem(int64_t w, int64_t den, int b1, int sc_exp, bool &ovf) {
  return scale2(tdiv(shl(w, b1, ovf), den, ovf), sc_exp, ovf);
}

}  // namespace igm
