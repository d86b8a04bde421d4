// FP64 refinement kernels (Sec. IV, Fig. 1; the start step and cast of Fig. 2
// and Sec. VI) and the
// standalone integer kernels behind the kernel-level entry points.
//
// FP64 rules: no contraction (built with -ffp-contract=off), each row sums its
// products in CSR order, every other step is elementwise, and norms use the
// order-free construction of dnrm_finish, so results do not depend on the
// launch shape.
#include <algorithm>
#include <mutex>

#include "igm_bsweep.hpp"
#include "igm_launch.hpp"
#include "igm_rows.hpp"
#include "igm_sweep.hpp"
#include "igm_sync.hpp"

namespace igm {

constexpr int kB = 256;  // threads per workgroup of the elementwise kernels

__device__ __forceinline__ unsigned long long wave_max_u64(unsigned long long v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    unsigned long long t = (unsigned long long)__shfl_xor((long long)v, o, 64);
    v = t > v ? t : v;
  }
  return v;
}

// The copy of reduction word w that this workgroup adds into.
__device__ __forceinline__ unsigned long long *red_copy(unsigned long long *w) {
  return w + (blockIdx.x % kRedCopies) * kRedWords;
}

// Maximum over the copies of reduction word w.
__device__ __forceinline__ unsigned long long red_max(const unsigned long long *w) {
  unsigned long long m = 0;
#pragma unroll
  for (int c = 0; c < kRedCopies; ++c) m = w[c * kRedWords] > m ? w[c * kRedWords] : m;
  return m;
}

// Max of non-negative doubles through their bit patterns (monotone for
// non-negative values; NaN patterns sort above infinity).
__device__ __forceinline__ void block_max_to(unsigned long long v, unsigned long long *dst) {
  __shared__ unsigned long long sh[kB / 64];
  v = wave_max_u64(v);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long m = 0;
    for (int k = 0; k < kB / 64; ++k) m = sh[k] > m ? sh[k] : m;
    if (m) atomicMax(red_copy(dst), m);
  }
}

// eq. (b): r = b - A x (scaled) and rhat = bhat - Ahat x (original).
// eq. (b) with G lanes per row (G = 4, 8, 16, 32, 64): the lanes of a group form the
// products of G consecutive entries at once, then every lane of the group adds
// them one after another in entry order, so r and rhat round exactly as the
// sums in CSR order of residual_row.
template <int G>
__global__ __launch_bounds__(kB) void k_residual_lanes(int64_t n, const int64_t *__restrict__ rp,
                                                       const int32_t *__restrict__ col, const double *__restrict__ a,
                                                       const double *__restrict__ ahat, const double *__restrict__ b,
                                                       const double *__restrict__ bhat, const double *__restrict__ x,
                                                       const double *__restrict__ cscale, double *r, double *rhat,
                                                       unsigned long long *red) {
  const int gl = (int)(threadIdx.x % G);
  const int lead = (int)(threadIdx.x & 63) - gl;  // the group's first lane in the wavefront
  const int64_t i = (int64_t)blockIdx.x * (kB / G) + threadIdx.x / G;
  unsigned long long m0 = 0, m1 = 0;
  if (i < n) {
    const int64_t lo = rp[i], hi = rp[i + 1];
    double acc = 0.0, acch = 0.0;
    for (int64_t e0 = lo; e0 < hi; e0 += G) {  // the same trip count in every lane of the group
      double p = 0.0, ph = 0.0;
      if (e0 + gl < hi) {
        const double xv = x[col[e0 + gl]];
        p = a[e0 + gl] * xv;
        ph = ahat[e0 + gl] * xv;
      }
#pragma unroll
      for (int j = 0; j < G; ++j) {
        const double pj = __shfl(p, lead + j, 64), phj = __shfl(ph, lead + j, 64);
        if (e0 + j < hi) {
          acc = acc + pj;
          acch = acch + phj;
        }
      }
    }
    double ri = b[i] - acc, rhi = bhat[i] - acch;
    if (cscale) ri = rhi / cscale[i];  // eq. (eq2), as in k_residual
    if (gl == 0) {
      r[i] = ri;
      rhat[i] = rhi;
      m0 = dbits(fabs(ri));
      m1 = dbits(fabs(rhi));
    }
  }
  block_max_to(m0, red + kRedMuR);
  __syncthreads();
  block_max_to(m1, red + kRedMuRhat);
}

__global__ __launch_bounds__(kB) void k_residual(int64_t n, const int64_t *__restrict__ rp,
                                                 const int32_t *__restrict__ col, const double *__restrict__ a,
                                                 const double *__restrict__ ahat, const double *__restrict__ b,
                                                 const double *__restrict__ bhat, const double *__restrict__ x,
                                                 const double *__restrict__ cscale, double *r, double *rhat,
                                                 unsigned long long *red) {
  const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  unsigned long long m0 = 0, m1 = 0;
  if (i < n) {
    double ri, rhi;
    residual_row(rp[i], rp[i + 1], col, a, ahat, x, b[i], bhat[i], ri, rhi);
    // eq. (eq2): x holds xhat and the scaled residual is D1^-1 (bhat - Ahat xhat)
    if (cscale) ri = rhi / cscale[i];
    r[i] = ri;
    rhat[i] = rhi;
    m0 = dbits(fabs(ri));
    m1 = dbits(fabs(rhi));
  }
  block_max_to(m0, red + kRedMuR);
  __syncthreads();
  block_max_to(m1, red + kRedMuRhat);
}

__global__ __launch_bounds__(kB) void k_absmax(int64_t n, const double *__restrict__ x, unsigned long long *dst) {
  unsigned long long m = 0;
  for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kB) {
    unsigned long long t = dbits(fabs(x[i]));
    m = t > m ? t : m;
  }
  block_max_to(m, dst);
}

// Exact sum of floor(2^96 (x_i / mu)^2) as three 40-bit limbs.
__global__ __launch_bounds__(kB) void k_dnrm_sum(int64_t n, const double *__restrict__ x,
                                                 const unsigned long long *mu_bits, unsigned long long *limbs) {
  const double mu = __longlong_as_double((long long)red_max(mu_bits));
  unsigned long long l0 = 0, l1 = 0, l2 = 0;
  if (mu > 0.0 && mu <= 1.7976931348623157e308) {
    for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kB) {
      const double t = x[i] / mu;
      const unsigned __int128 q = fix96(t * t);
      l0 += (unsigned long long)q & kLimbMask;
      l1 += (unsigned long long)(q >> 40) & kLimbMask;
      l2 += (unsigned long long)(q >> 80);
    }
  }
  __shared__ unsigned long long sh[3][kB / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    l0 += (unsigned long long)__shfl_xor((long long)l0, o, 64);
    l1 += (unsigned long long)__shfl_xor((long long)l1, o, 64);
    l2 += (unsigned long long)__shfl_xor((long long)l2, o, 64);
  }
  if ((threadIdx.x & 63) == 0) {
    sh[0][threadIdx.x >> 6] = l0;
    sh[1][threadIdx.x >> 6] = l1;
    sh[2][threadIdx.x >> 6] = l2;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    unsigned long long s0 = 0, s1 = 0, s2 = 0;
    for (int k = 0; k < kB / 64; ++k) { s0 += sh[0][k]; s1 += sh[1][k]; s2 += sh[2][k]; }
    s1 += s0 >> 40;
    s0 &= kLimbMask;
    s2 += s1 >> 40;
    s1 &= kLimbMask;
    unsigned long long *dst = red_copy(limbs);
    if (s0) atomicAdd(dst + 0, s0);
    if (s1) atomicAdd(dst + 1, s1);
    if (s2) atomicAdd(dst + 2, s2);
  }
}

// ||x|| = mu * sqrt(rn(S)) * 2^-48 with S the exact limb sum (all copies;
// S <= n 2^96 < 2^128, and every partial sum is at most S).
__device__ double dnrm_finish(const unsigned long long *limbs, const unsigned long long *mu_word) {
  const double mu = __longlong_as_double((long long)red_max(mu_word));
  if (!(mu > 0.0) || !(mu <= 1.7976931348623157e308)) return mu;
  unsigned __int128 S = 0;
  for (int c = 0; c < kRedCopies; ++c) {
    const unsigned long long *l = limbs + c * kRedWords;
    S += ((unsigned __int128)l[2] << 80) + ((unsigned __int128)l[1] << 40) + (unsigned __int128)l[0];
  }
  return mu * ldexp(sqrt(u128_to_double_rn(S)), -48);
}

__device__ __forceinline__ double relres(double rn, double bn) {
  if (bn > 0.0) return rn / bn;
  return rn == 0.0 ? 0.0 : __builtin_inf();
}

__global__ void k_fin_residual(const unsigned long long *red, const double *norms, double *scal) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double rn = dnrm_finish(red + kRedSumR, red + kRedMuR);
  const double rhn = dnrm_finish(red + kRedSumRhat, red + kRedMuRhat);
  scal[kScalGamma] = __longlong_as_double((long long)red_max(red + kRedMuR));
  scal[kScalRelresOrig] = relres(rhn, norms[1]);
  scal[kScalRelresScaled] = relres(rn, norms[0]);
}

__global__ void k_fin_norm(const unsigned long long *red, double *out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *out = dnrm_finish(red + kRedSumX, red + kRedMuX);
}

__global__ void k_fin_max(const unsigned long long *w, double *out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *out = __longlong_as_double((long long)red_max(w));
}

// FP64 start step (Sec. VI) for the diagonal or identity preconditioner, fused
// with eq. (scale):
// bk = r / gamma, r0 = (bk / Lbar_ii) / Ubar_ii.
__global__ __launch_bounds__(kB) void k_scale_diag(int64_t n, const double *__restrict__ r, const double *scal,
                                                   const int64_t *__restrict__ ld, const int64_t *__restrict__ ud,
                                                   int pre, double *bk, double *r0, unsigned long long *red) {
  const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  unsigned long long mb = 0;
  if (i < n) {
    const double g = scal[kScalGamma];
    const double t = r[i] / g;
    bk[i] = t;
    double u = t;
    if (pre != IGM_PRE_NONE) u = (t / (double)ld[i]) / (double)ud[i];
    r0[i] = u;
    mb = dbits(fabs(u));
  }
  block_max_to(mb, red + kRedMuR0);
}

__global__ __launch_bounds__(kB) void k_scale(int64_t n, const double *__restrict__ r, const double *scal, double *bk) {
  const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (i < n) bk[i] = r[i] / scal[kScalGamma];
}

// FP64 start step (Sec. VI) with ILU(0): the FP64 substitution with the integer factors
// converted to double, forward y_i = (bk_i - sum L_ij y_j) / Lbar_ii, then
// backward u_i = (y_i - sum U_ij u_j) / Ubar_ii in place; each row sums in CSR
// order. One launch per direction, run block by block on the schedules of
// the integer sweeps with their helper wavefront (igm_bsweep.hpp); a block
// waits for the blocks it reads, so the launch must be co-resident
// (cooperative).
constexpr int kSweepBlock = 256;  // the helper and up to three computing wavefronts

__global__ __launch_bounds__(kSweepBlock) void k_fp_bsweep(BlockSweepArgs b, const double *src, double *dst,
                                                           CycleState *state) {
  extern __shared__ double fsm[];
  bool ovf = false, to = false;
  block_sweep_int<kSweepBlock, 1, true>(b, src, dst, (char *)fsm, ovf, to);
  if (to) __hip_atomic_store(&state->timeout, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__global__ void k_fin_rho(const unsigned long long *red, double *scal, CycleState *st) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  const double rho = dnrm_finish(red + kRedSumR0, red + kRedMuR0);
  scal[kScalRho] = rho;
  if (!(rho > 0.0) || !(rho <= 1.7976931348623157e308)) st->range_err = 1;
}

// Cast of v1 to Q.df (Fig. 2; Sec. V-D.1): v1 = trunc(2^df r0 / rho), with a range check.
__global__ __launch_bounds__(kB) void k_cast_v1(int64_t n, const double *__restrict__ r0, const double *scal, int df,
                                                int64_t *v1, CycleState *st) {
  const int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x;
  if (i >= n) return;
  const double rho = scal[kScalRho];
  const double t = ldexp(r0[i] / rho, df);
  if (t >= -9223372036854775808.0 && t < 9223372036854775808.0) {
    v1[i] = (int64_t)t;
  } else {
    v1[i] = 0;
    st->range_err = 1;
  }
}

// ---- standalone integer kernels ------------------------------------------

// The standalone SpMV over SELL-64: one thread per row (a workgroup per 256
// rows), 16 entries in flight per row, the matrix streamed non-temporally.
__global__ __launch_bounds__(kB) void k_spmv(CycleArgs a, int nterms, const int64_t *__restrict__ v, int64_t *z) {
  bool o = false;
  for (int64_t row = (int64_t)blockIdx.x * kB + threadIdx.x; row < a.n; row += (int64_t)gridDim.x * kB)
    z[row] = spmv_row<16, true>(a, row, v, nterms, o);
  note_event(o, &a.state->first_ovf, ev_code(1, 1, 0));
}

// The standalone SpMV with G lanes per row (igm_rows.hpp): kB / G rows per
// workgroup pass; every lane runs the same number of passes.
template <int G>
__global__ __launch_bounds__(kB) void k_spmv_lanes(CycleArgs a, int nterms, const int64_t *__restrict__ v,
                                                   int64_t *z) {
  bool o = false;
  constexpr int RPW = kB / G;
  const int gl = (int)(threadIdx.x % G);
  for (int64_t r0 = (int64_t)blockIdx.x * RPW; r0 < a.n; r0 += (int64_t)gridDim.x * RPW) {
    const int64_t row = r0 + threadIdx.x / G;
    const int64_t zr = spmv_row_lanes(a, row, row < a.n, v, nterms, G, o);
    if (row < a.n && gl == 0) z[row] = zr;
  }
  note_event(o, &a.state->first_ovf, ev_code(1, 1, 0));
}

// The standalone SpMV with each chunk of kB rows split evenly by entries over
// the workgroup (spmv_chunk_merge); the loop over chunks is uniform.
__global__ __launch_bounds__(kB) void k_spmv_merge(CycleArgs a, int nterms, const int64_t *__restrict__ v,
                                                   int64_t *z) {
  __shared__ __align__(16) char lds[merge_lds_bytes(kB)];
  bool o = false;
  for (int64_t r0 = (int64_t)blockIdx.x * kB; r0 < a.n; r0 += (int64_t)gridDim.x * kB) {
    const int64_t zr = spmv_chunk_merge<kB>(a, r0, v, nterms, lds, o);
    if (r0 + threadIdx.x < a.n) z[r0 + threadIdx.x] = zr;
  }
  note_event(o, &a.state->first_ovf, ev_code(1, 1, 0));
}

__global__ __launch_bounds__(kB) void k_diag_solve(CycleArgs a, const int64_t *__restrict__ z, int64_t *w) {
  bool o = false;
  for (int64_t row = (int64_t)blockIdx.x * kB + threadIdx.x; row < a.n; row += (int64_t)gridDim.x * kB)
    w[row] = a.precond == IGM_PRE_NONE ? z[row] : tdiv_diag(tdiv_diag(z[row], a.ldiag[row], o), a.udiag[row], o);
  note_event(o, &a.state->first_ovf, ev_code(1, 2, 0));
}

__global__ __launch_bounds__(kB) void k_lower_level(CycleArgs a, int32_t lo, int32_t hi, const int64_t *__restrict__ z,
                                                    int64_t *y) {
  const int64_t q = lo + (int64_t)blockIdx.x * kB + threadIdx.x;
  if (q >= hi) return;
  bool o = false;
  const int64_t row = a.flev_rows[q];
  y[row] = lower_row(a, row, z[row], y, o);
  note_event(o, &a.state->first_ovf, ev_code(1, 2, 0));
}

__global__ __launch_bounds__(kB) void k_upper_level(CycleArgs a, int32_t lo, int32_t hi, int64_t *u) {
  const int64_t q = lo + (int64_t)blockIdx.x * kB + threadIdx.x;
  if (q >= hi) return;
  bool o = false;
  const int64_t row = a.blev_rows[q];
  u[row] = upper_row(a, row, u[row], u, o);
  note_event(o, &a.state->first_ovf, ev_code(1, 2, 0));
}

// Gram-Schmidt inner product (mode 0: h = asr(sum asr(w, b) v, df - b)) or the
// norm of w (mode 1:
// h = shl(isqrt(sum asr(w, b)^2), b)) in one launch: each workgroup adds its
// rows into an exact Acc and stores it with device-coherent stores; the last
// workgroup to take a ticket adds all of them and finishes. The ticket word
// is zero when the buffer is allocated and the last workgroup of every launch
// sets it back to zero.
constexpr int kRB = 512;     // threads per workgroup of the standalone reductions
constexpr int kRUnroll = 8;  // elements in flight per thread

__global__ __launch_bounds__(kRB) void k_reduce(int64_t n, const int64_t *__restrict__ w,
                                               const int64_t *__restrict__ v, int b, int df, int mode, Acc *parts,
                                               unsigned *ticket, int64_t *out, int64_t *first, int64_t code) {
  __shared__ Acc sh_wave[kRB / 64];
  __shared__ int last;
  Acc acc;
  acc.zero();
  bool o = false;
  const int64_t stride = (int64_t)gridDim.x * kRB;
  for (int64_t i0 = (int64_t)blockIdx.x * kRB + threadIdx.x; i0 < n; i0 += stride * kRUnroll) {
    int64_t wv[kRUnroll], vv[kRUnroll];
#pragma unroll
    for (int u = 0; u < kRUnroll; ++u) {
      const int64_t i = i0 + u * stride;
      wv[u] = i < n ? w[i] : 0;
      vv[u] = (mode == 0 && i < n) ? v[i] : 0;
    }
#pragma unroll
    for (int u = 0; u < kRUnroll; ++u) {
      const int64_t t = asr(wv[u], b);
      acc.add(mode == 0 ? mulw(t, vv[u], o) : sqrc(t, o));
    }
  }
  note_event(o, first, code);
  const Acc p = block_sum<kRB>(acc, sh_wave);
  if (threadIdx.x == 0) {
    st_coh(&parts[blockIdx.x].lo, p.lo);
    st_coh(&parts[blockIdx.x].hi, p.hi);
    wait_vm();
    last = __hip_atomic_fetch_add(ticket, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gridDim.x - 1;
  }
  __syncthreads();
  if (!last) return;
  Acc tot;
  tot.zero();
  for (int k = threadIdx.x; k < (int)gridDim.x; k += kRB) {
    Acc q;
    q.lo = ld_coh(&parts[k].lo);
    q.hi = ld_coh(&parts[k].hi);
    q.normalize();
    tot.add(q);
  }
  const Acc t = block_sum<kRB>(tot, sh_wave);
  if (threadIdx.x == 0) {
    bool of = false;
    const int64_t S = t.value(of);
    const int64_t r = mode == 0 ? asr(S, df - b) : shl(isqrt64(S), b, of);
    if (of) atomicMin((long long *)first, (long long)code);
    *out = r;
    *ticket = 0u;
  }
}

__global__ __launch_bounds__(kB) void k_axpy(int64_t n, int64_t h, int b, int df, int64_t *w,
                                             const int64_t *__restrict__ v, CycleState *st) {
  bool o = false;
  const int64_t hs = asr(h, b);
  for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kB)
    w[i] = subc(w[i], asr(mulc(hs, v[i], o), df - b), o);
  note_event(o, &st->first_ovf, ev_code(1, 3, 1));
}

__global__ __launch_bounds__(kB) void k_normalize(int64_t n, const int64_t *__restrict__ w, int64_t den, int b1,
                                                  int e, int64_t *v, CycleState *st) {
  bool o = false;
  for (int64_t i = (int64_t)blockIdx.x * kB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kB)
    v[i] = normalize_elem(w[i], den, b1, e, o);
  note_event(o, &st->first_ovf, ev_code(1, 5, 0));
}

// ---- host launchers --------------------------------------------------------

static inline unsigned blocks_for(int64_t n) { return (unsigned)((n + kB - 1) / kB); }
// Grid-stride kernels: at most four workgroups per compute unit, so each
// reduction copy takes at most 64 workgroup atomics.
static inline unsigned grid_stride_blocks(int64_t n) {
  int64_t b = (n + kB - 1) / kB;
  return (unsigned)(b < 1024 ? (b > 0 ? b : 1) : 1024);
}

hipError_t launch_residual(hipStream_t st, int64_t n, const int64_t *rp, const int32_t *col, const double *a,
                           const double *ahat, const double *b, const double *bhat, const double *x,
                           const double *cscale, double *r, double *rhat, unsigned long long *red, int lanes) {
  if (n <= 0) return hipSuccess;
  if (lanes == IGM_SPMV_MERGE) lanes = 16;  // FP64 sums keep their order: lanes per row
  const unsigned rows_blocks = (unsigned)((n + kB / std::max(lanes, 1) - 1) / (kB / std::max(lanes, 1)));
  if (lanes == 4)
    hipLaunchKernelGGL(k_residual_lanes<4>, dim3(rows_blocks), dim3(kB), 0, st, n, rp, col, a, ahat, b, bhat, x,
                       cscale, r, rhat, red);
  else if (lanes == 8)
    hipLaunchKernelGGL(k_residual_lanes<8>, dim3(rows_blocks), dim3(kB), 0, st, n, rp, col, a, ahat, b, bhat, x,
                       cscale, r, rhat, red);
  else if (lanes == 32)
    hipLaunchKernelGGL(k_residual_lanes<32>, dim3(rows_blocks), dim3(kB), 0, st, n, rp, col, a, ahat, b, bhat, x,
                       cscale, r, rhat, red);
  else if (lanes == 16)
    hipLaunchKernelGGL(k_residual_lanes<16>, dim3(rows_blocks), dim3(kB), 0, st, n, rp, col, a, ahat, b, bhat, x,
                       cscale, r, rhat, red);
  else if (lanes == 64)
    hipLaunchKernelGGL(k_residual_lanes<64>, dim3(rows_blocks), dim3(kB), 0, st, n, rp, col, a, ahat, b, bhat, x,
                       cscale, r, rhat, red);
  else
    hipLaunchKernelGGL(k_residual, dim3(blocks_for(n)), dim3(kB), 0, st, n, rp, col, a, ahat, b, bhat, x, cscale,
                       r, rhat, red);
  return hipGetLastError();
}

hipError_t launch_absmax(hipStream_t st, int64_t n, const double *x, unsigned long long *dst) {
  hipLaunchKernelGGL(k_absmax, dim3(grid_stride_blocks(n)), dim3(kB), 0, st, n, x, dst);
  return hipGetLastError();
}

hipError_t launch_dnrm_sum(hipStream_t st, int64_t n, const double *x, const unsigned long long *mu,
                           unsigned long long *limbs) {
  hipLaunchKernelGGL(k_dnrm_sum, dim3(grid_stride_blocks(n)), dim3(kB), 0, st, n, x, mu, limbs);
  return hipGetLastError();
}

hipError_t launch_fin_residual(hipStream_t st, const unsigned long long *red, const double *norms, double *scal) {
  hipLaunchKernelGGL(k_fin_residual, dim3(1), dim3(64), 0, st, red, norms, scal);
  return hipGetLastError();
}

hipError_t launch_fin_norm(hipStream_t st, const unsigned long long *red, double *out) {
  hipLaunchKernelGGL(k_fin_norm, dim3(1), dim3(64), 0, st, red, out);
  return hipGetLastError();
}

hipError_t launch_fin_max(hipStream_t st, const unsigned long long *w, double *out) {
  hipLaunchKernelGGL(k_fin_max, dim3(1), dim3(64), 0, st, w, out);
  return hipGetLastError();
}

hipError_t launch_start_vector(hipStream_t st, const CycleArgs &a, const double *r, double *scal, const double *lvalf,
                               const double *uvalf, double *bk, double *r0, unsigned long long *red) {
  const int64_t n = a.n;
  if (a.precond != IGM_PRE_ILU0) {
    hipLaunchKernelGGL(k_scale_diag, dim3(blocks_for(n)), dim3(kB), 0, st, n, r, (const double *)scal, a.ldiag,
                       a.udiag, a.precond, bk, r0, red);
  } else {
    hipLaunchKernelGGL(k_scale, dim3(blocks_for(n)), dim3(kB), 0, st, n, r, (const double *)scal, bk);
    // the progress words of the blocked sweeps serve here too (k_cycle
    // clears them again in every Arnoldi step)
    hipError_t e = hipMemsetAsync(a.bsf.prog, 0, sizeof(unsigned) * ((size_t)a.bsf.nb + a.bsb.nb) * kLevStride, st);
    if (e != hipSuccess) return e;
    const size_t lds = sweep_lds_bytes(a.bsf.S, a.bsf.max_levels);
    int per_cu = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, (const void *)k_fp_bsweep, kSweepBlock, lds);
    if (e != hipSuccess) return e;
    int dev = 0, cus = 0;
    if ((e = hipGetDevice(&dev)) != hipSuccess) return e;
    if ((e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev)) != hipSuccess) return e;
    const int cap = std::max(per_cu, 1) * cus;
    CycleState *state = a.state;
    const double *cbk = bk, *cr0 = r0;
    BlockSweepArgs bf = a.bsf, bb = a.bsb;
    void *argf[] = {&bf, &cbk, &r0, &state};
    e = hipLaunchCooperativeKernel((const void *)k_fp_bsweep, dim3(std::min(bf.nb, cap)), dim3(kSweepBlock), argf,
                                   lds, st);
    if (e != hipSuccess) return e;
    void *argb[] = {&bb, &cr0, &r0, &state};
    e = hipLaunchCooperativeKernel((const void *)k_fp_bsweep, dim3(std::min(bb.nb, cap)), dim3(kSweepBlock), argb,
                                   lds, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_absmax, dim3(grid_stride_blocks(n)), dim3(kB), 0, st, n, (const double *)r0,
                       red + kRedMuR0);
  }
  hipLaunchKernelGGL(k_dnrm_sum, dim3(grid_stride_blocks(n)), dim3(kB), 0, st, n, (const double *)r0,
                     (const unsigned long long *)(red + kRedMuR0), red + kRedSumR0);
  hipLaunchKernelGGL(k_fin_rho, dim3(1), dim3(64), 0, st, (const unsigned long long *)red, scal, a.state);
  hipLaunchKernelGGL(k_cast_v1, dim3(blocks_for(n)), dim3(kB), 0, st, n, (const double *)r0, (const double *)scal,
                     a.df, a.V, a.state);
  return hipGetLastError();
}

hipError_t launch_spmv(hipStream_t st, const CycleArgs &a, int nterms, const int64_t *v, int64_t *z) {
  const unsigned g = grid_stride_blocks(a.n);
  if (a.spmv_lanes == IGM_SPMV_MERGE) hipLaunchKernelGGL(k_spmv_merge, dim3(g), dim3(kB), 0, st, a, nterms, v, z);
  else if (a.spmv_lanes == 4) hipLaunchKernelGGL(k_spmv_lanes<4>, dim3(g), dim3(kB), 0, st, a, nterms, v, z);
  else if (a.spmv_lanes == 8) hipLaunchKernelGGL(k_spmv_lanes<8>, dim3(g), dim3(kB), 0, st, a, nterms, v, z);
  else if (a.spmv_lanes == 16) hipLaunchKernelGGL(k_spmv_lanes<16>, dim3(g), dim3(kB), 0, st, a, nterms, v, z);
  else if (a.spmv_lanes == 32) hipLaunchKernelGGL(k_spmv_lanes<32>, dim3(g), dim3(kB), 0, st, a, nterms, v, z);
  else if (a.spmv_lanes == 64) hipLaunchKernelGGL(k_spmv_lanes<64>, dim3(g), dim3(kB), 0, st, a, nterms, v, z);
  else hipLaunchKernelGGL(k_spmv, dim3(blocks_for(a.n)), dim3(kB), 0, st, a, nterms, v, z);
  return hipGetLastError();
}

hipError_t launch_precond(hipStream_t st, const CycleArgs &a, const int64_t *z, int64_t *w) {
  if (a.precond != IGM_PRE_ILU0) {
    hipLaunchKernelGGL(k_diag_solve, dim3(grid_stride_blocks(a.n)), dim3(kB), 0, st, a, z, w);
    return hipGetLastError();
  }
  for (int L = 0; L < a.nflev; ++L) {
    int32_t lo = a.flev_host[L], hi = a.flev_host[L + 1];
    hipLaunchKernelGGL(k_lower_level, dim3(blocks_for(hi - lo)), dim3(kB), 0, st, a, lo, hi, z, w);
  }
  for (int L = 0; L < a.nblev; ++L) {
    int32_t lo = a.blev_host[L], hi = a.blev_host[L + 1];
    hipLaunchKernelGGL(k_upper_level, dim3(blocks_for(hi - lo)), dim3(kB), 0, st, a, lo, hi, w);
  }
  return hipGetLastError();
}

hipError_t launch_reduce(hipStream_t st, int64_t n, const int64_t *w, const int64_t *v, int b, int df, int mode,
                         AccWords *parts, int64_t *out, CycleState *state, int64_t code) {
  static_assert(sizeof(AccWords) == sizeof(Acc), "partial-sum layout");
  // enough workgroups for every compute unit, each thread kRUnroll elements
  // per pass; parts holds kMaxReduceParts partials and then the ticket word
  const int64_t want = (n + (int64_t)kRB * kRUnroll - 1) / ((int64_t)kRB * kRUnroll);
  const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>(want, kMaxReduceParts));
  unsigned *ticket = (unsigned *)(parts + kMaxReduceParts);  // zero between launches
  hipLaunchKernelGGL(k_reduce, dim3(nb), dim3(kRB), 0, st, n, w, v, b, df, mode, (Acc *)parts, ticket, out,
                     &state->first_ovf, code);
  return hipGetLastError();
}

hipError_t launch_axpy(hipStream_t st, int64_t n, int64_t h, int b, int df, int64_t *w, const int64_t *v,
                       CycleState *state) {
  hipLaunchKernelGGL(k_axpy, dim3(grid_stride_blocks(n)), dim3(kB), 0, st, n, h, b, df, w, v, state);
  return hipGetLastError();
}

hipError_t launch_normalize(hipStream_t st, int64_t n, const int64_t *w, int64_t den, int b1, int e, int64_t *v,
                            CycleState *state) {
  hipLaunchKernelGGL(k_normalize, dim3(grid_stride_blocks(n)), dim3(kB), 0, st, n, w, den, b1, e, v, state);
  return hipGetLastError();
}

// ---- The standalone inner product and norm without allocation -------------
//
// The same k_reduce as igm_dot / igm_norm, with its scratch (per-workgroup
// partial sums, then the completion ticket) in this fixed device array
// instead of a system's buffers, and at most kNoAllocParts workgroups (one per
// compute unit of the device is plenty for a streaming reduction). Each
// device holds its own copy; host code reaches it only through the address
// hipGetSymbolAddress returns on that device, looked up once per device.
constexpr int kNoAllocParts = 256;
constexpr size_t kNoAllocScratchBytes = sizeof(Acc) * kNoAllocParts + 256;  // partials, then the ticket
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {

constexpr int kNoAllocDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_dev[kNoAllocDevices] = {nullptr};

// clears the ticket and the caller's event word before a reduction
__global__ void k_noalloc_init(unsigned *ticket, int64_t *event) {
  *ticket = 0u;
  *event = kNoEvent;
}

}  // namespace

}  // namespace igm

extern "C" igm_status igm_reduce_noalloc(int32_t mode, int64_t n, const int64_t *w, const int64_t *v, int32_t b,
                                         int32_t df, int64_t *out_dev, void *stream) {
  using namespace igm;
  if ((mode != 0 && mode != 1) || n < 1 || n > kNoAllocMaxN || !w || (mode == 0 && !v) || !out_dev || df < 1 ||
      df > 62 || b < 0 || b > df)
    return IGM_ERR_ARG;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return IGM_ERR_DEVICE;
  if (dev < 0 || dev >= kNoAllocDevices) return IGM_ERR_UNSUPPORTED;
  void *base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_dev[dev]) {  // first call on this device: its copy's address
      void *p = nullptr;
      if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return IGM_ERR_DEVICE;
      g_scratch_dev[dev] = p;
    }
    base = g_scratch_dev[dev];
  }
  hipStream_t st = (hipStream_t)stream;
  Acc *parts = (Acc *)base;
  unsigned *ticket = (unsigned *)((char *)base + sizeof(Acc) * kNoAllocParts);
  const int64_t want = (n + (int64_t)kRB * kRUnroll - 1) / ((int64_t)kRB * kRUnroll);
  const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>(want, kNoAllocParts));
  hipLaunchKernelGGL(k_noalloc_init, dim3(1), dim3(1), 0, st, ticket, out_dev + 1);
  // event codes as in igm_dot / igm_norm: step 1, stage 3 (inner product) or 4 (norm)
  const int64_t code = ((int64_t)1 << 24) | ((int64_t)(mode == 0 ? 3 : 4) << 16);
  hipLaunchKernelGGL(k_reduce, dim3(nb), dim3(kRB), 0, st, n, w, mode == 0 ? v : w, b, df, mode, parts, ticket,
                     out_dev, out_dev + 1, code);
  return hipGetLastError() == hipSuccess ? IGM_OK : IGM_ERR_DEVICE;
}
