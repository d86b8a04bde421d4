// Host launchers of the igmres kernels and the layout of their scratch words.
#pragma once

#include "igm_device.hpp"
#include "igm_internal.hpp"

namespace igm {

// Workgroup partials of the standalone reductions (igm_dot, igm_norm); the
// partial buffer holds this many plus one word for the completion ticket.
constexpr int kMaxReduceParts = 2048;
// Largest length igm_reduce_noalloc accepts (its grid strides over any length;
// the bound only keeps index arithmetic far from overflow).
constexpr int64_t kNoAllocMaxN = (int64_t)1 << 48;

// Scratch words of the FP64 reductions (d_red): maxima as double bit patterns,
// exact norm sums as three 40-bit limbs. The block of kRedWords words is held
// kRedCopies times, 256 bytes apart: workgroup b adds into copy b % kRedCopies,
// so atomics to one word from many workgroups do not all queue on one cache
// line; readers combine the copies (max of maxima, sum of limbs, both
// order-free).
enum : int {
  kRedMuR = 0, kRedMuRhat = 1, kRedMuR0 = 2, kRedMuX = 3,
  kRedSumR = 4, kRedSumRhat = 8, kRedSumR0 = 12, kRedSumX = 16,
  kRedWords = 32, kRedCopies = 16, kRedTotal = kRedWords * kRedCopies
};
// Device scalars (d_scal).
enum : int {
  kScalGamma = 0, kScalRho = 1, kScalRelresOrig = 2, kScalRelresScaled = 3, kScalNormB = 4, kScalNormBhat = 5,
  kScalOut = 6, kScalWords = 8
};

hipError_t launch_residual(hipStream_t st, int64_t n, const int64_t *rp, const int32_t *col, const double *a,
                           const double *ahat, const double *b, const double *bhat, const double *x,
                           const double *cscale, double *r, double *rhat, unsigned long long *red, int lanes);
hipError_t launch_absmax(hipStream_t st, int64_t n, const double *x, unsigned long long *dst);
hipError_t launch_dnrm_sum(hipStream_t st, int64_t n, const double *x, const unsigned long long *mu,
                           unsigned long long *limbs);
hipError_t launch_fin_residual(hipStream_t st, const unsigned long long *red, const double *norms, double *scal);
hipError_t launch_fin_norm(hipStream_t st, const unsigned long long *red, double *out);
// *out = the maximum recorded in word w of the reduction block, as a double
hipError_t launch_fin_max(hipStream_t st, const unsigned long long *w, double *out);
hipError_t launch_start_vector(hipStream_t st, const CycleArgs &a, const double *r, double *scal, const double *lvalf,
                               const double *uvalf, double *bk, double *r0, unsigned long long *red);
hipError_t launch_spmv(hipStream_t st, const CycleArgs &a, int nterms, const int64_t *v, int64_t *z);
hipError_t launch_precond(hipStream_t st, const CycleArgs &a, const int64_t *z, int64_t *w);
hipError_t launch_reduce(hipStream_t st, int64_t n, const int64_t *w, const int64_t *v, int b, int df, int mode,
                         AccWords *parts, int64_t *out, CycleState *state, int64_t code);
hipError_t launch_axpy(hipStream_t st, int64_t n, int64_t h, int b, int df, int64_t *w, const int64_t *v,
                       CycleState *state);
hipError_t launch_normalize(hipStream_t st, int64_t n, const int64_t *w, int64_t den, int b1, int e, int64_t *v,
                            CycleState *state);

}  // namespace igm
