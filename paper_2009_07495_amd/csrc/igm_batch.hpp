// Device records of the batched solver (many independent systems, one
// persistent launch).
#pragma once

#include "igm_internal.hpp"

namespace igm {

// One system of a batch: read-only inputs and setup products, its Krylov
// basis and its team exchange area. Field names of the integer matrix match
// CycleArgs so the per-row SpMV serves both kernels.
struct BatchSys {
  int64_t n;       // rows
  int64_t ldv;     // leading dimension of V (n rounded up to 16)
  int64_t x_off;   // offset of this system's unknowns in the solution vector
  int32_t team;    // workgroups that share the system
  int32_t nterms;  // integer matrix terms used by line 5
  int32_t alpha[kMaxTerms];
  const int64_t *row_ptr;
  const int32_t *col;
  const double *a, *ahat, *b, *bhat;  // scaled and original FP64 matrix / rhs
  const int64_t *sell_off;
  const int32_t *sell_w;
  const int32_t *sell_col;
  const int64_t *sell_val[kMaxTerms];
  const int64_t *ldiag, *udiag;  // cast diagonals of the Jacobi preconditioner
  int64_t *V;                    // (m+1) x ldv basis
  unsigned long long *words;     // kTeamSlots x kTeamWords exchange words
};

// Outcome of one system, written by its first member.
struct BatchResult {
  int32_t status, refinements, iterations, jstar;
  int64_t first_ovf;
  double relres_orig, relres_scaled;
  uint64_t t_begin, t_end;  // device wall clock (start and end of the solve)
  // wall-clock ticks of the first member's thread 0 per phase: 0 SpMV +
  // preconditioner, 1 inner products and updates (local work), 2 waits for
  // the inner-product sums, 3 norm, 4 normalisation, 5 FP64 refinement steps
  // (residual, norms, lines 1'-2, lines 21-23), 6 end-of-step barriers
  uint64_t phase[8];
};

struct BatchArgs {
  const BatchSys *sys;
  const int32_t *jobs;  // pairs (system, member) in claim order
  int32_t njobs;
  int32_t m, df, precond;
  int32_t b_dot, b_axpy, b_norm, b_div_num, b_div_den, b_rot, b_tmp, b_cs_num, b_cs_den;
  int32_t max_refine;
  int32_t phase_clock;  // record the phase clocks of each system's first member
  int64_t gtol;
  double tol;
  int32_t *queue;  // next job to claim
  int32_t *timeout;
  BatchResult *res;
  double *x;  // concatenated solutions (in: start, out: result)
};

const void *batch_kernel(int block, int R, int pre);
size_t batch_smem_bytes(int m);
// the (block, rows per thread) shapes instantiated for the batched kernel
extern const int kBatchShapes[][2];
extern const int kNumBatchShapes;

}  // namespace igm
