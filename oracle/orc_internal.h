/* Internal layout of the oracle's system object. TEST INFRASTRUCTURE ONLY. */
#ifndef ORC_INTERNAL_H
#define ORC_INTERNAL_H

#include "orc.h"

#define ORC_MAX_TERMS 8

struct orc_system {
  int64_t n, nnz;
  orc_policy pol;
  /* input pattern and values (CSR, columns strictly increasing per row) */
  int64_t *row_ptr;
  int32_t *col;
  int64_t *diag_pos; /* position of the diagonal entry in each row, -1 if absent */
  double *ahat, *bhat;
  /* initial scaling, eqs. (eq1)/(eq2), (eq3); cscale = sqrt(dhat) for eq. (eq2), else NULL */
  double *dhat, *a, *b, *cscale;
  /* integer matrices A_0..A_p on the input pattern, eq. (A) */
  int32_t nterms; /* p + 1 */
  int32_t alpha[ORC_MAX_TERMS + 1];
  int64_t *abar[ORC_MAX_TERMS + 1];
  /* preconditioner (Sec. VI-A) */
  double *lu;     /* FP64 ILU(0) of A on the pattern (ILU only) */
  int64_t *fac;   /* Lbar below, Ubar above the diagonal, on the pattern */
  int64_t *ldiag, *udiag;
  double bhat_norm;
};

#endif
