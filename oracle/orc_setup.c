/*
 * Setup of the oracle system: initial scaling (Sec. III), integer matrices
 * A_0..A_p (Sec. IV-B) and the integer ILU(0) / Jacobi preconditioner
 * (Sec. VI-A). TEST INFRASTRUCTURE ONLY (see orc.h).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "orc_internal.h"

static int bad_shift(int32_t b, int32_t df) { return b < 0 || b > df; }

static int check_policy(const orc_policy *p) {
  if (p->df < 1 || p->df > 62) return 1;
  if (p->alpha_a < 0 || p->alpha_a > 62) return 1;
  if (p->m < 1 || p->m > 4096) return 1;
  if (p->s_terms < 0 || p->s_terms > ORC_MAX_TERMS) return 1;
  if (p->precond < ORC_PRE_NONE || p->precond > ORC_PRE_ILU0) return 1;
  if (bad_shift(p->b_dot, p->df) || bad_shift(p->b_axpy, p->df) || bad_shift(p->b_rot, p->df)) return 1;
  if (p->b_norm < 0 || 2 * p->b_norm > 2 * p->df) return 1;
  if (p->b_tmp < 0 || p->b_tmp > p->df) return 1;
  if (bad_shift(p->b_div_num, 62) || bad_shift(p->b_div_den, 62)) return 1;
  if (bad_shift(p->b_cs_num, 62) || bad_shift(p->b_cs_den, 62)) return 1;
  if (p->max_refine < 0) return 1;
  if (p->shift_retry < 0 || p->shift_retry > 64) return 1;
  if (p->two_sided < 0 || p->two_sided > 1) return 1;
  if (p->gauss_seidel < 0 || p->gauss_seidel > 1) return 1;
  if (p->gauss_seidel && p->precond != ORC_PRE_ILU0) return 1;
  if (p->s_rule < 0 || p->s_rule > 1) return 1;
  if (!(p->tol >= 0.0)) return 1;
  return 0;
}

void orc_destroy(orc_system *s) {
  if (!s) return;
  free(s->row_ptr); free(s->col); free(s->diag_pos); free(s->ahat); free(s->bhat);
  free(s->dhat); free(s->a); free(s->b); free(s->cscale);
  for (int l = 0; l <= ORC_MAX_TERMS; ++l) free(s->abar[l]);
  free(s->lu); free(s->fac); free(s->ldiag); free(s->udiag);
  free(s);
}

/* Eq. (eq3): dhat_i = max_j |ahat_ij| / 2^alpha_a; eq. (eq1): A = Dhat^-1 Ahat,
 * b = Dhat^-1 bhat, each entry obtained by one FP64 division.
 * Eq. (eq2) (two_sided; the paper leaves D1 and D2 open, this reading takes
 * D1 = D2 = Dhat^(1/2) so a symmetric Ahat stays symmetric): s_i = sqrt(dhat_i),
 * a_ij = ahat_ij / (s_i * s_j), b_i = bhat_i / s_i, x = D2 xhat. */
static int scale(orc_system *s) {
  for (int64_t i = 0; i < s->n; ++i) {
    double mu = 0.0;
    for (int64_t e = s->row_ptr[i]; e < s->row_ptr[i + 1]; ++e)
      if (fabs(s->ahat[e]) > mu) mu = fabs(s->ahat[e]);
    if (mu == 0.0) return ORC_ERR_SINGULAR_ROW;
    double d = ldexp(mu, -s->pol.alpha_a);
    if (d == 0.0 || !isfinite(d)) return ORC_ERR_RANGE;
    s->dhat[i] = d;
    if (!s->cscale) {
      for (int64_t e = s->row_ptr[i]; e < s->row_ptr[i + 1]; ++e) s->a[e] = s->ahat[e] / d;
      s->b[i] = s->bhat[i] / d;
    } else {
      s->cscale[i] = sqrt(d);
    }
  }
  if (s->cscale) {
    for (int64_t i = 0; i < s->n; ++i) {
      for (int64_t e = s->row_ptr[i]; e < s->row_ptr[i + 1]; ++e)
        s->a[e] = s->ahat[e] / (s->cscale[i] * s->cscale[s->col[e]]);
      s->b[i] = s->bhat[i] / s->cscale[i];
    }
  }
  return ORC_OK;
}

/* Sec. IV-B: A_0 = trunc(A); then repeatedly take the remainder R, its
 * exponent alpha_l = alpha_a - floor(log2 max|R|) (eq. (alpha1)), and
 * A_l = trunc(R * 2^alpha_l), so A = A_0 + sum_l 2^-alpha_l A_l (eq. (A)). */
static int build_terms(orc_system *s) {
  int64_t nnz = s->nnz;
  int32_t rerr = 0;
  double *R = (double *)malloc(sizeof(double) * (nnz ? nnz : 1));
  if (!R) return ORC_ERR_ARG;
  s->abar[0] = (int64_t *)malloc(sizeof(int64_t) * (nnz ? nnz : 1));
  s->alpha[0] = 0;
  for (int64_t e = 0; e < nnz; ++e) {
    s->abar[0][e] = orc_trunc(s->a[e], &rerr);
    R[e] = s->a[e] - (double)s->abar[0][e]; /* exact: fractional part */
  }
  s->nterms = 1;
  for (int l = 1; l <= s->pol.s_terms; ++l) {
    double mu = 0.0;
    for (int64_t e = 0; e < nnz; ++e)
      if (fabs(R[e]) > mu) mu = fabs(R[e]);
    if (mu == 0.0) break; /* A represented exactly by the terms so far */
    int ex;
    frexp(mu, &ex); /* mu = f * 2^ex, f in [0.5, 1): floor(log2 mu) = ex - 1 */
    int32_t al = s->pol.alpha_a - (ex - 1);
    if (al > 1070) break;
    s->alpha[l] = al;
    s->abar[l] = (int64_t *)malloc(sizeof(int64_t) * (nnz ? nnz : 1));
    for (int64_t e = 0; e < nnz; ++e) {
      double t = ldexp(R[e], al);
      s->abar[l][e] = orc_trunc(t, &rerr);
      R[e] = ldexp(t - (double)s->abar[l][e], -al); /* exact remainder */
    }
    s->nterms = l + 1;
  }
  free(R);
  return rerr ? ORC_ERR_RANGE : ORC_OK;
}

/* FP64 ILU(0) of the scaled A restricted to its pattern, row by row (IKJ):
 * for each row i and each k < i of the row in increasing order, the
 * multiplier a_ik /= a_kk, then a_ij -= a_ik * a_kj for every j > k present in
 * both rows. Result: multipliers (L, unit diagonal) below, U on and above. */
static int ilu0(orc_system *s) {
  int64_t n = s->n;
  double *lu = s->lu;
  int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * n);
  if (!pos) return ORC_ERR_ARG;
  for (int64_t j = 0; j < n; ++j) pos[j] = -1;
  memcpy(lu, s->a, sizeof(double) * s->nnz);
  int rc = ORC_OK;
  for (int64_t i = 0; i < n && rc == ORC_OK; ++i) {
    for (int64_t e = s->row_ptr[i]; e < s->row_ptr[i + 1]; ++e) pos[s->col[e]] = e;
    for (int64_t e = s->row_ptr[i]; e < s->row_ptr[i + 1]; ++e) {
      int64_t k = s->col[e];
      if (k >= i) break;
      double piv = lu[s->diag_pos[k]];
      if (piv == 0.0) { rc = ORC_ERR_ZERO_PIVOT; break; }
      lu[e] = lu[e] / piv;
      for (int64_t f = s->diag_pos[k] + 1; f < s->row_ptr[k + 1]; ++f) {
        int64_t q = pos[s->col[f]];
        if (q >= 0) lu[q] = lu[q] - lu[e] * lu[f];
      }
    }
    for (int64_t e = s->row_ptr[i]; e < s->row_ptr[i + 1]; ++e) pos[s->col[e]] = -1;
    if (rc == ORC_OK && lu[s->diag_pos[i]] == 0.0) rc = ORC_ERR_ZERO_PIVOT;
  }
  free(pos);
  return rc;
}

/* Gauss-Seidel splitting (policy gauss_seidel; a reading: the paper reports
 * a Gauss-Seidel preconditioner, Sec. VII-D, without its construction):
 * M = D + L_A (the diagonal and the strict lower part of A) written as
 * L D U with L = I + L_A D^-1 and U = I. The multipliers below the diagonal
 * are a_ik / a_kk, nothing is eliminated and no entry remains above the
 * diagonal; the split of eqs. (dl)-(u1) then gives Lbar and a diagonal Ubar. */
static int gs_split(orc_system *s) {
  double *lu = s->lu;
  memcpy(lu, s->a, sizeof(double) * s->nnz);
  for (int64_t i = 0; i < s->n; ++i) {
    for (int64_t e = s->row_ptr[i]; e < s->row_ptr[i + 1]; ++e) {
      int64_t k = s->col[e];
      if (k < i) {
        double piv = s->a[s->diag_pos[k]];
        if (piv == 0.0) return ORC_ERR_ZERO_PIVOT;
        lu[e] = s->a[e] / piv;
      } else if (k > i) {
        lu[e] = 0.0;
      }
    }
    if (lu[s->diag_pos[i]] == 0.0) return ORC_ERR_ZERO_PIVOT;
  }
  return ORC_OK;
}

/* Eqs. (dl), (dl2), (l1), (u1): D_l = |d|^1/2, D_u = sgn(d)|d|^1/2,
 * Ltilde = L D_l, Utilde = D_u U (U with unit diagonal, i.e. the stored upper
 * entries divided by d_i), then each entry cast to int64. */
static int cast_factors(orc_system *s, const double *dvals, int with_offdiag) {
  int32_t rerr = 0;
  int64_t n = s->n;
  for (int64_t i = 0; i < n; ++i) {
    double d = dvals[i];
    if (d == 0.0 || !isfinite(d)) return ORC_ERR_ZERO_PIVOT;
    double dl = sqrt(fabs(d));
    double du = d < 0.0 ? -dl : dl;
    s->ldiag[i] = orc_trunc(dl, &rerr);
    s->udiag[i] = orc_trunc(du, &rerr);
    if (rerr) return ORC_ERR_RANGE;
    if (s->ldiag[i] == 0 || s->udiag[i] == 0) return ORC_ERR_ZERO_PIVOT;
    if (!with_offdiag) continue;
    for (int64_t e = s->row_ptr[i]; e < s->row_ptr[i + 1]; ++e) {
      int64_t j = s->col[e];
      if (j < i) {
        double dj = sqrt(fabs(dvals[j]));
        s->fac[e] = orc_trunc(s->lu[e] * dj, &rerr);
      } else if (j > i) {
        s->fac[e] = orc_trunc(du * (s->lu[e] / d), &rerr);
      }
    }
    if (rerr) return ORC_ERR_RANGE;
  }
  return ORC_OK;
}

static int build_precond(orc_system *s) {
  int64_t n = s->n;
  if (s->pol.precond == ORC_PRE_NONE) return ORC_OK;
  for (int64_t i = 0; i < n; ++i)
    if (s->diag_pos[i] < 0) return ORC_ERR_ZERO_PIVOT;
  s->fac = (int64_t *)calloc(s->nnz ? s->nnz : 1, sizeof(int64_t));
  s->ldiag = (int64_t *)malloc(sizeof(int64_t) * n);
  s->udiag = (int64_t *)malloc(sizeof(int64_t) * n);
  double *dv = (double *)malloc(sizeof(double) * n);
  if (!s->fac || !s->ldiag || !s->udiag || !dv) { free(dv); return ORC_ERR_ARG; }
  int rc;
  if (s->pol.precond == ORC_PRE_ILU0) {
    s->lu = (double *)malloc(sizeof(double) * (s->nnz ? s->nnz : 1));
    if (!s->lu) { free(dv); return ORC_ERR_ARG; }
    rc = s->pol.gauss_seidel ? gs_split(s) : ilu0(s);
    if (rc == ORC_OK) {
      for (int64_t i = 0; i < n; ++i) dv[i] = s->lu[s->diag_pos[i]];
      rc = cast_factors(s, dv, 1);
    }
  } else {
    /* Jacobi: the same construction on the diagonal-only pattern. */
    for (int64_t i = 0; i < n; ++i) dv[i] = s->a[s->diag_pos[i]];
    rc = cast_factors(s, dv, 0);
  }
  free(dv);
  return rc;
}

int orc_create(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val, const double *b,
               const orc_policy *pol, orc_system **out) {
  *out = NULL;
  if (n < 1 || !row_ptr || !col || !val || !b || !pol) return ORC_ERR_ARG;
  if (check_policy(pol)) return ORC_ERR_ARG;
  if (row_ptr[0] != 0) return ORC_ERR_ARG;
  for (int64_t i = 0; i < n; ++i) {
    if (row_ptr[i + 1] < row_ptr[i]) return ORC_ERR_ARG;
    for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e) {
      if (col[e] < 0 || col[e] >= n) return ORC_ERR_ARG;
      if (e > row_ptr[i] && col[e] <= col[e - 1]) return ORC_ERR_ARG;
      if (!isfinite(val[e])) return ORC_ERR_ARG;
    }
    if (!isfinite(b[i])) return ORC_ERR_ARG;
  }
  int64_t nnz = row_ptr[n];
  orc_system *s = (orc_system *)calloc(1, sizeof(orc_system));
  if (!s) return ORC_ERR_ARG;
  s->n = n;
  s->nnz = nnz;
  s->pol = *pol;
  size_t nz = nnz ? (size_t)nnz : 1;
  s->row_ptr = (int64_t *)malloc(sizeof(int64_t) * (n + 1));
  s->col = (int32_t *)malloc(sizeof(int32_t) * nz);
  s->diag_pos = (int64_t *)malloc(sizeof(int64_t) * n);
  s->ahat = (double *)malloc(sizeof(double) * nz);
  s->bhat = (double *)malloc(sizeof(double) * n);
  s->dhat = (double *)malloc(sizeof(double) * n);
  s->a = (double *)malloc(sizeof(double) * nz);
  s->b = (double *)malloc(sizeof(double) * n);
  if (pol->two_sided) s->cscale = (double *)malloc(sizeof(double) * n);
  if (!s->row_ptr || !s->col || !s->diag_pos || !s->ahat || !s->bhat || !s->dhat || !s->a || !s->b ||
      (pol->two_sided && !s->cscale)) {
    orc_destroy(s);
    return ORC_ERR_ARG;
  }
  memcpy(s->row_ptr, row_ptr, sizeof(int64_t) * (n + 1));
  memcpy(s->col, col, sizeof(int32_t) * nnz);
  memcpy(s->ahat, val, sizeof(double) * nnz);
  memcpy(s->bhat, b, sizeof(double) * n);
  for (int64_t i = 0; i < n; ++i) {
    s->diag_pos[i] = -1;
    for (int64_t e = row_ptr[i]; e < row_ptr[i + 1]; ++e)
      if (col[e] == i) s->diag_pos[i] = e;
  }
  int rc = scale(s);
  if (rc == ORC_OK) rc = build_terms(s);
  if (rc == ORC_OK) rc = build_precond(s);
  if (rc != ORC_OK) { orc_destroy(s); return rc; }
  s->bhat_norm = orc_dnrm(n, s->bhat);
  *out = s;
  return ORC_OK;
}

int64_t orc_n(const orc_system *s) { return s->n; }
int64_t orc_nnz(const orc_system *s) { return s->nnz; }
int32_t orc_nterms(const orc_system *s) { return s->nterms; }

void orc_get_scaled(const orc_system *s, double *dhat, double *a, double *b) {
  if (dhat) memcpy(dhat, s->dhat, sizeof(double) * s->n);
  if (a) memcpy(a, s->a, sizeof(double) * s->nnz);
  if (b) memcpy(b, s->b, sizeof(double) * s->n);
}

void orc_get_terms(const orc_system *s, int64_t *abar, int32_t *alpha) {
  for (int l = 0; l < s->nterms; ++l) {
    if (abar) memcpy(abar + (size_t)l * s->nnz, s->abar[l], sizeof(int64_t) * s->nnz);
    if (alpha) alpha[l] = s->alpha[l];
  }
}

void orc_get_precond(const orc_system *s, int64_t *fac, int64_t *ldiag, int64_t *udiag) {
  if (s->pol.precond == ORC_PRE_NONE) return;
  if (fac) memcpy(fac, s->fac, sizeof(int64_t) * s->nnz);
  if (ldiag) memcpy(ldiag, s->ldiag, sizeof(int64_t) * s->n);
  if (udiag) memcpy(udiag, s->udiag, sizeof(int64_t) * s->n);
}

int orc_get_ilu_fp(const orc_system *s, double *lu) {
  if (!s->lu) return 0;
  memcpy(lu, s->lu, sizeof(double) * s->nnz);
  return 1;
}
