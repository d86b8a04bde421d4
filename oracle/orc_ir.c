/*
 * FP64 iterative refinement around the integer GMRES call (Sec. IV, Fig. 1)
 * and the FP64 steps of Fig. 2 and Sec. VI (start vector, closing least-squares
 * step).
 * TEST INFRASTRUCTURE ONLY (see orc.h).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "orc_internal.h"

/* uint128 -> double, rounded to nearest (ties to even); gcc's conversion. */
double orc_u128_to_double(uint64_t lo, uint64_t hi) {
  unsigned __int128 v = ((unsigned __int128)hi << 64) | lo;
  return (double)v;
}

/* Order-free FP64 2-norm (a reproducibility rule of this implementation; the
 * paper only says the norm is taken in FP): mu = max|x_i|; each (x_i/mu)^2 is
 * rounded once, scaled by 2^96 and floored to an integer; the integers are
 * summed exactly; the sum is rounded once to double; ||x|| = mu * sqrt(S) 2^-48.
 * The relative error stays within a few ulps of the textbook norm and the
 * result does not depend on the summation order. Requires n < 2^32. */
double orc_dnrm(int64_t n, const double *x) {
  double mu = 0.0;
  for (int64_t i = 0; i < n; ++i)
    if (fabs(x[i]) > mu) mu = fabs(x[i]);
  if (mu == 0.0 || !isfinite(mu)) return mu;
  unsigned __int128 S = 0;
  for (int64_t i = 0; i < n; ++i) {
    double t = x[i] / mu;
    double q = ldexp(t * t, 96);
    S += (unsigned __int128)floor(q);
  }
  double D = orc_u128_to_double((uint64_t)S, (uint64_t)(S >> 64));
  return mu * ldexp(sqrt(D), -48);
}

/* r = b - A x (scaled system, eq. (b)) and rhat = bhat - Ahat x (original
 * system, eq. (org)); each row sums its products in CSR order, then one
 * subtraction. */
void orc_residual(const orc_system *s, const double *x, double *r, double *rhat) {
  for (int64_t i = 0; i < s->n; ++i) {
    double acc = 0.0, acch = 0.0;
    for (int64_t e = s->row_ptr[i]; e < s->row_ptr[i + 1]; ++e) {
      acc = acc + s->a[e] * x[s->col[e]];
      acch = acch + s->ahat[e] * x[s->col[e]];
    }
    /* eq. (eq2): x holds xhat; the scaled residual is D1^-1 (bhat - Ahat xhat) */
    if (r) r[i] = s->cscale ? (s->bhat[i] - acch) / s->cscale[i] : s->b[i] - acc;
    if (rhat) rhat[i] = s->bhat[i] - acch;
  }
}

/* FP64 start step (Sec. VI): r0 = Mbar^-1 bk in FP64 with the integer factors converted to
 * double: forward rows in increasing order, backward in decreasing order;
 * each row sums its off-diagonal products in CSR order, subtracts, divides. */
static void precond_fp(const orc_system *s, const double *bk, double *u) {
  int64_t n = s->n;
  if (s->pol.precond == ORC_PRE_NONE) {
    memcpy(u, bk, sizeof(double) * n);
    return;
  }
  int ilu = s->pol.precond == ORC_PRE_ILU0;
  for (int64_t i = 0; i < n; ++i) {
    double acc = 0.0;
    if (ilu)
      for (int64_t e = s->row_ptr[i]; e < s->diag_pos[i]; ++e) acc = acc + (double)s->fac[e] * u[s->col[e]];
    u[i] = (bk[i] - acc) / (double)s->ldiag[i];
  }
  for (int64_t i = n - 1; i >= 0; --i) {
    double acc = 0.0;
    if (ilu)
      for (int64_t e = s->diag_pos[i] + 1; e < s->row_ptr[i + 1]; ++e) acc = acc + (double)s->fac[e] * u[s->col[e]];
    u[i] = (u[i] - acc) / (double)s->udiag[i];
  }
}

/* Eqs. (gammak), (scale), then the start step and cast of Fig. 2 and Sec. VI
 * with x^(k) = 0:
 * gamma = max|r|, bk = r / gamma, r0 = Mbar^-1 bk, rho = ||r0||,
 * v1 = trunc(2^df * r0 / rho). Returns ORC_ERR_RANGE if a cast fails and
 * ORC_OK otherwise; gamma == 0 means r == 0. */
int orc_start_vector(const orc_system *s, const double *r, double *bk, double *r0, int64_t *v1, double *gamma,
                     double *rho) {
  int64_t n = s->n;
  double g = 0.0;
  for (int64_t i = 0; i < n; ++i)
    if (fabs(r[i]) > g) g = fabs(r[i]);
  *gamma = g;
  *rho = 0.0;
  if (g == 0.0) return ORC_OK;
  for (int64_t i = 0; i < n; ++i) bk[i] = r[i] / g;
  precond_fp(s, bk, r0);
  double rh = orc_dnrm(n, r0);
  *rho = rh;
  if (!(rh > 0.0) || !isfinite(rh)) return ORC_ERR_RANGE;
  int32_t rerr = 0;
  for (int64_t i = 0; i < n; ++i) v1[i] = orc_trunc(ldexp(r0[i] / rh, s->pol.df), &rerr);
  return rerr ? ORC_ERR_RANGE : ORC_OK;
}

static double relres(double rn, double bn) {
  if (bn > 0.0) return rn / bn;
  return rn == 0.0 ? 0.0 : INFINITY;
}

static int shrink_exponent(int32_t *num, int32_t *den) {
  int32_t *e = *num > 0 ? num : (*den > 0 ? den : NULL);
  if (!e) return 0;
  *e = *e > 4 ? *e - 4 : 0;
  return 1;
}

int orc_shift_retry(orc_policy *p, int64_t code) {
  if (code == ORC_NO_EVENT) return 0;
  int32_t stage = (int32_t)((code >> 16) & 0xFF);
  int32_t sub = (int32_t)(code & 0xFFFF);
  int32_t *b;
  switch (stage) {
    case 3: b = (sub % 2 == 0) ? &p->b_dot : &p->b_axpy; break; /* inner product / update */
    case 4: b = &p->b_norm; break;                               /* norm */
    case 6: b = &p->b_rot; break;                                /* earlier rotations */
    case 7: b = &p->b_tmp; break;                                /* rotation radius */
    case 5: return shrink_exponent(&p->b_div_num, &p->b_div_den); /* normalisation */
    case 8: return shrink_exponent(&p->b_cs_num, &p->b_cs_den);   /* new rotation */
    default: return 0;                                             /* SpMV, preconditioner, rotation of g */
  }
  if (*b >= p->df) return 0;
  *b = *b + 4 > p->df ? p->df : *b + 4;
  return 1;
}

void orc_get_policy(const orc_system *s, orc_policy *out) { *out = s->pol; }

/* Fig. 1: refine x until the FP64 relative residual of the original system
 * drops below tol; each refinement solves Abar^(k) x^(k) = b^(k) with one
 * int-GMRES(m) call and adds gamma^(k) x^(k) (eq. (update)). */
int orc_solve(orc_system *s, double *x, orc_stats *st) {
  int64_t n = s->n;
  int32_t m = s->pol.m;
  double *r = (double *)malloc(sizeof(double) * n);
  double *rh = (double *)malloc(sizeof(double) * n);
  double *bk = (double *)malloc(sizeof(double) * n);
  double *r0 = (double *)malloc(sizeof(double) * n);
  double *xk = (double *)malloc(sizeof(double) * n);
  int64_t *v1 = (int64_t *)malloc(sizeof(int64_t) * n);
  orc_trace t;
  memset(&t, 0, sizeof(t));
  t.m = m;
  t.H = (int64_t *)malloc(sizeof(int64_t) * (size_t)(m + 1) * m);
  t.c = (int64_t *)malloc(sizeof(int64_t) * m);
  t.s = (int64_t *)malloc(sizeof(int64_t) * m);
  t.g = (int64_t *)malloc(sizeof(int64_t) * (m + 1));
  t.V = (int64_t *)malloc(sizeof(int64_t) * (size_t)n * (m + 1));
  st->status = ORC_NOT_CONVERGED;
  st->refinements = 0;
  st->iterations = 0;
  st->first_ovf = ORC_NO_EVENT;
  st->shift_retries = 0;
  if (!r || !rh || !bk || !r0 || !xk || !v1 || !t.H || !t.c || !t.s || !t.g || !t.V) {
    st->status = ORC_ERR_ARG;
    goto done;
  }
  double bn_s = orc_dnrm(n, s->b);
  for (int32_t k = 0;; ++k) {
    orc_residual(s, x, r, rh);
    double ro = relres(orc_dnrm(n, rh), s->bhat_norm);
    double rs = relres(orc_dnrm(n, r), bn_s);
    st->relres_orig = ro;
    st->relres_scaled = rs;
    if (k < st->hist_cap) {
      if (st->hist_relres_orig) st->hist_relres_orig[k] = ro;
      if (st->hist_relres_scaled) st->hist_relres_scaled[k] = rs;
    }
    if (!isfinite(ro)) { st->status = ORC_ERR_RANGE; break; }
    if (ro < s->pol.tol) { st->status = ORC_OK; break; }
    if (k >= s->pol.max_refine) { st->status = ORC_NOT_CONVERGED; break; }
    double gamma, rho;
    int rc = orc_start_vector(s, r, bk, r0, v1, &gamma, &rho);
    if (k < st->hist_cap) {
      if (st->hist_gamma) st->hist_gamma[k] = gamma;
      if (st->hist_rho) st->hist_rho[k] = rho;
    }
    if (rc != ORC_OK) { st->status = rc; break; }
    if (gamma == 0.0) { st->status = ORC_OK; break; }
    /* the call, repeated from the same v1 while a retry can adjust a shift */
    for (;;) {
      orc_cycle(s, v1, k + 1, &t);
      if (t.first_ovf == ORC_NO_EVENT || st->shift_retries >= s->pol.shift_retry) break;
      if (!orc_shift_retry(&s->pol, t.first_ovf)) break;
      st->shift_retries += 1;
    }
    st->refinements += 1;
    st->iterations += t.steps;
    if (k < st->hist_cap && st->hist_jstar) st->hist_jstar[k] = t.jstar;
    if (t.first_ovf != ORC_NO_EVENT) {
      st->first_ovf = t.first_ovf;
      st->status = ORC_ERR_OVERFLOW;
      break;
    }
    if (t.jstar == 0) { st->status = ORC_ERR_BREAKDOWN; break; }
    orc_cycle_update(s, &t, rho, xk);
    /* eq. (update); with eq. (eq2) the correction returns to xhat = D2^-1 x */
    for (int64_t l = 0; l < n; ++l) x[l] = x[l] + gamma * (s->cscale ? xk[l] / s->cscale[l] : xk[l]);
  }
done:
  free(r); free(rh); free(bk); free(r0); free(xk); free(v1);
  free(t.H); free(t.c); free(t.s); free(t.g); free(t.V);
  return st->status;
}
