/*
 * The int-GMRES(m) call of the paper (Fig. 2, Sec. V) with the left
 * preconditioner of Sec. VI. TEST INFRASTRUCTURE ONLY (see orc.h).
 *
 * Readings of the paper taken here (each one also listed in the design notes):
 *  - right shifts are arithmetic (floor), divisions truncate toward zero;
 *  - the Gram-Schmidt inner product shifts only w (beta_2 = 0), its update
 *    shifts only h, the earlier rotations shift only the h entries
 *    (Sec. V-D.2, V-D.3);
 *  - the minus signs of the rotations (of H and of g) are applied to the
 *    operand s before the multiplication; the rotation of g uses the old g_j
 *    for both updates;
 *  - a zero (shifted) denominator in the normalisation ends the call after
 *    the Givens update of column j; in the new rotation it ends the call
 *    without column j.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "orc_internal.h"

typedef __int128 i128;

static int fits64(i128 x) { return x >= (i128)INT64_MIN && x <= (i128)INT64_MAX; }
static int64_t wrap64(i128 x) { return (int64_t)(uint64_t)(unsigned __int128)x; }

static void event(int64_t *first, int64_t code) {
  if (code < *first) *first = code;
}

/* Product of two int64 words; flags a product that leaves int64. */
static int64_t pmul(int64_t a, int64_t b, int32_t *ovf) {
  i128 p = (i128)a * (i128)b;
  if (!fits64(p)) *ovf = 1;
  return wrap64(p);
}

/* Integer SpMV (Fig. 2; Sec. V-C.3, eq. (matvec)): z = A_0 v + sum_{l=1..s} asr(A_l v, alpha_l).
 * Matrix entries have no fraction bits, v and z are Q df; no shift on A_0 v. */
void orc_spmv(const orc_system *s, int32_t nterms, const int64_t *v, int64_t *z, int32_t j, int64_t *first) {
  if (nterms > s->nterms) nterms = s->nterms;
  for (int64_t i = 0; i < s->n; ++i) {
    int32_t ovf = 0;
    i128 total = 0;
    for (int l = 0; l < nterms; ++l) {
      i128 acc = 0;
      for (int64_t e = s->row_ptr[i]; e < s->row_ptr[i + 1]; ++e) acc += pmul(s->abar[l][e], v[s->col[e]], &ovf);
      if (!fits64(acc)) ovf = 1;
      int64_t t = wrap64(acc);
      if (l > 0) t = orc_asr(t, s->alpha[l]);
      total += t;
    }
    if (!fits64(total)) ovf = 1;
    z[i] = wrap64(total);
    if (ovf) event(first, ORC_CODE(j, 1, 0));
  }
}

/* Preconditioner apply (Sec. VI, VI-A): w = Mbar^-1 z with Mbar = Lbar Ubar, by forward then
 * backward substitution in integers: the FP substitution with the data type
 * changed, so each division is C integer division (truncation). */
void orc_precond_apply(const orc_system *s, const int64_t *z, int64_t *w, int32_t j, int64_t *first) {
  int64_t n = s->n;
  if (s->pol.precond == ORC_PRE_NONE) {
    memcpy(w, z, sizeof(int64_t) * n);
    return;
  }
  int ilu = s->pol.precond == ORC_PRE_ILU0;
  int32_t ovf = 0;
  /* forward: Lbar y = z (y stored in w) */
  for (int64_t i = 0; i < n; ++i) {
    i128 acc = z[i];
    if (ilu)
      for (int64_t e = s->row_ptr[i]; e < s->diag_pos[i]; ++e) acc -= pmul(s->fac[e], w[s->col[e]], &ovf);
    if (!fits64(acc)) ovf = 1;
    w[i] = orc_tdiv(wrap64(acc), s->ldiag[i], &ovf);
  }
  /* backward: Ubar u = y (in place, rows in decreasing order) */
  for (int64_t i = n - 1; i >= 0; --i) {
    i128 acc = w[i];
    if (ilu)
      for (int64_t e = s->diag_pos[i] + 1; e < s->row_ptr[i + 1]; ++e) acc -= pmul(s->fac[e], w[s->col[e]], &ovf);
    if (!fits64(acc)) ovf = 1;
    w[i] = orc_tdiv(wrap64(acc), s->udiag[i], &ovf);
  }
  if (ovf) event(first, ORC_CODE(j, 2, 0));
}

#define HH(i, k) t->H[(size_t)(i) * m + (k)]

/* The paper makes s(k) a solver parameter bounded by S (Fig. 1) without a
 * rule; reading: either the same S in every refinement (the paper's
 * experiments, S = 0), or one more correction term per refinement, starting
 * from Abar_0 alone, until S is reached. */
int32_t orc_s_of_k(const orc_policy *p, int32_t k) {
  if (p->s_rule == 0) return p->s_terms;
  return k - 1 < p->s_terms ? k - 1 : p->s_terms;
}

int orc_cycle(const orc_system *s, const int64_t *v1, int32_t k, orc_trace *t) {
  const orc_policy *p = &s->pol;
  int64_t n = s->n;
  int32_t m = t->m, f = p->df;
  int64_t *z = (int64_t *)malloc(sizeof(int64_t) * n);
  int64_t *w = (int64_t *)malloc(sizeof(int64_t) * n);
  if (!z || !w) { free(z); free(w); return ORC_ERR_ARG; }
  memset(t->H, 0, sizeof(int64_t) * (size_t)(m + 1) * m);
  memset(t->c, 0, sizeof(int64_t) * m);
  memset(t->s, 0, sizeof(int64_t) * m);
  memset(t->g, 0, sizeof(int64_t) * (m + 1));
  memcpy(t->V, v1, sizeof(int64_t) * n);
  t->first_ovf = ORC_NO_EVENT;
  t->breakdown = 0;
  t->jstar = m;
  t->steps = 0;
  /* g = (1, 0, ..., 0) in Q df */
  t->g[0] = (int64_t)1 << f;
  int32_t nterms = orc_s_of_k(p, k) + 1;
  for (int32_t j = 1; j <= m; ++j) { /* Arnoldi step j */
    int32_t ovf;
    const int64_t *vj = t->V + (size_t)(j - 1) * n;
    t->steps = j;
    /* SpMV, then the preconditioner apply */
    orc_spmv(s, nterms, vj, z, j, &t->first_ovf);
    orc_precond_apply(s, z, w, j, &t->first_ovf);
    /* modified Gram-Schmidt, i in increasing order */
    for (int32_t i = 1; i <= j; ++i) {
      const int64_t *vi = t->V + (size_t)(i - 1) * n;
      ovf = 0;
      int64_t h = orc_dot(n, w, vi, p->b_dot, f, &ovf); /* h_ij = (w, v_i) */
      if (ovf) event(&t->first_ovf, ORC_CODE(j, 3, 2 * (i - 1)));
      HH(i - 1, j - 1) = h;
      ovf = 0; /* w -= h_ij v_i */
      orc_axpy(n, w, vi, h, p->b_axpy, f, &ovf);
      if (ovf) event(&t->first_ovf, ORC_CODE(j, 3, 2 * (i - 1) + 1));
    }
    /* h_{j+1,j} = ||w|| */
    ovf = 0;
    int64_t hn = orc_norm(n, w, p->b_norm, f, &ovf);
    if (ovf) event(&t->first_ovf, ORC_CODE(j, 4, 0));
    HH(j, j - 1) = hn;
    /* normalisation: v_{j+1} = w / h_{j+1,j} (division of Sec. V-B.3) */
    int64_t den = orc_asr(hn, p->b_div_den);
    int lucky = den == 0;
    if (!lucky) {
      ovf = 0;
      orc_normalize(n, w, den, p->b_div_num, p->b_div_den, f, t->V + (size_t)j * n, &ovf);
      if (ovf) event(&t->first_ovf, ORC_CODE(j, 5, 0));
    }
    /* apply the previous rotations to column j */
    for (int32_t i = 1; i <= j - 1; ++i) {
      int64_t a = orc_asr(HH(i - 1, j - 1), p->b_rot);
      int64_t b = orc_asr(HH(i, j - 1), p->b_rot);
      int64_t c = t->c[i - 1], sn = t->s[i - 1];
      ovf = 0;
      int64_t msn = wrap64(-(i128)sn);
      if (!fits64(-(i128)sn)) ovf = 1;
      i128 top = (i128)pmul(c, a, &ovf) + pmul(sn, b, &ovf);
      i128 bot = (i128)pmul(msn, a, &ovf) + pmul(c, b, &ovf);
      if (!fits64(top) || !fits64(bot)) ovf = 1;
      HH(i - 1, j - 1) = orc_asr(wrap64(top), f - p->b_rot);
      HH(i, j - 1) = orc_asr(wrap64(bot), f - p->b_rot);
      if (ovf) event(&t->first_ovf, ORC_CODE(j, 6, i));
    }
    /* rotation radius: tmp = sqrt(h_jj^2 + h_{j+1,j}^2), a 2-element norm */
    ovf = 0;
    int64_t pair[2] = {HH(j - 1, j - 1), HH(j, j - 1)};
    int64_t tmp = orc_norm(2, pair, p->b_tmp, f, &ovf);
    if (ovf) event(&t->first_ovf, ORC_CODE(j, 7, 0));
    /* new rotation: c_j = h_jj / tmp, s_j = h_{j+1,j} / tmp */
    ovf = 0;
    int32_t zero = 0;
    int64_t cj = orc_div(pair[0], tmp, p->b_cs_num, p->b_cs_den, f, &ovf, &zero);
    int64_t sj = orc_div(pair[1], tmp, p->b_cs_num, p->b_cs_den, f, &ovf, &zero);
    if (zero) { /* H_j singular: column j cannot be used */
      t->breakdown = 2;
      t->jstar = j - 1;
      break;
    }
    if (ovf) event(&t->first_ovf, ORC_CODE(j, 8, 0));
    t->c[j - 1] = cj;
    t->s[j - 1] = sj;
    /* rotation of g: products of Q df numbers without operand shifts */
    ovf = 0;
    int64_t gj = t->g[j - 1];
    int64_t msj = wrap64(-(i128)sj);
    if (!fits64(-(i128)sj)) ovf = 1;
    t->g[j - 1] = orc_asr(pmul(cj, gj, &ovf), f);
    t->g[j] = orc_asr(pmul(msj, gj, &ovf), f);
    if (ovf) event(&t->first_ovf, ORC_CODE(j, 9, 0));
    /* h_jj = tmp, h_{j+1,j} = 0 */
    HH(j - 1, j - 1) = tmp;
    HH(j, j - 1) = 0;
    if (lucky) {
      t->breakdown = 1;
      t->jstar = j;
      break;
    }
    if (p->gtol >= 0) {
      int64_t gn = t->g[j] < 0 ? -t->g[j] : t->g[j];
      if (gn <= p->gtol) { t->jstar = j; break; }
    }
  }
  free(z);
  free(w);
  return ORC_OK;
}

/* Closing FP64 step of Fig. 2: cast H and g to FP (exact scaling by 2^-df), y = rho H^-1 g by
 * back substitution (row i: y_i = (g_i - sum_{k>i} H_ik y_k) / H_ii with the
 * sum over k increasing), then x_l = sum_{i} y_i * (v_il 2^-df), i increasing. */
void orc_cycle_update(const orc_system *s, const orc_trace *t, double rho, double *x) {
  int64_t n = s->n;
  int32_t m = t->m, js = t->jstar, f = s->pol.df;
  double *y = (double *)malloc(sizeof(double) * (js > 0 ? js : 1));
  for (int32_t i = js - 1; i >= 0; --i) {
    double acc = 0.0;
    for (int32_t k = i + 1; k < js; ++k) acc = acc + ldexp((double)HH(i, k), -f) * y[k];
    y[i] = (ldexp((double)t->g[i], -f) - acc) / ldexp((double)HH(i, i), -f);
  }
  for (int32_t i = 0; i < js; ++i) y[i] = rho * y[i];
  for (int64_t l = 0; l < n; ++l) {
    double acc = 0.0;
    for (int32_t i = 0; i < js; ++i) acc = acc + y[i] * ldexp((double)t->V[(size_t)i * n + l], -f);
    x[l] = acc;
  }
  free(y);
}
