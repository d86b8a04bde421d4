/*
 * The paper's comparator ("Double", Sec. VII-A): standard FP64 GMRES(m),
 * restarted every m iterations, with the FP64 relative residual of the
 * original system checked once per restart. Used only for iteration-count
 * context in tests. Left preconditioning with the FP64 ILU(0) (L unit lower,
 * U upper with the pivots) or the diagonal of A. TEST INFRASTRUCTURE ONLY.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include "orc_internal.h"

static void apply_m(const orc_system *s, const double *r, double *u) {
  int64_t n = s->n;
  if (s->pol.precond == ORC_PRE_NONE) { memcpy(u, r, sizeof(double) * n); return; }
  if (s->pol.precond == ORC_PRE_JACOBI) {
    for (int64_t i = 0; i < n; ++i) u[i] = r[i] / s->a[s->diag_pos[i]];
    return;
  }
  for (int64_t i = 0; i < n; ++i) {
    double acc = r[i];
    for (int64_t e = s->row_ptr[i]; e < s->diag_pos[i]; ++e) acc -= s->lu[e] * u[s->col[e]];
    u[i] = acc;
  }
  for (int64_t i = n - 1; i >= 0; --i) {
    double acc = u[i];
    for (int64_t e = s->diag_pos[i] + 1; e < s->row_ptr[i + 1]; ++e) acc -= s->lu[e] * u[s->col[e]];
    u[i] = acc / s->lu[s->diag_pos[i]];
  }
}

static void spmv_fp(const orc_system *s, const double *x, double *y) {
  for (int64_t i = 0; i < s->n; ++i) {
    double acc = 0.0;
    for (int64_t e = s->row_ptr[i]; e < s->row_ptr[i + 1]; ++e) acc += s->a[e] * x[s->col[e]];
    y[i] = acc;
  }
}

static double dot(int64_t n, const double *a, const double *b) {
  double acc = 0.0;
  for (int64_t i = 0; i < n; ++i) acc += a[i] * b[i];
  return acc;
}

int orc_gmres64(const orc_system *s, int32_t m, double tol, int32_t max_restart, double *x, int32_t *iterations) {
  int64_t n = s->n;
  double *V = (double *)malloc(sizeof(double) * (size_t)n * (m + 1));
  double *H = (double *)calloc((size_t)(m + 1) * m, sizeof(double));
  double *cs = (double *)malloc(sizeof(double) * m), *sn = (double *)malloc(sizeof(double) * m);
  double *g = (double *)malloc(sizeof(double) * (m + 1)), *y = (double *)malloc(sizeof(double) * m);
  double *r = (double *)malloc(sizeof(double) * n), *rh = (double *)malloc(sizeof(double) * n);
  double *t = (double *)malloc(sizeof(double) * n);
  int status = ORC_NOT_CONVERGED;
  *iterations = 0;
  for (int32_t it = 0; it <= max_restart; ++it) {
    orc_residual(s, x, r, rh);
    double rel = orc_dnrm(n, rh) / s->bhat_norm;
    if (rel < tol) { status = ORC_OK; break; }
    if (it == max_restart) break;
    apply_m(s, r, V);
    double beta = sqrt(dot(n, V, V));
    if (beta == 0.0) { status = ORC_OK; break; }
    for (int64_t l = 0; l < n; ++l) V[l] /= beta;
    memset(g, 0, sizeof(double) * (m + 1));
    g[0] = beta;
    int32_t js = m;
    for (int32_t j = 0; j < m; ++j) {
      double *w = V + (size_t)(j + 1) * n;
      spmv_fp(s, V + (size_t)j * n, t);
      apply_m(s, t, w);
      for (int32_t i = 0; i <= j; ++i) {
        double h = dot(n, w, V + (size_t)i * n);
        H[i * m + j] = h;
        for (int64_t l = 0; l < n; ++l) w[l] -= h * V[(size_t)i * n + l];
      }
      double hn = sqrt(dot(n, w, w));
      H[(j + 1) * m + j] = hn;
      if (hn != 0.0)
        for (int64_t l = 0; l < n; ++l) w[l] /= hn;
      for (int32_t i = 0; i < j; ++i) {
        double a = H[i * m + j], b = H[(i + 1) * m + j];
        H[i * m + j] = cs[i] * a + sn[i] * b;
        H[(i + 1) * m + j] = -sn[i] * a + cs[i] * b;
      }
      double a = H[j * m + j], b = H[(j + 1) * m + j];
      double tt = sqrt(a * a + b * b);
      cs[j] = a / tt;
      sn[j] = b / tt;
      H[j * m + j] = tt;
      H[(j + 1) * m + j] = 0.0;
      g[j + 1] = -sn[j] * g[j];
      g[j] = cs[j] * g[j];
      *iterations += 1;
      if (hn == 0.0) { js = j + 1; break; }
    }
    for (int32_t i = js - 1; i >= 0; --i) {
      double acc = g[i];
      for (int32_t k = i + 1; k < js; ++k) acc -= H[i * m + k] * y[k];
      y[i] = acc / H[i * m + i];
    }
    for (int32_t i = 0; i < js; ++i)
      for (int64_t l = 0; l < n; ++l) x[l] += y[i] * V[(size_t)i * n + l];
  }
  free(V); free(H); free(cs); free(sn); free(g); free(y); free(r); free(rh); free(t);
  return status;
}
