/* Sanitizer run of the oracle (test infrastructure): whole solves on small
 * seeded systems with every preset, an overflow with and without shift
 * retries, and the setup error paths. Exit status 0 when every status is the
 * expected one; the sanitizers abort on any memory error or undefined
 * behaviour. */
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "../../oracle/orc.h"

typedef struct {
  int64_t n, nnz;
  int64_t *rp;
  int32_t *col;
  double *val, *b;
} csr;

/* 5-point Laplacian on a k x k grid, b = A * ones */
static csr poisson(int k) {
  csr a;
  a.n = (int64_t)k * k;
  a.rp = malloc(sizeof(int64_t) * (a.n + 1));
  a.col = malloc(sizeof(int32_t) * 5 * a.n);
  a.val = malloc(sizeof(double) * 5 * a.n);
  a.b = malloc(sizeof(double) * a.n);
  int64_t e = 0;
  for (int i = 0; i < k; ++i)
    for (int j = 0; j < k; ++j) {
      int64_t r = (int64_t)i * k + j;
      a.rp[r] = e;
      double s = 0.0;
      const int64_t nb[5] = {r - k, r - 1, r, r + 1, r + k};
      const int ok[5] = {i > 0, j > 0, 1, j < k - 1, i < k - 1};
      for (int t = 0; t < 5; ++t)
        if (ok[t]) {
          a.col[e] = (int32_t)nb[t];
          a.val[e] = nb[t] == r ? 4.0 : -1.0;
          s += a.val[e];
          ++e;
        }
      a.b[r] = s;
    }
  a.rp[a.n] = e;
  a.nnz = e;
  return a;
}

static void free_csr(csr *a) { free(a->rp); free(a->col); free(a->val); free(a->b); }

static orc_policy preset(int which) {
  orc_policy p;
  memset(&p, 0, sizeof(p));
  p.df = 30; p.m = 30; p.max_refine = 2000; p.gtol = -1; p.tol = 1e-10;
  if (which == 0) { /* Table IV */
    p.alpha_a = 16; p.precond = ORC_PRE_NONE;
    p.b_dot = p.b_axpy = p.b_norm = p.b_rot = p.b_tmp = 16;
    p.b_div_num = p.b_cs_num = 16; p.b_div_den = p.b_cs_den = 14;
  } else { /* Table VI (ILU) or its diagonal-only variant */
    p.alpha_a = 32; p.precond = which == 1 ? ORC_PRE_ILU0 : ORC_PRE_JACOBI;
    p.b_div_num = p.b_cs_num = 30;
  }
  return p;
}

static int solve(const csr *a, orc_policy p, int expect, int32_t *retries) {
  orc_system *s = NULL;
  int rc = orc_create(a->n, a->rp, a->col, a->val, a->b, &p, &s);
  if (rc != ORC_OK) return rc == expect ? 0 : 1;
  double *x = calloc((size_t)a->n, sizeof(double));
  orc_stats st;
  memset(&st, 0, sizeof(st));
  rc = orc_solve(s, x, &st);
  if (retries) *retries = st.shift_retries;
  free(x);
  orc_destroy(s);
  if (rc != expect) fprintf(stderr, "status %d, expected %d\n", rc, expect);
  return rc == expect ? 0 : 1;
}

int main(void) {
  int bad = 0;
  csr a = poisson(12);
  for (int w = 0; w < 3; ++w) bad += solve(&a, preset(w), ORC_OK, NULL);
  orc_policy z = preset(0);
  z.b_dot = z.b_axpy = z.b_norm = z.b_rot = z.b_tmp = 0; /* overflows in the inner product */
  bad += solve(&a, z, ORC_ERR_OVERFLOW, NULL);
  int32_t r = 0;
  z.shift_retry = 40;
  bad += solve(&a, z, ORC_OK, &r);
  bad += r > 0 ? 0 : 1;
  /* an all-zero row and a NaN entry */
  for (int64_t e = a.rp[5]; e < a.rp[6]; ++e) a.val[e] = 0.0;
  bad += solve(&a, preset(0), ORC_ERR_SINGULAR_ROW, NULL);
  a.val[a.rp[5]] = 0.0 / 0.0;
  bad += solve(&a, preset(1), ORC_ERR_ARG, NULL);
  free_csr(&a);
  printf("oracle sanitizer run: %d failures\n", bad);
  return bad ? 1 : 0;
}
