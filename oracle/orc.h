/*
 * CPU oracle for the integer-arithmetic GMRES(m) solver with FP64 iterative
 * refinement of Iwashita, Suzuki and Fukaya, "An Integer Arithmetic-Based
 * Sparse Linear Solver Using a GMRES Method and Iterative Refinement"
 * (ScalA'20, arXiv 2009.07495).
 *
 * TEST INFRASTRUCTURE ONLY. This plain, slow, single-threaded C11 code is the
 * yardstick the GPU library is checked against. Only the test suite, the
 * smoke check and the benchmark's CPU-baseline leg may load it; the GPU
 * library never calls it and shares no code, header or table with it.
 *
 * Conventions (all integer words are int64, two's complement, "intWL" with
 * WL = 64, Sec. II):
 *   asr(x, b)  = floor(x / 2^b)             arithmetic right shift (Sec. V-A)
 *   shl(x, b)  = x * 2^b                     left shift, range-checked
 *   sc(x, e)   = shl(x, e) if e >= 0 else asr(x, -e)
 *   tdiv(a, d) = a / d truncated toward 0   C integer division (Sec. V-B.3)
 *   isqrt(x)   = floor(sqrt(x)), integer Babylonian iteration (Sec. V-B.4)
 *   trunc(y)   = C cast double -> int64, toward 0
 * Every integer operation is evaluated exactly in __int128; a result that does
 * not fit in int64 is an overflow event and the stored word is the exact
 * result reduced mod 2^64 (what 64-bit hardware produces). Sums of products
 * are exact sums of the (wrapped) int64 products, so they do not depend on the
 * summation order. Overflow events are reported as the smallest event code
 * (see ORC_CODE) seen during a cycle.
 *
 * Floating point is IEEE binary64 with no contraction (-ffp-contract=off);
 * every FP64 sum is taken in a fixed order stated at its definition, and the
 * 2-norm is the order-free "dnrm" defined in orc_ir.c, so the whole run is
 * reproducible bit for bit.
 *
 * Parity status: the primitives, setup, FP64 steps and whole solves are pinned
 * by tests against definitions, closed forms, textbook special cases, dense
 * solves and the invariants the paper states. The exact bits of the integer
 * cycle (the cast of v1 and the integer loop of Fig. 2) have no worked example in the
 * paper; they are pinned only through those properties.
 */
#ifndef ORC_H
#define ORC_H

#include <stdint.h>

enum {
  ORC_OK = 0,
  ORC_NOT_CONVERGED = 1,
  ORC_ERR_ARG = -1,
  ORC_ERR_SINGULAR_ROW = -2,
  ORC_ERR_ZERO_PIVOT = -3,
  ORC_ERR_OVERFLOW = -4,
  ORC_ERR_RANGE = -5,
  ORC_ERR_BREAKDOWN = -8,
};

enum { ORC_PRE_NONE = 0, ORC_PRE_JACOBI = 1, ORC_PRE_ILU0 = 2 };

/* Solver parameters: the arguments of Table I plus the operand shifts of
 * Table II (one beta per shifted operand). */
typedef struct {
  int32_t df;          /* fraction bits d_f of the Q d_m.d_f words */
  int32_t alpha_a;     /* initial scaling exponent, eq. (eq3) */
  int32_t s_terms;     /* s: number of correction matrices A_1..A_s used, eq. (AA) */
  int32_t m;           /* iterations per int-GMRES call (= per refinement) */
  int32_t precond;     /* ORC_PRE_* */
  int32_t b_dot;       /* Gram-Schmidt inner product: beta_1 on w */
  int32_t b_axpy;      /* Gram-Schmidt update: beta_1 on h */
  int32_t b_norm;      /* norm of w: beta_1 = beta_2 */
  int32_t b_div_num;   /* normalisation: numerator * 2^beta_1 */
  int32_t b_div_den;   /* normalisation: denominator / 2^beta_2 */
  int32_t b_rot;       /* earlier rotations on column j: beta_2 on the h entries */
  int32_t b_tmp;       /* rotation radius t_mp: beta_1 = beta_2 */
  int32_t b_cs_num;    /* new rotation c_j, s_j: numerator * 2^beta_1 */
  int32_t b_cs_den;    /* new rotation c_j, s_j: denominator / 2^beta_2 */
  int32_t max_refine;  /* refinement limit (not given in the paper) */
  int32_t shift_retry; /* overflow-driven shift retries allowed per solve, 0 = none (see orc_shift_retry) */
  int64_t gtol;        /* stop a cycle early when |g_{j+1}| <= gtol; < 0: never */
  double tol;          /* FP64 relative residual target on the original system */
  int32_t two_sided;   /* 0: eq. (eq1); 1: eq. (eq2) with D1 = D2 = Dhat^(1/2) (see orc_setup.c) */
  int32_t gauss_seidel; /* with ORC_PRE_ILU0: the Gauss-Seidel splitting instead of ILU(0) (orc_setup.c) */
  int32_t s_rule;      /* s(k) of eq. (AA), S = s_terms: 0 s(k) = S; 1 s(k) = min(S, k - 1) (orc_s_of_k) */
} orc_policy;

/* Overflow event code: (step j, stage, sub-index), ordered as executed.
 * Stages, as the steps of Fig. 2 and Sec. VI: 1 SpMV, 2 preconditioner apply,
 * 3 Gram-Schmidt (sub = 2(i-1) + {0 inner product, 1 update}), 4 norm of w,
 * 5 normalisation, 6 earlier rotations (sub = i), 7 rotation radius, 8 new
 * rotation, 9 rotation of g. */
#define ORC_CODE(j, stage, sub) (((int64_t)(j) << 24) | ((int64_t)(stage) << 16) | (int64_t)(sub))
#define ORC_NO_EVENT INT64_MAX

/* ---- fixed-point primitives (orc_fx.c) ---------------------------------- */
int64_t orc_asr(int64_t x, int32_t b);
int64_t orc_shl(int64_t x, int32_t b, int32_t *ovf);
int64_t orc_sc(int64_t x, int32_t e, int32_t *ovf);
int64_t orc_tdiv(int64_t a, int64_t d, int32_t *ovf);
int64_t orc_isqrt(int64_t x);
int64_t orc_trunc(double y, int32_t *range_err);
int64_t orc_mul(int64_t t1, int64_t t2, int32_t b1, int32_t b2, int32_t df, int32_t *ovf);
int64_t orc_div(int64_t t1, int64_t t2, int32_t b1, int32_t b2, int32_t df, int32_t *ovf, int32_t *zero);
int64_t orc_dot(int64_t n, const int64_t *w, const int64_t *v, int32_t b, int32_t df, int32_t *ovf);
int64_t orc_norm(int64_t n, const int64_t *w, int32_t b, int32_t df, int32_t *ovf);
void orc_axpy(int64_t n, int64_t *w, const int64_t *v, int64_t h, int32_t b, int32_t df, int32_t *ovf);
void orc_normalize(int64_t n, const int64_t *w, int64_t den, int32_t b1, int32_t b2, int32_t df, int64_t *v,
                   int32_t *ovf);

/* ---- FP64 helpers (orc_ir.c) --------------------------------------------- */
double orc_dnrm(int64_t n, const double *x);
double orc_u128_to_double(uint64_t lo, uint64_t hi);

/* ---- system setup (orc_setup.c) ------------------------------------------ */
typedef struct orc_system orc_system;

int orc_create(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
               const double *b, const orc_policy *pol, orc_system **out);
void orc_destroy(orc_system *s);
int64_t orc_n(const orc_system *s);
int64_t orc_nnz(const orc_system *s);
int32_t orc_nterms(const orc_system *s);
/* Scaled system: dhat[n], a[nnz], b[n] (any may be NULL). */
void orc_get_scaled(const orc_system *s, double *dhat, double *a, double *b);
/* Integer matrices on the input pattern: abar[(l)*nnz + e] for l = 0..nterms-1,
 * alpha[l] (alpha[0] = 0). */
void orc_get_terms(const orc_system *s, int64_t *abar, int32_t *alpha);
/* Integer preconditioner: fac[nnz] holds Lbar (col < row) / Ubar (col > row)
 * on the input pattern (0 elsewhere and for Jacobi); ldiag[n], udiag[n]. */
void orc_get_precond(const orc_system *s, int64_t *fac, int64_t *ldiag, int64_t *udiag);
/* FP64 ILU(0) factors before the cast: lu[nnz] (multipliers below the
 * diagonal, U above and on it). Returns 0 if no ILU was built. */
int orc_get_ilu_fp(const orc_system *s, double *lu);

/* ---- integer kernels (orc_cycle.c) --------------------------------------- */
void orc_spmv(const orc_system *s, int32_t nterms, const int64_t *v, int64_t *z, int32_t j, int64_t *first);
void orc_precond_apply(const orc_system *s, const int64_t *z, int64_t *w, int32_t j, int64_t *first);

typedef struct {
  int32_t m;          /* in: columns allocated */
  int32_t jstar;      /* out: columns usable for the closing least-squares step */
  int32_t breakdown;  /* out: 0 none, 1 normalisation denominator 0, 2 new-rotation denominator 0 */
  int32_t steps;      /* out: Arnoldi steps executed */
  int64_t first_ovf;  /* out: smallest overflow event code, ORC_NO_EVENT if none */
  int64_t *H;         /* (m+1) x m, row-major: H[i*m + j], 0-based */
  int64_t *c, *s;     /* m */
  int64_t *g;         /* m+1 */
  int64_t *V;         /* n x (m+1), column j at V + j*n */
} orc_trace;

/* s(k) of eq. (AA) for refinement k = 1, 2, ...: the correction matrices
 * A_1..A_s(k) the k-th int-GMRES call uses. */
int32_t orc_s_of_k(const orc_policy *p, int32_t k);
/* The integer loop of Fig. 2 of refinement k starting from the integer v1
 * (v1 cast to Q df); its matrix is Abar^(k) of eq. (AA). */
int orc_cycle(const orc_system *s, const int64_t *v1, int32_t k, orc_trace *t);
/* Closing FP64 step of Fig. 2: x[n] = sum_i y_i v_i with y = rho * H^-1 g (FP64). */
void orc_cycle_update(const orc_system *s, const orc_trace *t, double rho, double *x);

/* ---- refinement driver (orc_ir.c) ---------------------------------------- */
typedef struct {
  int32_t status;
  int32_t refinements;   /* int-GMRES calls made */
  int32_t iterations;    /* sum of Arnoldi steps */
  int32_t hist_cap;      /* in: capacity of the hist_* arrays (may be 0) */
  int64_t first_ovf;
  double relres_orig, relres_scaled;
  double *hist_relres_orig;   /* [hist_cap] value at the top of refinement k */
  double *hist_relres_scaled;
  double *hist_gamma;
  double *hist_rho;
  int32_t *hist_jstar;
  int32_t shift_retries; /* int-GMRES calls repeated with adjusted shifts */
  int32_t pad_;
} orc_stats;

/* Runs Fig. 1 from x. With pol.shift_retry > 0 an int-GMRES call that
 * overflows is repeated with the shifts orc_shift_retry chooses, and the
 * adjusted shifts stay in the system's policy. */
int orc_solve(orc_system *s, double *x, orc_stats *st);
/* Overflow-driven shift retry. The paper reports that an auto-tuning of the
 * operand shift was investigated for the solver without preconditioner
 * (Sec. VII-D) but gives no rule; this is the reading used here. From the
 * stage of the first overflow event of a call (ORC_CODE): the right shift
 * applied before a product grows by 4, capped at df (inner product: b_dot,
 * update: b_axpy, norm: b_norm, earlier rotations: b_rot, rotation radius:
 * b_tmp); for a division (normalisation, new rotation) the numerator's
 * exponent shrinks by 4 (not below 0), or the denominator's once the
 * numerator's is 0. Returns 1 if a shift changed, 0 if none can (SpMV,
 * preconditioner apply, rotation of g, or shifts at their limits). */
int orc_shift_retry(orc_policy *p, int64_t code);
/* The system's current policy (shifts adjusted by retries included). */
void orc_get_policy(const orc_system *s, orc_policy *out);
/* Pieces of one refinement, for step-level parity checks. */
void orc_residual(const orc_system *s, const double *x, double *r, double *rhat);
int orc_start_vector(const orc_system *s, const double *r, double *bk, double *r0, int64_t *v1,
                     double *gamma, double *rho);

/* ---- FP64 GMRES(m) comparator (orc_gmres64.c) ---------------------------- */
int orc_gmres64(const orc_system *s, int32_t m, double tol, int32_t max_restart, double *x,
                int32_t *iterations);

#endif
