/*
 * igmres.h -- C ABI of the MI355X (gfx950) integer-arithmetic GMRES(m) solver
 * with FP64 iterative refinement.
 *
 * Method: T. Iwashita, K. Suzuki, T. Fukaya, "An Integer Arithmetic-Based
 * Sparse Linear Solver Using a GMRES Method and Iterative Refinement",
 * ScalA'20 (arXiv 2009.07495).
 *
 * The caller hands in an FP64 system Ahat xhat = bhat in CSR form (Sec. III,
 * eq. (org)). The library scales it (eqs. (eq1), (eq3)), casts the matrix to
 * integers (Sec. IV-B), builds the optional integer preconditioner (Sec. VI),
 * and refines xhat in FP64 (Sec. IV, Fig. 1) until the FP64 relative residual
 * of the original system drops below the tolerance. Each refinement runs one
 * int-GMRES(m) call (Fig. 2) whose main loop is integer-only and runs on the
 * GPU as hand-written HIP kernels.
 *
 * Conventions for every call:
 *  - Plain C types only. No exceptions cross the boundary; every call returns
 *    an igm_status (negative = error, positive = warning) and never aborts.
 *  - Host pointers are read during the call only; the caller keeps ownership.
 *    "Device pointers" are HIP device allocations on the system's device
 *    (e.g. torch CUDA tensors), also owned by the caller.
 *  - All device work of a system is ordered on the system's HIP stream (the
 *    null stream unless igm_set_stream was called). Calls that return host
 *    results synchronise that stream before returning.
 *  - One system is not thread-safe; distinct systems may be used from
 *    distinct threads.
 *  - Integer words are int64 two's complement fixed-point numbers in
 *    Q(63 - df).df format (Sec. II, WL = 64).
 */
#ifndef IGMRES_H
#define IGMRES_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct igm_system igm_system;

typedef enum {
  IGM_OK = 0,
  IGM_NOT_CONVERGED = 1,      /* warning: refinement limit reached; x holds the last iterate */
  IGM_PENDING = 2,            /* served request not finished yet (igm_server_wait timed out) */
  IGM_ERR_ARG = -1,           /* invalid argument, CSR or policy */
  IGM_ERR_SINGULAR_ROW = -2,  /* a row of Ahat is all zero: eq. (eq3) undefined */
  IGM_ERR_ZERO_PIVOT = -3,    /* zero ILU(0) pivot, missing diagonal, or a cast diagonal of 0 */
  IGM_ERR_OVERFLOW = -4,      /* an integer word left int64 in a cycle (stats name where) */
  IGM_ERR_RANGE = -5,         /* an FP64 -> int64 cast out of range, or a non-finite residual */
  IGM_ERR_OOM = -6,           /* device or host allocation failed */
  IGM_ERR_DEVICE = -7,        /* HIP error, or a device-side wait that timed out */
  IGM_ERR_BREAKDOWN = -8,     /* a cycle produced no usable Krylov column */
  IGM_ERR_UNSUPPORTED = -9    /* a size or option the library does not support */
} igm_status;

enum { IGM_PRE_NONE = 0, IGM_PRE_JACOBI = 1, IGM_PRE_ILU0 = 2 };

/* Presets: the paper's two settings (Sec. VII-B / Table IV, Sec. VII-C /
 * Table VI) and a diagonal-only variant of the ILU construction. */
enum { IGM_PRESET_PAPER_NOPREC = 0, IGM_PRESET_PAPER_ILU = 1, IGM_PRESET_JACOBI = 2 };

/* Row-to-lane mappings of the integer SpMV (igm_policy.spmv_lanes); 4, 16 and
 * 64 (lanes per row) are mappings too. */
enum { IGM_SPMV_MEASURE = -1, IGM_SPMV_AUTO = 0, IGM_SPMV_SELL = 1, IGM_SPMV_MERGE = 2 };

/* Overflow event code (igm_stats.first_ovf, igm_cycle_trace.first_ovf):
 *   (step j << 24) | (stage << 16) | sub
 * stages follow the steps of Fig. 2 and Sec. VI: 1 = integer SpMV w = A v_j,
 * 2 = preconditioner apply M^-1 w, 3 = modified Gram-Schmidt (sub = 2(i-1)
 * for the inner product with v_i, 2(i-1)+1 for the update of w), 4 = norm
 * h_{j+1,j} = ||w||, 5 = normalisation v_{j+1} = w / h_{j+1,j}, 6 = earlier
 * Givens rotations applied to column j (sub = i), 7 = rotation radius
 * t_mp = sqrt(h_jj^2 + h_{j+1,j}^2), 8 = new rotation c_j, s_j, 9 = rotation
 * of g. The smallest code of a cycle is reported. IGM_NO_EVENT if none. */
#define IGM_NO_EVENT INT64_MAX

/* Solver parameters (Table I arguments, Table II operand shifts). */
typedef struct {
  int32_t struct_size;  /* sizeof(igm_policy) */
  int32_t df;           /* fraction bits d_f, 1..62 (paper: 30) */
  int32_t alpha_a;      /* eq. (eq3) exponent, 0..62 (paper: 16 / 32) */
  int32_t s_terms;      /* s of eq. (AA): correction matrices used, 0..8 (paper: 0) */
  int32_t m;            /* int-GMRES iterations per refinement, 1..1024 */
  int32_t precond;      /* IGM_PRE_* (Sec. VI) */
  int32_t b_dot;        /* Gram-Schmidt inner product: shift of w */
  int32_t b_axpy;       /* Gram-Schmidt update: shift of h */
  int32_t b_norm;       /* norm of w: shift of both operands */
  int32_t b_div_num;    /* normalisation: numerator * 2^b */
  int32_t b_div_den;    /* normalisation: denominator / 2^b */
  int32_t b_rot;        /* earlier rotations on column j: shift of the h entries */
  int32_t b_tmp;        /* rotation radius: shift of both operands */
  int32_t b_cs_num;     /* new rotation c_j, s_j: numerator * 2^b */
  int32_t b_cs_den;     /* new rotation c_j, s_j: denominator / 2^b */
  int32_t max_refine;   /* refinement limit (the paper gives none) */
  int64_t gtol;         /* end a cycle early when |g_{j+1}| <= gtol (Sec. V-A); < 0 = never */
  double tol;           /* stop when ||bhat - Ahat x|| / ||bhat|| < tol (Sec. III) */
  int32_t grid_blocks;  /* launch tuning: workgroups of the cycle kernel; 0 = automatic */
  int32_t phase_clock;  /* 1 = record where int-GMRES calls spend their time (igm_stats.phase_us); costs a few % */
  /* Overflow-driven shift retries allowed per solve, 0..64 (0 = none, the
   * paper's setting; every solver). The paper reports that an
   * auto-tuning of the operand shift was tried for the solver without
   * preconditioner (Sec. VII-D) but gives no rule; the rule here: when an
   * int-GMRES call overflows, the stage of its first event (see the event
   * code) picks one shift: the Gram-Schmidt inner product and update, the
   * norm, the earlier rotations and the rotation radius raise b_dot, b_axpy,
   * b_norm, b_rot, b_tmp by 4 (at most df); the normalisation and the new
   * rotation lower b_div_num (or b_cs_num) by 4 (not below 0), or the
   * denominator's exponent once the numerator's is 0. The call is then
   * repeated from the same v1. Overflow in the SpMV, the preconditioner apply
   * or the rotation of g, or with the shift at its limit, ends the solve with
   * IGM_ERR_OVERFLOW as without retries. Adjusted shifts stay in the system's
   * policy (igm_get_policy) for later solves; in the batched and served
   * solvers they last for the rest of that system's solve (each solve starts
   * from the policy's shifts). */
  int32_t shift_retry;
  /* 0: scaling of eq. (eq1) (rows by Dhat, the paper's setting); 1: eq. (eq2)
   * with D1 = D2 = Dhat^(1/2) (the paper leaves D1, D2 open; this choice keeps
   * a symmetric matrix symmetric): A = D1^-1 Ahat D2^-1, b = D1^-1 bhat,
   * computed as a_ij = ahat_ij / (s_i s_j), s = sqrt(dhat); the scaled
   * residual of Fig. 1 is D1^-1 (bhat - Ahat xhat) and each correction
   * returns through D2^-1. Every solver supports it. */
  int32_t two_sided;
  /* With precond = IGM_PRE_ILU0 only: 1 = build the factors from the
   * Gauss-Seidel splitting M = D + L_A instead of ILU(0) (the paper reports a
   * Gauss-Seidel preconditioner, Sec. VII-D, without its construction; here M
   * is written as L D U with L = I + L_A D^-1 and U = I and split as in
   * Sec. VI, so Lbar carries (a_ij / a_jj)|a_jj|^(1/2) below the diagonal and
   * Ubar is diagonal). Every solver supports it. */
  int32_t gauss_seidel;
  /* Launch tuning of the ILU(0) sweeps of the single-system solver (the bits
   * do not depend on either): rows per block of the blocked sweeps, a multiple
   * of 64 (0 = automatic: as many as the workgroup's LDS holds, at most
   * 16384), and lanes per row of the integer sweeps: 0, 4, 8 or 16 are
   * accepted, and the sweeps run 4 lanes per row whatever the value (building
   * the 8- and 16-lane sweeps into the cycle kernel as well made it spill). */
  int32_t sweep_rows;
  int32_t sweep_lanes;
  /* s(k) of eq. (AA), the correction matrices used by the int-GMRES call of
   * refinement k = 1, 2, ... (the paper makes s(k) a solver parameter bounded
   * by S, Fig. 1, without a rule): 0 = s(k) = S = s_terms in every refinement
   * (the paper's experiments, S = 0); 1 = s(k) = min(S, k - 1), Abar_0 alone in
   * the first refinement and one more term in each later one. */
  int32_t s_rule;
  /* Launch tuning of the single-system solver's integer SpMV and FP64
   * residual (the bits do not depend on it), IGM_SPMV_* or lanes per row:
   * IGM_SPMV_SELL (1) = one thread per row over the SELL-64 layout (rows of
   * similar length); 4, 8, 16, 32 or 64 = that many lanes of a wavefront per
   * row over the CSR layout (64 = a wavefront per row); IGM_SPMV_MERGE (2) = each
   * workgroup's chunk of rows split evenly by entries over its threads, rows
   * cut anywhere (heavy-tailed row lengths; chunks of 1024 rows must hold
   * fewer than 2^30 entries); IGM_SPMV_AUTO (0) = from the row lengths: SELL
   * unless SELL-64 would more than double the entries loaded, then MERGE;
   * IGM_SPMV_MEASURE (-1) = at setup each mapping (SELL, MERGE, 4 to 64
   * lanes) runs the standalone SpMV a few times and the fastest is kept. The FP64 residual runs one thread per
   * row with SELL, 16 lanes per row with MERGE, else the SpMV's lanes. Every
   * mapping but SELL also keeps the integer matrices in CSR order (8 bytes per
   * entry and term). */
  int32_t spmv_lanes;
  int32_t reserved_[3];
} igm_policy;

/* Fill *out with a preset (IGM_PRESET_*): df = 30, s = 0, m = 30, tol = 1e-10,
 * max_refine = 2000, gtol = -1. IGM_ERR_ARG for an unknown preset. */
igm_status igm_policy_preset(int32_t preset, igm_policy *out);

/* Build a system from an FP64 CSR matrix (row_ptr[n+1] int64, col[nnz] int32
 * with strictly increasing columns per row, val[nnz]) and right-hand side
 * b[n], all host memory, copied during the call. Performs the row scaling of
 * eq. (eq3)/(eq1), the integer matrices of eq. (A), the integer ILU(0) or
 * Jacobi factors of eqs. (dl)-(ilu2), and uploads everything to the current
 * HIP device. Errors: IGM_ERR_ARG (bad CSR, non-finite value, bad policy),
 * IGM_ERR_SINGULAR_ROW, IGM_ERR_ZERO_PIVOT, IGM_ERR_RANGE, IGM_ERR_OOM,
 * IGM_ERR_DEVICE. On error *out is NULL. */
igm_status igm_create_system(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
                             const double *b, const igm_policy *pol, igm_system **out);

/* Replace the policy; redoes the policy-dependent setup (scaling, integer
 * matrices, preconditioner). Same errors as igm_create_system; on error the
 * system keeps its previous policy. */
igm_status igm_set_policy(igm_system *s, const igm_policy *pol);

/* Replace the right-hand side bhat (host, n doubles). */
igm_status igm_set_rhs(igm_system *s, const double *b);

/* Use a caller-created HIP stream (hipStream_t passed as void*, e.g. the
 * handle of a torch stream) for all later device work; NULL = null stream. */
igm_status igm_set_stream(igm_system *s, void *hip_stream);

/* Solve (Fig. 1): x[n] (host) holds the starting iterate on entry (zeros =
 * the paper's setting) and the final iterate on return. IGM_OK,
 * IGM_NOT_CONVERGED, or an error; on IGM_ERR_OVERFLOW / IGM_ERR_BREAKDOWN x
 * holds the last iterate before the failed refinement. */
igm_status igm_solve(igm_system *s, double *x);

/* Same as igm_solve with x a device pointer to n doubles on the system's
 * device; no host copies of x are made. */
igm_status igm_solve_device(igm_system *s, double *x_dev);

typedef struct {
  int32_t struct_size;     /* sizeof(igm_stats) */
  int32_t status;          /* status of the last solve */
  int32_t refinements;     /* int-GMRES calls of the last solve */
  int32_t iterations;      /* Arnoldi steps of the last solve */
  int64_t first_ovf;       /* overflow event code of the failed cycle, IGM_NO_EVENT if none */
  double relres_orig;      /* final ||bhat - Ahat x|| / ||bhat|| */
  double relres_scaled;    /* final ||b - A x|| / ||b|| (scaled system, Fig. 1) */
  double time_solve_ms;    /* wall time of the last solve */
  double time_cycle_ms;    /* GPU time in the int-GMRES kernels of the last solve */
  double time_setup_ms;    /* host + upload time of the last setup */
  int64_t n, nnz;
  int32_t nterms;          /* integer matrices built (A_0 .. A_p) */
  int32_t grid_blocks;     /* workgroups of the cycle kernel */
  int32_t rows_per_thread; /* rows held in registers by each thread */
  int32_t block_threads;   /* threads per workgroup */
  int32_t levels_fwd;      /* ILU forward level sets */
  int32_t levels_bwd;      /* ILU backward level sets */
  int64_t device_bytes;    /* device memory held by the system */
  int32_t last_error_line; /* source line of the last HIP error, 0 if none */
  int32_t shift_retries;   /* int-GMRES calls of the last solve repeated with adjusted shifts */
  double time_kernel_ms;   /* GPU time of the kernels of the last kernel-level call (igm_spmv ...) */
  /* Where the last int-GMRES call spent its time, seen by workgroup 0 (us;
   * recorded only with igm_policy.phase_clock = 1, zeros otherwise):
   * 0 SpMV + preconditioner, 1 inner products and updates (local work),
   * 2 waits for the grid-wide inner-product sums, 3 norm, 4 normalisation,
   * 5 Givens rotations, 6 end-of-step barriers, 7 the whole call. */
  double phase_us[8];
  int32_t spmv_lanes;      /* lanes per row of the integer SpMV and FP64 residual (1 = SELL-64) */
  int32_t sweep_rows;      /* ILU(0): rows per block of the blocked sweeps */
  int32_t reserved_[2];
} igm_stats;

/* Copy the statistics of the system's last setup and solve. */
igm_status igm_get_stats(const igm_system *s, igm_stats *out);

/* Copy the system's current policy: the one it was built with, with the
 * shifts that overflow retries adjusted (igm_policy.shift_retry). */
igm_status igm_get_policy(const igm_system *s, igm_policy *out);

/* Per-refinement history of the last solve: entry k (0-based) holds the
 * values at the top of refinement k+1: relres of the original and scaled
 * system, gamma^(k) (eq. (gammak)), rho = ||r0|| (the FP64 start step of Fig. 2 and Sec. VI), and the number of
 * columns used (j*). Any pointer may be NULL. Returns the number of entries
 * written (<= cap) in *count. */
igm_status igm_get_history(const igm_system *s, int32_t cap, double *relres_orig, double *relres_scaled,
                           double *gamma, double *rho, int32_t *jstar, int32_t *count);

/* One int-GMRES(m) call, the integer loop of Fig. 2 (Arnoldi steps with
 * Givens rotations), from the integer start vector v1 (host, n int64 words:
 * v1 cast to Q.df as in Fig. 2), with the system's policy, as the call of
 * refinement k >= 1 (its matrix is Abar^(k) of eq. (AA); k < 1 is IGM_ERR_ARG).
 * Outputs (caller-allocated host arrays; V may be NULL):
 *   H[(m+1)*m] row-major (H[i*m + j], 0-based) after the rotations,
 *   c[m], s[m], g[m+1], V[(m+1)*n] (basis vector j at V + j*n).
 * m is taken from trace->m, which must equal the policy's m. */
typedef struct {
  int32_t m;          /* in */
  int32_t jstar;      /* out: columns usable by the closing FP64 least-squares step */
  int32_t breakdown;  /* out: 0 none, 1 zero denominator in the normalisation, 2 in the new rotation */
  int32_t steps;      /* out: Arnoldi steps executed */
  int64_t first_ovf;  /* out: overflow event code or IGM_NO_EVENT */
  int64_t *H, *c, *s, *g, *V;
} igm_cycle_trace;

igm_status igm_int_cycle(igm_system *s, const int64_t *v1, int32_t k, igm_cycle_trace *trace);

/* Kernel-level entry points (each runs one GPU kernel family on device
 * buffers, for checking a single step of the method and for timing it).
 * All vectors are device pointers of length n unless stated otherwise;
 * *first_ovf receives the overflow event code with step j = 1. */

/* Integer SpMV w = A v (Fig. 2; Sec. V-C.3, eq. (matvec)): z = A_0 v + sum_{l=1..nterms-1}
 * asr(A_l v, alpha_l) over the system's integer matrices (nterms clamped to
 * the number built). */
igm_status igm_spmv(igm_system *s, int32_t nterms, const int64_t *v, int64_t *z, int64_t *first_ovf);

/* Preconditioner apply (Sec. VI, VI-A): w = Mbar^-1 z by integer forward/backward substitution
 * (truncating division), level-scheduled; w = z without a preconditioner. */
igm_status igm_precond(igm_system *s, const int64_t *z, int64_t *w, int64_t *first_ovf);

/* Gram-Schmidt inner product (Fig. 2; Sec. V-C.1, Table II): *h = asr(sum_l asr(w_l, b_dot) v_l, df - b_dot). */
igm_status igm_dot(igm_system *s, const int64_t *w, const int64_t *v, int64_t *h, int64_t *first_ovf);

/* Gram-Schmidt update (Fig. 2): w_l -= asr(asr(h, b_axpy) v_l, df - b_axpy), in place. */
igm_status igm_axpy(igm_system *s, int64_t h, int64_t *w, const int64_t *v, int64_t *first_ovf);

/* Norm of w (Fig. 2; Sec. V-C.2): *h = shl(isqrt(sum_l asr(w_l, b_norm)^2), b_norm). */
igm_status igm_norm(igm_system *s, const int64_t *w, int64_t *h, int64_t *first_ovf);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the inner
 * product of igm_dot (mode 0) or the norm of igm_norm (mode 1) over n words
 * of the caller's device vectors w (and v for mode 0), with shift b and d_f =
 * df given directly instead of by a system. Nothing is allocated and nothing
 * is waited for: the kernels are enqueued on `stream` (a hipStream_t; NULL =
 * null stream), and out_dev (device, 2 words) receives the result in
 * out_dev[0] and the overflow event code (step 1, stage 3 or 4) or
 * IGM_NO_EVENT in out_dev[1]. The kernels' scratch (256 per-workgroup partial
 * sums and a completion ticket, 4.3 KB) is a fixed array of the library on
 * each device, cleared by the call itself; it keeps the last call's contents.
 * Calls that overlap on one device (other streams, other threads) race on it
 * and must be serialised by the caller. Errors: IGM_ERR_ARG (mode, n outside
 * 1..2^48, null pointers, df outside 1..62, b outside 0..df), IGM_ERR_DEVICE,
 * IGM_ERR_UNSUPPORTED (device index above 63). */
igm_status igm_reduce_noalloc(int32_t mode, int64_t n, const int64_t *w, const int64_t *v, int32_t b, int32_t df,
                              int64_t *out_dev, void *stream);

/* Normalisation v = w / h (Fig. 2; Sec. V-B.3): v_l = sc(tdiv(shl(w_l, b_div_num), asr(h, b_div_den)),
 * df - b_div_num - b_div_den). IGM_ERR_BREAKDOWN if the shifted denominator is 0. */
igm_status igm_normalize(igm_system *s, const int64_t *w, int64_t h, int64_t *v, int64_t *first_ovf);

/* Refinement step (eq. (b)): r = b - A x (scaled system) and rhat = bhat -
 * Ahat x (original system), FP64, each row summed in CSR order. */
igm_status igm_residual(igm_system *s, const double *x, double *r, double *rhat);

/* The order-free FP64 2-norm used for every norm of the refinement loop
 * (mu = max|x_i|, exact integer sum of floor(2^96 (x_i/mu)^2), one rounding). */
igm_status igm_fp_norm(igm_system *s, const double *x, int64_t len, double *norm);

/* Start vector: eqs. (gammak), (scale), the FP64 start step of Sec. VI and the
 * cast of Fig. 2: gamma = max|r|, bk = r / gamma,
 * r0 = Mbar^-1 bk (FP64 substitution with the integer factors), rho =
 * ||r0||, v1 = trunc(2^df r0 / rho). IGM_ERR_RANGE if a cast is out of range.
 * *gamma = 0 means r = 0 (nothing written to v1). */
igm_status igm_start_vector(igm_system *s, const double *r, double *bk, double *r0, int64_t *v1, double *gamma,
                            double *rho);

/* Release all device and host memory of the system. NULL is a no-op. */
void igm_destroy(igm_system *s);

/* ---- Batched solver: many independent systems in one persistent launch ----
 * Fig. 1 and Fig. 2 applied to every system of a batch independently, with
 * one shared policy (any preconditioner; m <= 64). Each system is solved by a
 * team of 1..256 workgroups that claim it from a device-side queue, largest
 * systems first; all refinements of a system run inside the launch. The
 * results of a system are bit-identical to those of igm_solve_device on that
 * system alone. */
typedef struct igm_batch igm_batch;

/* Build a batch of nsys >= 1 systems from host arrays laid end to end:
 * n[nsys] rows per system; row_ptr holds nsys arrays of n_s + 1 entries (each
 * starting at 0 and ending at that system's nnz_s); col and val hold the nnz_s
 * entries of each system in turn; b holds the n_s entries of each right-hand
 * side in turn. Every system is set up and validated as igm_create_system
 * would (same errors); *failed (may be NULL) receives the index of the first
 * system that failed, -1 if none. IGM_ERR_UNSUPPORTED for m > 64 or a system
 * larger than 256 workgroups of every launch shape. On error *out is NULL. */
igm_status igm_batch_create(int32_t nsys, const int64_t *n, const int64_t *row_ptr, const int32_t *col,
                            const double *val, const double *b, const igm_policy *pol, int32_t *failed,
                            igm_batch **out);

/* Use a caller-created HIP stream for all later device work of the batch. */
igm_status igm_batch_set_stream(igm_batch *bt, void *hip_stream);

/* Launch shape: threads per workgroup and rows per thread, one of (1024, 8),
 * (1024, 4), (512, 8), (512, 16), (256, 8), (256, 16). System s gets
 * ceil(n_s / (block * rows_per_thread)) workgroups. IGM_ERR_UNSUPPORTED if a
 * system would need more than 256 or the device cannot hold that many at
 * once; IGM_ERR_ARG for a shape not in the list. */
igm_status igm_batch_set_shape(igm_batch *bt, int32_t block, int32_t rows_per_thread);

/* Record (1) or not (0) per-phase clocks of each system's solve, returned in
 * igm_batch_get_result's phase_us (0 SpMV + preconditioner, 1 inner products
 * and updates, 2 waits for their sums, 3 norm, 4 normalisation, 5 FP64
 * refinement steps, 6 end-of-step barriers, 7 whole solve). Costs a few %. */
igm_status igm_batch_set_phase_clock(igm_batch *bt, int32_t on);

/* Time one solve of the batch (from x = 0, in a buffer of the batch; the
 * caller's memory is not touched) with every usable shape and keep the
 * fastest. The chosen shape is stored in *block and *rows_per_thread (either
 * may be NULL). Results do not depend on the shape. */
igm_status igm_batch_autotune(igm_batch *bt, int32_t *block, int32_t *rows_per_thread);

/* Solve every system. x_dev: device pointer to sum(n_s) doubles laid end to
 * end in system order: starting iterates in (zeros = the paper's setting),
 * solutions out. Returns IGM_OK if every system returned IGM_OK,
 * IGM_ERR_DEVICE on a device failure, otherwise the status of the first
 * system (in system order) that did not return IGM_OK. */
igm_status igm_batch_solve_device(igm_batch *bt, double *x_dev);

/* Same with x a host array of sum(n_s) doubles. */
igm_status igm_batch_solve(igm_batch *bt, double *x);

/* Result of system i in the last solve: status, refinements, iterations,
 * first_ovf, shift_retries, relres_orig, relres_scaled, time_solve_ms (device wall time from
 * the start to the end of the system's solve), n, nnz, nterms, grid_blocks
 * (its team size), block_threads, rows_per_thread. */
igm_status igm_batch_get_result(const igm_batch *bt, int32_t i, igm_stats *out);

/* Whole-batch statistics of the last solve: status as returned by the solve,
 * refinements and iterations summed over the systems, time_solve_ms (host
 * wall time), time_kernel_ms (GPU time of the launch by HIP events),
 * time_setup_ms, n and nnz summed, grid_blocks / block_threads /
 * rows_per_thread of the launch, device_bytes. */
igm_status igm_batch_get_stats(const igm_batch *bt, igm_stats *out);

/* Release all device and host memory of the batch. NULL is a no-op. */
void igm_batch_destroy(igm_batch *bt);

/* ---- Served solver: continuous batching of a stream of solve requests ----
 * A persistent kernel stays resident on the device and takes jobs from a ring
 * in pinned host memory while it runs. Submitted requests are prepared on
 * host threads (validation, scaling, integer matrices, preconditioner) into
 * a staging area of pinned host memory, then admitted as soon as a slot,
 * device memory for the request's whole footprint (inputs, factors, Krylov
 * basis, work vectors) and enough idle workgroups for its team are free;
 * requests that do not fit wait while smaller ones behind them may pass. The
 * kernel's workgroups copy an admitted request's inputs to the device
 * themselves and write x back to the staging area, so no runtime copy runs
 * while the kernel is resident. Requests overlap on the device, each solved
 * as by the batched solver (bit-identical to igm_solve_device on the system
 * alone). The kernel occupies all but reserve_cus compute units until the
 * server is destroyed. Thread-safe: submit, poll and wait may be called from
 * any threads. */
typedef struct igm_server igm_server;

typedef struct {
  int32_t struct_size;      /* sizeof(igm_server_config) */
  int32_t block;            /* launch shape: (1024, 8), (1024, 4), (512, 8) or (512, 16); 0 = (512, 16) */
  int32_t rows_per_thread;
  int32_t max_slots;        /* requests resident at once; 0 = 256 */
  int32_t setup_threads;    /* host threads preparing requests; 0 = 8 */
  int32_t reserve_cus;      /* compute units the resident kernel leaves free; 0 = 8, < 0 = none.
                               This does not make other device work safe beside a server: work
                               the application enqueued on the same device while a server existed
                               did not complete (see igm_server_create) */
  int64_t pool_bytes;       /* device memory for resident requests; 0 = 16 GiB */
  int64_t stage_bytes;      /* pinned host memory for prepared requests and results; 0 = 4 GiB */
  /* 0: the host makes a request's structure (validation, diagonal positions,
   * factor patterns and level sets, SELL-64 offsets and columns) and the
   * request's team computes the values on the device before solving it
   * (scaling of eqs. (eq1)/(eq3), the integer matrix of eq. (A), the FP64
   * ILU(0) of Sec. VI-A level by level, the factor casts, the SELL-64 values;
   * the same operations in the same order as the host, so the same bits),
   * wherever that applies (one matrix term, no Gauss-Seidel splitting,
   * ILU(0) factors that fit in the request's basis array), else on the host;
   * 1: the whole setup on the host. */
  int32_t host_setup;
  int32_t reserved_[5];
} igm_server_config;

/* Start a server on the current device. Errors: IGM_ERR_ARG, IGM_ERR_OOM,
 * IGM_ERR_DEVICE, IGM_ERR_UNSUPPORTED (shape). While the server exists, enqueue
 * no other device work on that device (kernels, copies, allocations through a
 * framework): such work was seen not to complete beside the resident kernel,
 * and waiting for it then never returns. Destroy the server first. */
igm_status igm_server_create(const igm_server_config *cfg, igm_server **out);

/* Submit one solve (the arguments of igm_create_system plus an optional
 * starting iterate x0[n], NULL = zeros). Host arrays are copied during the
 * call. *ticket receives the request's number. Errors found while preparing
 * the request (IGM_ERR_ARG, IGM_ERR_SINGULAR_ROW, ...) and requests that can
 * never fit (IGM_ERR_UNSUPPORTED: m > 64, footprint above the pool, more than
 * 256 or than all resident workgroups) are reported as the request's status.
 * The persistent kernel waits for work for as long as the server exists (it
 * stops only in igm_server_destroy); if it has ended through a device failure,
 * the call returns IGM_ERR_DEVICE and requests not yet admitted finish with
 * that status. */
igm_status igm_server_submit(igm_server *sv, int64_t n, const int64_t *row_ptr, const int32_t *col,
                             const double *val, const double *b, const double *x0, const igm_policy *pol,
                             int64_t *ticket);

/* Non-blocking check of a request (returns IGM_OK). If it has finished,
 * *done = 1, x (host,
 * n doubles, may be NULL) receives the solution, *stats (may be NULL) its
 * statistics, and the request is forgotten (a ticket is collected once).
 * Statistics of a served request: status, refinements, iterations,
 * first_ovf, shift_retries, relres_orig/scaled, n, nnz, grid_blocks (team size);
 * time_solve_ms = submission to result (latency), time_setup_ms = submission
 * to prepared, time_cycle_ms = admission to result, time_kernel_ms = device
 * time of the solve. IGM_ERR_ARG for an unknown ticket. */
igm_status igm_server_poll(igm_server *sv, int64_t ticket, int32_t *done, double *x, igm_stats *stats);

/* Blocking version of igm_server_poll with a timeout in ms (< 0 = no limit):
 * IGM_OK once the request has finished (its own status is stats->status),
 * IGM_PENDING if the timeout expired (the request stays pending). */
igm_status igm_server_wait(igm_server *sv, int64_t ticket, double timeout_ms, double *x, igm_stats *stats);

typedef struct {
  int32_t struct_size;
  int32_t slots_used;       /* requests resident now */
  int64_t submitted, completed, prepared_waiting, resident;
  int64_t pool_bytes, pool_used, pool_peak;
  int64_t workgroups, workgroups_busy;
  int32_t block_threads, rows_per_thread;
  int64_t setup_waiting;    /* submitted, not yet prepared */
  int64_t jobs_published;   /* workgroup jobs handed to the persistent kernel so far */
  int32_t kernel_alive;     /* the persistent kernel is running */
  int32_t reserved_[5];
} igm_server_stats;

igm_status igm_server_get_stats(igm_server *sv, igm_server_stats *out);

/* Finish every request already submitted (waiting at most timeout_ms, < 0 =
 * no limit), stop the persistent kernel and release everything. NULL is a
 * no-op. */
void igm_server_destroy(igm_server *sv, double timeout_ms);

/* Static description of a status code. */
const char *igm_status_str(igm_status st);

#ifdef __cplusplus
}
#endif

#endif /* IGMRES_H */
