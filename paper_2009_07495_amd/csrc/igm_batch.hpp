// Device records of the batched and served solvers (many independent
// systems, one persistent launch).
#pragma once

#include <vector>

#include "igm_internal.hpp"

namespace igm {

struct BatchResult;

// One system: its policy, read-only inputs and setup products, its Krylov
// basis, work vectors and team exchange area. Field names of the integer
// matrix and factors match CycleArgs so the per-row kernels serve all paths.
struct BatchSys {
  int64_t n;       // rows
  int64_t ldv;     // leading dimension of V (n rounded up to 16)
  int32_t team;    // workgroups that share the system
  int32_t nterms;  // integer matrix terms used by the SpMV (at most; see s_rule)
  int32_t s_rule;  // s(k) of eq. (AA): 0 = nterms in every refinement, 1 = min(nterms, k) in refinement k
  int32_t m, df, precond, max_refine;
  int32_t b_dot, b_axpy, b_norm, b_div_num, b_div_den, b_rot, b_tmp, b_cs_num, b_cs_den;
  int32_t nflev, nblev;  // ILU level sets
  int32_t seq;           // served mode: request number reported on completion
  int32_t max_level;     // rows of the largest ILU level set
  int32_t sweep_threads; // ILU, teams of several workgroups: threads per member in the sweeps
  int64_t gtol;
  double tol;
  int32_t alpha[kMaxTerms];
  const int64_t *row_ptr;
  const int32_t *col;
  const double *a, *ahat, *b, *bhat;  // scaled and original FP64 matrix / rhs
  const int64_t *sell_off;
  const int32_t *sell_w;
  const int32_t *sell_col;
  const int64_t *sell_val[kMaxTerms];
  const int64_t *ldiag, *udiag;  // cast diagonals (Jacobi, ILU)
  const int64_t *lptr, *uptr;    // strict triangles of the integer ILU factors
  const int32_t *lcol, *ucol;
  const int64_t *lval, *uval;
  const double *lvalf, *uvalf;   // the same values in FP64 (start step)
  const int32_t *flev_ptr, *flev_rows, *blev_ptr, *blev_rows;
  // device setup (device_setup = 1): the kernel computes a, b, sell_val[0],
  // ldiag, udiag, lval, uval, lvalf, uvalf from ahat, bhat and the structure
  // (diag_pos: each row's diagonal entry) before the solve
  int32_t device_setup;
  int32_t alpha_a;
  const int64_t *diag_pos;
  // eq. (eq2) (two-sided scaling): s_i = sqrt(dhat_i), null for eq. (eq1);
  // the scaled residual is rhat_i / s_i and the update adds gamma x^(k)_i / s_i
  const double *cscale;
  // int-GMRES calls that overflow are repeated from the same v1 with adjusted
  // shifts, at most shift_retry times per solve (igm_policy.shift_retry)
  int32_t shift_retry;
  int32_t pad_;
  int64_t *V;                    // (m+1) x ldv basis
  int64_t *zbuf, *wbuf;          // ILU: SpMV output and preconditioned vector
  double *fbuf;                  // ILU: FP64 substitution of the start step
  unsigned *lev_cnt;             // ILU: level completion counters (cleared by the kernel)
  double *x;                     // solution (in: start, out: result)
  unsigned long long *words;     // team exchange words
  BatchResult *res;              // written by the first member
  // served mode: the members first copy the staged inputs (pinned host
  // memory, up_bytes from src) into the region at dst, meet on the arrival
  // counter, and finally copy x out to x_out (pinned host memory)
  const char *src;
  char *dst;
  int64_t up_bytes;
  double *x_out;
  unsigned long long *arrive;
  int64_t arrive_target;
};

// Outcome of one system, written by its first member.
struct BatchResult {
  int32_t status, refinements, iterations, jstar;
  int64_t first_ovf;
  int32_t shift_retries;  // calls repeated with adjusted shifts
  int32_t pad_;
  double relres_orig, relres_scaled;
  uint64_t t_begin, t_end;  // device wall clock (start and end of the solve)
  // wall-clock ticks of the first member's thread 0 per phase: 0 SpMV +
  // preconditioner, 1 inner products and updates (local work), 2 waits for
  // the inner-product sums, 3 norm, 4 normalisation, 5 FP64 refinement steps
  // (residual, norms, start step and cast of v1, closing least-squares step),
  // 6 end-of-step barriers
  uint64_t phase[8];
};

struct BatchArgs {
  BatchSys *sys;        // system records (served mode: one per slot)
  const int32_t *jobs;  // batch mode: pairs (system, member) in claim order
  int32_t njobs;        // batch mode: number of jobs
  int32_t phase_clock;  // record the phase clocks of each system's first member
  int32_t *queue;       // next claim
  int32_t *timeout;     // set when a team wait timed out
  // served mode: the host publishes jobs while the kernel runs (pinned host memory)
  const int32_t *host_jobs;       // ring of pairs (slot, member)
  const int64_t *host_published;  // jobs published so far
  const int32_t *host_stop;       // 1 = exit once no published job is left
  int32_t *host_done;             // per slot: seq of the last completed request
  int32_t ring;                   // capacity of host_jobs in pairs (0 = batch mode)
  int32_t pad_;
};

// ---- host side, shared by the batched and the served solver ----

// A validated system with its host setup products (everything the device
// needs, in the layouts the kernels read).
struct HostSystem {
  int64_t n = 0, nnz = 0;
  igm_policy pol{};
  hvec<int64_t> row_ptr;
  hvec<int32_t> col;
  hvec<double> ahat, bhat;
  HostSetup h;
  int nterms = 1;
  hvec<double> lvalf, uvalf;  // FP64 copies of the integer factors (start step)
  // the values of the setup (scaling, integer matrix, factors) are computed
  // by the solving kernel from the inputs; the host made the structure only
  bool device_setup = false;
};

// Largest m of the batched kernel (H lives in LDS).
constexpr int kMaxBatchM = 64;

// Validates (as igm_create_system) and runs the host setup of one system.
// With allow_device_setup the host makes only the structure when the kernel
// can compute the values (one matrix term, no Gauss-Seidel splitting, ILU(0)
// factors that fit in the basis array during the setup).
igm_status prepare_system(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
                          const double *b, const igm_policy &pol, HostSystem &out, bool allow_device_setup = false);
// Device bytes of one system's region (inputs, setup products, basis, work
// vectors, exchange words; the solution vector only if own_x).
size_t system_bytes(const HostSystem &hs, bool own_x);
// Leading part of the region (own_x) that holds data: inputs, setup
// products, x and the exchange words; the work arrays follow it.
size_t image_bytes(const HostSystem &hs);
// Writes that leading part into img (host memory): the arrays, x = x0 (zeros
// if x0 is null), zero exchange words.
void build_image(const HostSystem &hs, char *img, const double *x0);
// The record of a system placed at device address base (own_x), pointers
// only (team = 1, no result, served fields unset).
void record_for(const HostSystem &hs, bool own_x, char *base, BatchSys &S);
// Queues the uploads of one system into the region at `base` on `st` and
// fills its record (team = 1, res = nullptr; x = the region's own vector if
// own_x, else left null). The host vectors must live until `st` has drained.
hipError_t place_system(const HostSystem &hs, char *base, bool own_x, hipStream_t st, BatchSys &S);

const void *batch_kernel(int block, int R);
// the served variant (jobs from a host ring, records read coherently):
// shapes (1024, 8), (1024, 4), (512, 8) and (512, 16)
const void *serve_kernel(int block, int R);
size_t batch_smem_bytes(int m);
// the (block, rows per thread) shapes instantiated for the batched kernel
extern const int kBatchShapes[][2];
extern const int kNumBatchShapes;

}  // namespace igm
