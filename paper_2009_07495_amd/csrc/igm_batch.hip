// Batched and served solver: many independent systems, each solved
// completely (Fig. 1 of the paper: FP64 iterative refinement around
// int-GMRES(m) calls, Fig. 2 with the preconditioned product of Sec. VI) by a
// team of workgroups
// inside one persistent cooperative launch. Every system carries its own
// policy (shifts, m, preconditioner: none, Jacobi or ILU(0)).
//
// Workgroups claim jobs (system, member) from a queue: in batch mode a list
// the host laid out before the launch (largest systems first), in served mode
// a ring in pinned host memory that the host appends to while the kernel runs
// (a workgroup whose claim is not yet published waits, bounded, for it). The
// members of one system are consecutive, so they start together and every
// started team can finish.
// Thread t of member q owns rows q*BLOCK + t + k*T*BLOCK (k < R) of its system
// and keeps its rows of w (Arnoldi step) and of the FP64 vectors r, rhat and
// r0 (refinement step) in registers; rows >= n hold zeros. Every reduction is
// exact (integer sums, maxima, and the order-free FP64 norm), so the bits of a
// system depend neither on its team size, the launch shape, nor the other
// systems of the batch: they equal those of the single-system solver.
#include "igm_batch.hpp"
#include "igm_dsetup.hpp"
#include "igm_rows.hpp"
#include "igm_sweep.hpp"
#include "igm_team.hpp"

namespace igm {

// entries of an ILU row loaded before a sweep waits (the kernel is short of
// registers; the single-system kernel loads 16)
constexpr int kBatchSweepPre = 8;

namespace {

constexpr int kGivensThread = 64;  // runs the scalar Givens work (wavefront 1, lane 0)
constexpr double kDblMax = 1.7976931348623157e308;

__device__ __forceinline__ double relres_of(double rn, double bn) {
  if (bn > 0.0) return rn / bn;
  return rn == 0.0 ? 0.0 : __builtin_inf();
}

__device__ __forceinline__ bool finite_pos(double v) { return v > 0.0 && v <= kDblMax; }

__device__ __forceinline__ double from_bits(unsigned long long b) { return __longlong_as_double((long long)b); }

// Adds floor(2^96 (x / mu)^2) to three 32-bit limb sums.
__device__ __forceinline__ void add_sq_limbs(double x, double mu, unsigned long long (&l)[3]) {
  const double t = x / mu;
  const unsigned __int128 q = fix96(t * t);
  l[0] += (unsigned long long)q & 0xFFFFFFFFull;
  l[1] += (unsigned long long)(q >> 32) & 0xFFFFFFFFull;
  l[2] += (unsigned long long)(q >> 64);
}

// ||x|| = mu * sqrt(rn(S)) * 2^-48 from the exact limb sums S (the
// order-free FP64 norm; mu = max |x_i|).
__device__ __forceinline__ double norm_from(const unsigned long long (&l)[3], double mu) {
  if (!finite_pos(mu)) return mu;
  const unsigned __int128 S =
      ((unsigned __int128)l[2] << 64) + ((unsigned __int128)l[1] << 32) + (unsigned __int128)l[0];
  return mu * ldexp(sqrt(u128_to_double_rn(S)), -48);
}

// Order-free norms of two register-resident vectors (rows >= n hold 0);
// returns the norms and the maxima of |x|.
template <int BLOCK, int R>
__device__ __forceinline__ void team_norm2(Team &tm, TeamShared &sh, const double (&xa)[R], const double (&xb)[R],
                                           double &na, double &nb, double &mua, double &mub) {
  unsigned long long mx[2] = {0, 0};
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const unsigned long long ta = dbits(fabs(xa[k])), tb = dbits(fabs(xb[k]));
    mx[0] = ta > mx[0] ? ta : mx[0];
    mx[1] = tb > mx[1] ? tb : mx[1];
  }
  team_reduce<BLOCK, 2, true>(tm, sh, mx);
  mua = from_bits(mx[0]);
  mub = from_bits(mx[1]);
  unsigned long long la[3] = {0, 0, 0}, lb[3] = {0, 0, 0};
  if (finite_pos(mua)) {
#pragma unroll
    for (int k = 0; k < R; ++k) add_sq_limbs(xa[k], mua, la);
  }
  if (finite_pos(mub)) {
#pragma unroll
    for (int k = 0; k < R; ++k) add_sq_limbs(xb[k], mub, lb);
  }
  team_reduce<BLOCK, 3, false>(tm, sh, la);
  team_reduce<BLOCK, 3, false>(tm, sh, lb);
  na = norm_from(la, mua);
  nb = norm_from(lb, mub);
}

template <int BLOCK, int R>
__device__ __forceinline__ double team_norm1(Team &tm, TeamShared &sh, const double (&x)[R]) {
  unsigned long long mx[1] = {0};
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const unsigned long long t = dbits(fabs(x[k]));
    mx[0] = t > mx[0] ? t : mx[0];
  }
  team_reduce<BLOCK, 1, true>(tm, sh, mx);
  const double mu = from_bits(mx[0]);
  unsigned long long l[3] = {0, 0, 0};
  if (finite_pos(mu)) {
#pragma unroll
    for (int k = 0; k < R; ++k) add_sq_limbs(x[k], mu, l);
  }
  team_reduce<BLOCK, 3, false>(tm, sh, l);
  return norm_from(l, mu);
}

// overflow events travel through the max-reductions as 2^53 - code (0 = none)
constexpr int64_t kEvBias = (int64_t)1 << 53;

// A team's working shifts: the policy's, adjusted by overflow retries
// (adjust_shift_fields). Kept wavefront-uniform so they stay in scalar registers.
struct CallShifts {
  int32_t b_dot, b_axpy, b_norm, b_div_num, b_div_den, b_rot, b_tmp, b_cs_num, b_cs_den;
  __device__ void uniform() {
    int32_t *f[] = {&b_dot, &b_axpy, &b_norm, &b_div_num, &b_div_den, &b_rot, &b_tmp, &b_cs_num, &b_cs_den};
#pragma unroll
    for (int32_t *p : f) *p = __builtin_amdgcn_readfirstlane(*p);
  }
};

}  // namespace

// minimum wavefronts per SIMD the compiler must allow, which bounds the
// registers per thread (4 -> 128, 2 -> 256). A 1024-thread workgroup always
// has 4 per SIMD; smaller workgroups get 256 registers (one or two resident
// per compute unit): the kernel then spills far less, which measured faster
// than more resident workgroups.
#ifndef IGM_BATCH_WAVES_SMALL
#define IGM_BATCH_WAVES_SMALL 2
#endif
template <int BLOCK>
constexpr int batch_waves() { return BLOCK >= 1024 ? 4 : IGM_BATCH_WAVES_SMALL; }

template <int BLOCK, int R, bool SERVED>
__global__ __launch_bounds__(BLOCK, batch_waves<BLOCK>()) void k_batch(BatchArgs ba) {
  extern __shared__ int64_t smem[];
  __shared__ TeamShared tsh;
  __shared__ BatchSys srec;  // served mode: this job's record, read coherently
  __shared__ int sh_job, sh_sid, sh_member, sh_stop, sh_jstar, sh_steps;
  __shared__ long long sh_ovf;  // smallest overflow event of the current call in this workgroup

  const int tid = threadIdx.x;

  for (;;) {
    // ---- claim the next job: (system, member)
    if (tid == 0) {
      const int c = atomicAdd(ba.queue, 1);
      int job = -1;  // -1: nothing left, leave
      int sid = 0, member = 0;
      if (!SERVED) {
        if (c < ba.njobs) {
          job = c;
          sid = ba.jobs[2 * c];
          member = ba.jobs[2 * c + 1];
        }
      } else {
        // served mode: wait until the host has published job c, or has
        // asked the kernel to stop (it does so only once every request it
        // admitted has finished, so no published job is ever left behind);
        // a workgroup never leaves on its own, since the host may publish
        // into the ticket it holds at any time. The pause between polls of
        // host memory grows to ~16 x 8k clocks.
        for (int64_t idle = 0;; ++idle) {
          if (c < __hip_atomic_load(ba.host_published, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM)) {
            job = c;
            break;
          }
          if (__hip_atomic_load(ba.host_stop, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM)) break;
          const int pauses = idle < 64 ? 1 : 16;
          for (int k = 0; k < pauses; ++k) __builtin_amdgcn_s_sleep(127);
        }
        if (job >= 0) {
          const int64_t e = 2 * (int64_t)(c % ba.ring);
          sid = __hip_atomic_load(ba.host_jobs + e, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
          member = __hip_atomic_load(ba.host_jobs + e + 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
        }
      }
      sh_job = job;
      sh_sid = sid;
      sh_member = member;
    }
    team_init(tsh);
    __syncthreads();
    // uniform values: the record then loads through scalar loads
    const int job = __builtin_amdgcn_readfirstlane(sh_job);
    if (job < 0) break;
    const int sid = __builtin_amdgcn_readfirstlane(sh_sid);
    const int member = __builtin_amdgcn_readfirstlane(sh_member);
    if (SERVED) {
      // the host wrote this slot's record and inputs before publishing the
      // job; the record is read with coherent loads into LDS (a slot's record
      // changes between requests)
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "");
      static_assert(sizeof(BatchSys) % 8 == 0, "record copied in 64-bit words");
      const unsigned long long *src = (const unsigned long long *)(ba.sys + sid);
      for (int i = tid; i < (int)(sizeof(BatchSys) / 8); i += BLOCK)
        ((unsigned long long *)&srec)[i] = __hip_atomic_load(src + i, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      __syncthreads();
    }
    const BatchSys &S = SERVED ? srec : ba.sys[sid];
    if (SERVED) {
      // the members copy the staged inputs (pinned host memory) into the
      // request's device region, each its share, then meet on the slot's
      // arrival counter (monotonic: the target counts every member of every
      // request the slot has held)
      const int64_t units = S.up_bytes / 16;
      const int64_t per = (units + S.team - 1) / S.team;
      const int64_t lo = (int64_t)member * per, hi = lo + per < units ? lo + per : units;
      const uint4 *__restrict__ src = (const uint4 *)S.src;
      uint4 *__restrict__ dst = (uint4 *)S.dst;
      for (int64_t i = lo + tid; i < hi; i += BLOCK) dst[i] = src[i];
      __syncthreads();
      if (tid == 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __hip_atomic_fetch_add(S.arrive, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        for (int spin = 0;; ++spin) {
          if ((int64_t)__hip_atomic_load(S.arrive, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= S.arrive_target)
            break;
          if (spin >= kSpinLimit) {
            tsh.abort = 1;
            __hip_atomic_store(ba.timeout, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
          }
          __builtin_amdgcn_s_sleep(IGM_POLL_SLEEP);
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      }
      __syncthreads();
    }
    const int m = S.m, df = S.df, pre = S.precond;
    int64_t *sc = smem;                                 // c_1..c_m
    int64_t *ss = sc + m;                               // s_1..s_m
    int64_t *sg = ss + m;                               // g_1..g_{m+1}
    int64_t *col = sg + m + 1;                          // current column h_{1..j+1, j}
    int64_t *sH = col + m + 1;                          // H, (m+1) x m, row-major
    double *sy = (double *)(sH + (size_t)(m + 1) * m);  // y of the closing least-squares step
    Team tm{S.words, S.team, member, 0, ba.timeout};
    const int64_t n = S.n, ldv = S.ldv;
    const int64_t TB = (int64_t)S.team * BLOCK;
    const int64_t g0 = (int64_t)member * BLOCK + tid;
    // row slots k < nk hold at least one row of this wavefront (wave-uniform)
    const int64_t wbase = (int64_t)member * BLOCK + (tid & ~63);
    const int nk = __builtin_amdgcn_readfirstlane(
        wbase < n ? (int)((n - wbase + TB - 1) / TB < R ? (n - wbase + TB - 1) / TB : R) : 0);
    double *__restrict__ x = S.x;
    const uint64_t t_begin = wall_clock64();
    const bool timer = ba.phase_clock && member == 0 && tid == 0;
    uint64_t ph[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    uint64_t t_prev = t_begin;
#define IGM_TICK(k)                      \
  if (timer) {                           \
    const uint64_t t_ = wall_clock64();  \
    ph[k] += t_ - t_prev;                \
    t_prev = t_;                         \
  }

    // served requests with a device setup: the values of the setup first
    const igm_status setup_status =
        (SERVED && S.device_setup) ? device_setup<BLOCK>(tm, tsh, S, g0, TB) : IGM_OK;

    // ILU level counters start from zero for every solve; the exchanges of
    // the norms below order these stores before any member's first sweep
    if (pre == IGM_PRE_ILU0 && S.team > 1) {
      for (int64_t i = g0; i < (int64_t)S.nflev + S.nblev; i += TB) st_coh(S.lev_cnt + i * kLevStride, 0u);
      wait_vm();
    }
    unsigned sround = 0;  // sweeps run since the counters were cleared
    const int64_t spos0 = (int64_t)member * S.sweep_threads + tid;
    const int64_t sstride = (int64_t)S.team * S.sweep_threads;
    const bool sweeper = tid < S.sweep_threads;

    // denominators of the two relative residuals
    double nb, nbh;
    {
      double xa[R], xb[R], mua, mub;
#pragma unroll
      for (int k = 0; k < R; ++k) {
        const int64_t row = g0 + k * TB;
        xa[k] = row < n ? S.b[row] : 0.0;
        xb[k] = row < n ? S.bhat[row] : 0.0;
      }
      team_norm2<BLOCK, R>(tm, tsh, xa, xb, nb, nbh, mua, mub);
    }

    int status = IGM_NOT_CONVERGED, refinements = 0, iterations = 0, jstar_last = -1, retries = 0;
    CallShifts sf{S.b_dot, S.b_axpy, S.b_norm, S.b_div_num, S.b_div_den, S.b_rot, S.b_tmp, S.b_cs_num, S.b_cs_den};
    sf.uniform();
    // an int-GMRES call that overflows and can adjust a shift is repeated: the
    // refinement starts again from the same x, so the residual step rebuilds
    // the same v1 bit for bit
    bool again = false;
    int64_t first_ovf = kNoEvent;
    double ro = 0.0, rs = 0.0;
    for (int kref = 0;; kref += again ? 0 : 1) {
      again = false;
      if (tsh.abort) break;
      if (setup_status != IGM_OK) { status = setup_status; break; }
      // integer matrix terms of this refinement (k = kref + 1): Abar_0 and s(k) corrections, eq. (AA)
      const int nterms_k = S.s_rule ? (S.nterms < kref + 1 ? S.nterms : kref + 1) : S.nterms;
      // ---- eq. (b): r = b - A x and rhat = bhat - Ahat x, rows in CSR order
      double r[R], rh[R];
#pragma unroll
      for (int k = 0; k < R; ++k) {
        const int64_t row = g0 + k * TB;
        r[k] = 0.0;
        rh[k] = 0.0;
        if (row < n) {
          residual_row(S.row_ptr[row], S.row_ptr[row + 1], S.col, S.a, S.ahat, x, S.b[row], S.bhat[row], r[k], rh[k]);
          // eq. (eq2): x holds xhat and the scaled residual is D1^-1 (bhat - Ahat xhat)
          if (S.cscale) r[k] = rh[k] / S.cscale[row];
        }
      }
      double nr, nrh, gamma, mu_rh;
      team_norm2<BLOCK, R>(tm, tsh, r, rh, nr, nrh, gamma, mu_rh);
      ro = relres_of(nrh, nbh);
      rs = relres_of(nr, nb);
      if (tsh.abort) break;
      if (!(ro <= kDblMax && ro >= -kDblMax)) { status = IGM_ERR_RANGE; break; }
      if (ro < S.tol) { status = IGM_OK; break; }
      if (kref >= S.max_refine) { status = IGM_NOT_CONVERGED; break; }
      // gamma = max |r| (eq. (gammak)); gamma == 0 means r == 0
      if (gamma == 0.0) { status = IGM_OK; break; }
      // ---- FP64 start step (Sec. VI): b^(k) = r / gamma, r0 = Mbar^-1 b^(k) in FP64
#pragma unroll
      for (int k = 0; k < R; ++k) {
        const int64_t row = g0 + k * TB;
        if (row < n) {
          const double t = r[k] / gamma;
          double u = t;
          if (pre == IGM_PRE_JACOBI) u = (t / (double)S.ldiag[row]) / (double)S.udiag[row];
          r[k] = u;
        }
      }
      if (pre == IGM_PRE_ILU0) {
        // FP64 forward and backward substitution with the integer factors
        // (converted exactly) in place in fbuf; each row sums in CSR order
        // and then divides by its diagonal
#pragma unroll
        for (int k = 0; k < R; ++k) {
          const int64_t row = g0 + k * TB;
          if (row < n) st_coh(S.fbuf + row, r[k]);
        }
        team_barrier_coh(tm, tsh);
        if (S.team == 1) {
          // one workgroup: levels separated by workgroup barriers
          for (int L = 0; L < S.nflev; ++L) {
            for (int64_t q = S.flev_ptr[L] + tid; q < S.flev_ptr[L + 1]; q += BLOCK) {
              const int64_t i = S.flev_rows[q];
              S.fbuf[i] = fp_sub_row(S.lptr[i], S.lptr[i + 1], S.lcol, S.lvalf, S.fbuf, ld_coh(S.fbuf + i),
                                     (double)S.ldiag[i]);
            }
            __syncthreads();
          }
          for (int L = 0; L < S.nblev; ++L) {
            for (int64_t q = S.blev_ptr[L] + tid; q < S.blev_ptr[L + 1]; q += BLOCK) {
              const int64_t i = S.blev_rows[q];
              S.fbuf[i] = fp_sub_row(S.uptr[i], S.uptr[i + 1], S.ucol, S.uvalf, S.fbuf, S.fbuf[i],
                                     (double)S.udiag[i]);
            }
            __syncthreads();
          }
#pragma unroll
          for (int k = 0; k < R; ++k) {
            const int64_t row = g0 + k * TB;
            r[k] = row < n ? S.fbuf[row] : 0.0;
          }
        } else {
          // several members: each row waits only for the level below it
          bool fo = false, to = false;
          if (sweeper && !tsh.abort)
            level_sweep<true, true, kBatchSweepPre>(S, S.flev_ptr, S.flev_rows, S.nflev, S.lev_cnt, sround, spos0, sstride, S.fbuf,
                                    S.fbuf, fo, to);
          team_barrier_coh(tm, tsh);
          if (sweeper && !tsh.abort)
            level_sweep<false, true, kBatchSweepPre>(S, S.blev_ptr, S.blev_rows, S.nblev, S.lev_cnt + (int64_t)S.nflev * kLevStride,
                                     sround, spos0, sstride, S.fbuf, S.fbuf, fo, to);
          ++sround;
          if (to) team_abort(tm, tsh);
          team_barrier_coh(tm, tsh);
#pragma unroll
          for (int k = 0; k < R; ++k) {
            const int64_t row = g0 + k * TB;
            r[k] = row < n ? ld_coh(S.fbuf + row) : 0.0;
          }
        }
      }
      const double rho = team_norm1<BLOCK, R>(tm, tsh, r);
      if (tsh.abort) break;
      if (!finite_pos(rho)) { status = IGM_ERR_RANGE; break; }
      // ---- cast of v1 to Q.df: v1 = trunc(2^df r0 / rho)
      {
        unsigned long long rerr[1] = {0};
#pragma unroll
        for (int k = 0; k < R; ++k) {
          const int64_t row = g0 + k * TB;
          if (row < n) {
            const double t = ldexp(r[k] / rho, df);
            int64_t v = 0;
            if (t >= -9223372036854775808.0 && t < 9223372036854775808.0) v = (int64_t)t;
            else rerr[0] = 1;
            S.V[row] = v;
          }
        }
        team_reduce<BLOCK, 1, true>(tm, tsh, rerr);
        if (rerr[0]) { status = IGM_ERR_RANGE; break; }
      }
      IGM_TICK(5)

      // ---- the integer loop of Fig. 2: the int-GMRES(m) call
      if (tid == 0) {
        for (int i = 0; i < m; ++i) { sc[i] = 0; ss[i] = 0; }
        for (int i = 0; i <= m; ++i) { sg[i] = 0; col[i] = 0; }
        sg[0] = (int64_t)1 << df;  // g = e_1 in Q.df
        sh_stop = 0; sh_jstar = m; sh_steps = 0;
        sh_ovf = (long long)kNoEvent;
      }
      team_barrier(tm, tsh);  // v1 visible to the team

      const int sh_dot = df - sf.b_dot;
      auto fin_dot = [&](int64_t Sv, bool &o) { return asr(Sv, sh_dot); };
      auto fin_norm = [&](int64_t Sv, bool &o) { return shl(isqrt64(Sv), sf.b_norm, o); };
      auto record = [&](int64_t code) { atomicMin(&sh_ovf, (long long)code); };

      int64_t w[R];
      int64_t carry = 0, hn = 0;
      bool lucky = false;
      // earlier rotation i (1-based) on (carry, col[i]); thread kGivensThread only
      auto rotate = [&](int j, int i) {
        const int64_t x0 = asr(carry, sf.b_rot), x1 = asr(col[i], sf.b_rot);
        const int64_t c = sc[i - 1], s = ss[i - 1];
        bool o = false;
        const int64_t ms = subc(0, s, o);
        const int64_t top = addc(mulw(x0, c, o), mulw(x1, s, o), o);
        const int64_t bot = addc(mulw(x0, ms, o), mulw(x1, c, o), o);
        col[i - 1] = asr(top, df - sf.b_rot);
        carry = asr(bot, df - sf.b_rot);
        if (o) record(ev_code(j, 6, i));
      };
      // radius, new rotation, rotation of g and H update for column j on (carry, hn); thread kGivensThread only
      auto givens = [&](int j) {
        col[j - 1] = carry;
        col[j] = hn;
        bool o = false;  // rotation radius t_mp
        const int64_t p0 = asr(col[j - 1], sf.b_tmp), p1 = asr(col[j], sf.b_tmp);
        const int64_t ssq = addc(sqrc(p0, o), sqrc(p1, o), o);
        const int64_t tmp = shl(isqrt64(ssq), sf.b_tmp, o);
        if (o) record(ev_code(j, 7, 0));
        const int64_t den2 = asr(tmp, sf.b_cs_den);  // new rotation c_j, s_j
        int stop = 0;
        if (den2 == 0) {  // new rotation: zero denominator
          sh_jstar = j - 1;
          stop = 1;
        } else {
          bool oc = false;
          const int e2 = df - sf.b_cs_num - sf.b_cs_den;
          const int64_t cj = normalize_elem(col[j - 1], den2, sf.b_cs_num, e2, oc);
          const int64_t sj = normalize_elem(col[j], den2, sf.b_cs_num, e2, oc);
          if (oc) record(ev_code(j, 8, 0));
          sc[j - 1] = cj;
          ss[j - 1] = sj;
          bool og = false;  // rotation of g, both from the old g_j
          const int64_t gj = sg[j - 1];
          const int64_t msj = subc(0, sj, og);
          sg[j - 1] = asr(mulw(gj, cj, og), df);
          sg[j] = asr(mulw(gj, msj, og), df);
          if (og) record(ev_code(j, 9, 0));
          col[j - 1] = tmp;  // h_jj = t_mp, h_{j+1,j} = 0
          col[j] = 0;
          if (lucky) {  // normalisation: zero denominator
            sh_jstar = j;
            stop = 1;
          } else if (S.gtol >= 0) {
            const int64_t gn = sg[j] < 0 ? -sg[j] : sg[j];
            if (gn <= S.gtol) { sh_jstar = j; stop = 1; }
          }
        }
        for (int i = 0; i <= j; ++i) sH[(size_t)i * m + (j - 1)] = col[i];
        sh_steps = j;
        sh_stop = stop;
      };

      for (int j = 1; j <= m; ++j) {  // Arnoldi step j
        const int64_t *__restrict__ vj = S.V + (size_t)(j - 1) * ldv;
        // ---- integer SpMV, then the preconditioner apply
        {
          bool o1 = false, o2 = false;
#pragma unroll
          for (int k = 0; k < R; ++k) {
            const int64_t row = g0 + k * TB;
            int64_t z = 0;
            if (row < n) {
              z = spmv_row(S, row, vj, nterms_k, o1);
              if (pre == IGM_PRE_JACOBI) z = tdiv_diag(tdiv_diag(z, S.ldiag[row], o2), S.udiag[row], o2);
            }
            w[k] = z;
          }
          if (o1) record(ev_code(j, 1, 0));
          if (pre == IGM_PRE_ILU0) {
            // preconditioner apply: integer forward and backward substitution; z, y and u
            // pass between members through device-coherent stores and loads
#pragma unroll
            for (int k = 0; k < R; ++k) {
              const int64_t row = g0 + k * TB;
              if (row < n) st_coh(S.zbuf + row, w[k]);
            }
            team_barrier_coh(tm, tsh);
            if (S.team == 1) {  // one workgroup, as for the start step
              for (int L = 0; L < S.nflev; ++L) {
                for (int64_t q = S.flev_ptr[L] + tid; q < S.flev_ptr[L + 1]; q += BLOCK) {
                  const int64_t row = S.flev_rows[q];
                  S.wbuf[row] = lower_row(S, row, ld_coh(S.zbuf + row), S.wbuf, o2);
                }
                __syncthreads();
              }
              for (int L = 0; L < S.nblev; ++L) {
                for (int64_t q = S.blev_ptr[L] + tid; q < S.blev_ptr[L + 1]; q += BLOCK) {
                  const int64_t row = S.blev_rows[q];
                  S.wbuf[row] = upper_row(S, row, S.wbuf[row], S.wbuf, o2);
                }
                __syncthreads();
              }
#pragma unroll
              for (int k = 0; k < R; ++k) {
                const int64_t row = g0 + k * TB;
                w[k] = row < n ? S.wbuf[row] : 0;
              }
            } else {
              bool to = false;
              if (sweeper && !tsh.abort)
                level_sweep<true, false, kBatchSweepPre>(S, S.flev_ptr, S.flev_rows, S.nflev, S.lev_cnt, sround, spos0, sstride,
                                         S.zbuf, S.wbuf, o2, to);
              team_barrier_coh(tm, tsh);
              if (sweeper && !tsh.abort)
                level_sweep<false, false, kBatchSweepPre>(S, S.blev_ptr, S.blev_rows, S.nblev,
                                          S.lev_cnt + (int64_t)S.nflev * kLevStride, sround, spos0, sstride, S.wbuf,
                                          S.wbuf, o2, to);
              ++sround;
              if (to) team_abort(tm, tsh);
              team_barrier_coh(tm, tsh);
#pragma unroll
              for (int k = 0; k < R; ++k) {
                const int64_t row = g0 + k * TB;
                w[k] = row < n ? ld_coh(S.wbuf + row) : 0;
              }
            }
          }
          if (o2) record(ev_code(j, 2, 0));
        }
        IGM_TICK(0)
        // ---- modified Gram-Schmidt, i increasing; v_{i+1} is
        // loaded before the reduction of (w, v_i) so its latency overlaps,
        // and the earlier rotation i-2 runs inside the wait.
        int64_t vv[R];
#pragma unroll
        for (int k = 0; k < R; ++k) {
          const int64_t row = g0 + k * TB;
          vv[k] = row < n ? S.V[row] : 0;
        }
        for (int i = 1; i <= j; ++i) {
          Acc acc;
          acc.zero();
          bool o = false;
#pragma unroll
          for (int k = 0; k < R; ++k)  // inner product: only w is shifted
            if (k < nk) acc.add(mulw(asr(w[k], sf.b_dot), vv[k], o));
          if (o) record(ev_code(j, 3, 2 * (i - 1)));
          int64_t vnext[R];
          if (i < j) {
            const int64_t *vi1 = S.V + (size_t)i * ldv;
#pragma unroll
            for (int k = 0; k < R; ++k) {
              const int64_t row = g0 + k * TB;
              vnext[k] = row < n ? vi1[row] : 0;
            }
          }
          IGM_TICK(1)
          bool os = false;
          const int64_t h = team_sum<BLOCK>(tm, acc, tsh, fin_dot, [&] {
            if (tid == kGivensThread && i >= 3) rotate(j, i - 2);
          }, os);
          IGM_TICK(2)
          if (os && tid == 0) record(ev_code(j, 3, 2 * (i - 1)));
          if (tid == kGivensThread) {
            col[i - 1] = h;
            if (i == 1) carry = h;
          }
          // update of w: only h is shifted
          const int64_t hs = asr(h, sf.b_axpy);
          bool ou = false;
#pragma unroll
          for (int k = 0; k < R; ++k)
            if (k < nk) w[k] = subc(w[k], asr(mulw(hs, vv[k], ou), df - sf.b_axpy), ou);
          if (ou) record(ev_code(j, 3, 2 * (i - 1) + 1));
          if (i < j) {
#pragma unroll
            for (int k = 0; k < R; ++k) vv[k] = vnext[k];
          }
          IGM_TICK(1)
        }
        // ---- norm of w (the last rotation j-1 runs during this reduction)
        {
          Acc acc;
          acc.zero();
          bool o = false;
#pragma unroll
          for (int k = 0; k < R; ++k)
            if (k < nk) acc.add(sqrc(asr(w[k], sf.b_norm), o));
          if (o) record(ev_code(j, 4, 0));
          bool os = false;
          hn = team_sum<BLOCK>(tm, acc, tsh, fin_norm, [&] {
            if (tid == kGivensThread && j >= 2) rotate(j, j - 1);
          }, os);
          if (os && tid == 0) record(ev_code(j, 4, 0));
        }
        IGM_TICK(3)
        // ---- normalisation v_{j+1} = w / h_{j+1,j}
        const int64_t den = asr(hn, sf.b_div_den);
        lucky = den == 0;
        if (!lucky) {
          int64_t *__restrict__ vn = S.V + (size_t)j * ldv;
          const int e = df - sf.b_div_num - sf.b_div_den;
          bool ov = false;
#pragma unroll
          for (int k = 0; k < R; ++k) {
            const int64_t row = g0 + k * TB;
            if (row < n) vn[row] = normalize_elem(w[k], den, sf.b_div_num, e, ov);
          }
          if (ov) record(ev_code(j, 5, 0));
        }
        IGM_TICK(4)
        // v_{j+1} becomes visible to the team; the new rotation runs meanwhile
        team_barrier(tm, tsh, [&] {
          if (tid == kGivensThread) givens(j);
        });
        IGM_TICK(6)
        if (sh_stop || tsh.abort) break;
      }
      if (tsh.abort) break;

      // the call's first overflow event over the team
      int64_t ev;
      {
        unsigned long long e1[1] = {0};
        if (tid == 0 && sh_ovf != (long long)kNoEvent) e1[0] = (unsigned long long)(kEvBias - (int64_t)sh_ovf);
        team_reduce<BLOCK, 1, true>(tm, tsh, e1);
        ev = e1[0] ? kEvBias - (int64_t)e1[0] : kNoEvent;
      }
      if (tsh.abort) break;
      // every thread of every member takes the same decision from the same event
      if (ev != kNoEvent && retries < S.shift_retry && adjust_shift_fields(sf, df, ev)) {
        retries += 1;
        sf.uniform();
        again = true;
        continue;
      }
      const int js = sh_jstar;
      refinements += 1;
      iterations += sh_steps;
      jstar_last = js;
      if (tsh.abort) break;
      if (ev != kNoEvent) { first_ovf = ev; status = IGM_ERR_OVERFLOW; break; }
      if (js == 0) { status = IGM_ERR_BREAKDOWN; break; }

      // ---- closing least-squares step and x += gamma x^(k) (eq. (update))
      if (tid == 0) {
        for (int i = js - 1; i >= 0; --i) {  // back substitution, inner sum k increasing
          double acc = 0.0;
          for (int k = i + 1; k < js; ++k) acc = acc + ldexp((double)sH[(size_t)i * m + k], -df) * sy[k];
          sy[i] = (ldexp((double)sg[i], -df) - acc) / ldexp((double)sH[(size_t)i * m + i], -df);
        }
        for (int i = 0; i < js; ++i) sy[i] = rho * sy[i];
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < R; ++k) {
        const int64_t row = g0 + k * TB;
        if (row < n) {
          double acc = 0.0;
          for (int i = 0; i < js; ++i) acc = acc + sy[i] * ldexp((double)S.V[(size_t)i * ldv + row], -df);
          x[row] = x[row] + gamma * (S.cscale ? acc / S.cscale[row] : acc);
        }
      }
      team_barrier(tm, tsh);  // x visible to the team
      IGM_TICK(5)
    }
#undef IGM_TICK
    if (tsh.abort) status = IGM_ERR_DEVICE;
    if (SERVED) {  // x back to the requester's pinned buffer
#pragma unroll
      for (int k = 0; k < R; ++k) {
        const int64_t row = g0 + k * TB;
        if (row < n) S.x_out[row] = x[row];
      }
    }
    // every member's writes of x are published before the result is
    team_barrier(tm, tsh);
    if (member == 0 && tid == 0) {
      BatchResult &res = *S.res;
      res.status = status;
      res.refinements = refinements;
      res.iterations = iterations;
      res.jstar = jstar_last;
      res.first_ovf = first_ovf;
      res.shift_retries = retries;
      res.relres_orig = ro;
      res.relres_scaled = rs;
      res.t_begin = t_begin;
      res.t_end = wall_clock64();
      for (int k = 0; k < 7; ++k) res.phase[k] = ph[k];
      res.phase[7] = res.t_end - t_begin;
      if (SERVED) {  // results and x reach memory, then the host is told
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
        __hip_atomic_store(ba.host_done + sid, S.seq, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
      }
    }
    __syncthreads();
  }
}

template <int BLOCK, int R, bool SERVED>
static const void *batch_kernel_ptr() {
  return (const void *)&k_batch<BLOCK, R, SERVED>;
}

const int kBatchShapes[][2] = {{1024, 8}, {1024, 4}, {512, 8}, {512, 16}, {256, 8}, {256, 16}};
const int kNumBatchShapes = 6;

const void *batch_kernel(int block, int R) {
#define IGM_K(BB, RR) \
  if (block == BB && R == RR) return batch_kernel_ptr<BB, RR, false>();
  IGM_K(1024, 8)
  IGM_K(1024, 4)
  IGM_K(512, 8)
  IGM_K(512, 16)
  IGM_K(256, 8)
  IGM_K(256, 16)
#undef IGM_K
  return nullptr;
}

const void *serve_kernel(int block, int R) {
  if (block == 1024 && R == 8) return batch_kernel_ptr<1024, 8, true>();
  if (block == 1024 && R == 4) return batch_kernel_ptr<1024, 4, true>();
  if (block == 512 && R == 8) return batch_kernel_ptr<512, 8, true>();
  if (block == 512 && R == 16) return batch_kernel_ptr<512, 16, true>();
  return nullptr;
}

size_t batch_smem_bytes(int m) {
  return sizeof(int64_t) * (4 * (size_t)m + 2 + (size_t)(m + 1) * m) + sizeof(double) * (size_t)m;
}

}  // namespace igm
