// The int-GMRES(m) call of the paper (the integer loop of Fig. 2, with the
// preconditioned product of Sec. VI, and optionally the closing FP64
// least-squares step of Fig. 2 plus the refinement update of eq. (update)) as
// one persistent cooperative kernel.
//
// Layout: thread t of workgroup b owns rows r = b*BLOCK + t + k*T (k < R,
// T = gridDim.x*BLOCK) and keeps w_r in registers for the whole Arnoldi step;
// consecutive lanes own consecutive rows, so every vector access and the
// SELL-64 matrix stream are coalesced. Each inner product of the modified
// Gram-Schmidt loop is one exact grid reduction (igm_sync.hpp). The scalar
// Givens work (rotations of H and g) runs in thread kGivens of every workgroup on identical
// data, so all workgroups take the same decisions without extra
// communication; it is scheduled inside the waits of the grid reductions and
// barriers. Workgroup 0 stores H, c, s, g for the caller.
#pragma once
#include "igm_bsweep.hpp"
#include "igm_rows.hpp"
#include "igm_sync.hpp"

namespace igm {

// thread that runs the scalar Givens work (wavefront 1, lane 0)
constexpr int kGivens = 64;

// v_{j+1} passes to the other workgroups' SpMV gathers through write-through
// (device-coherent) stores and a barrier that only waits for them to
// complete: no cache write-back or invalidation, so cached matrix lines
// survive the step. Plain loads of v_{j+1} are safe because its cache lines
// are first touched in a launch by their one owner workgroup's stores (a
// workgroup owns whole blocks of BLOCK consecutive rows, BLOCK a multiple of
// the 16 words of a cache line), other workgroups first read them
// after that barrier, and a launch starts with caches coherent with memory.

// One integer sweep of the ILU(0) preconditioner apply, 4 lanes per row
// (the bits do not depend on the width; building 8 and 16 lanes per row into
// the kernel as well raised its spills, so igm_policy.sweep_lanes is not used).
template <int BLOCK>
__device__ __forceinline__ void ilu_sweep(const BlockSweepArgs &b, const int64_t *src, int64_t *dst,
                                          char *lds, bool &ovf, bool &to) {
  block_sweep_int<BLOCK, 4>(b, src, dst, lds, ovf, to);
}

// The integer SpMV of row `row` (chunk of BLOCK rows from row0, the one this
// workgroup owns) with row-to-lane mapping MAP: one thread per row over SELL-64,
// a.spmv_lanes lanes per row over CSR, or the chunk's entries split evenly
// over the workgroup (both through the LDS at lds; every thread calls).
template <int BLOCK, int MAP>
__device__ __forceinline__ int64_t cycle_spmv(const CycleArgs &a, int64_t row, int64_t row0,
                                              const int64_t *__restrict__ vj, char *lds, bool &ovf) {
  if constexpr (MAP == kMapMerge) {
    return spmv_chunk_merge<BLOCK>(a, row0, vj, a.nterms, lds, ovf);
  } else if constexpr (MAP == kMapLanes) {
    int64_t *zl = (int64_t *)lds;
    spmv_chunk_lanes<BLOCK>(a, row0, vj, a.nterms, a.spmv_lanes, zl, ovf);
    __syncthreads();
    const int64_t z = zl[threadIdx.x];
    __syncthreads();
    return z;
  } else {
    // the matrix is streamed: each Arnoldi step reads it once, and its lines
    // would only evict the basis and the gathered vector
    return spmv_row<kRowChunk, true>(a, row, vj, a.nterms, ovf);
  }
}

template <int BLOCK, int R, int PRE, int MAP>
__global__ __launch_bounds__(BLOCK) void k_cycle(CycleArgs a) {
  extern __shared__ int64_t smem[];
  const int m = a.m;
  int64_t *sc = smem;             // c_1..c_m
  int64_t *ss = sc + m;           // s_1..s_m
  int64_t *sg = ss + m;           // g_1..g_{m+1}
  int64_t *col = sg + m + 1;      // current column h_{1..j+1, j}
  double *sy = (double *)(col + m + 1);  // y of the closing least-squares step
  __shared__ SyncShared ssh;
  __shared__ int sh_stop, sh_jstar, sh_breakdown, sh_steps, sh_update;

  const int tid = threadIdx.x;
  const int64_t T = (int64_t)gridDim.x * BLOCK;
  const int64_t gt = (int64_t)blockIdx.x * BLOCK + tid;
  const int df = a.df;
  int64_t *first = &a.state->first_ovf;
  GridSync gs{a.sync, a.sync_cap, (int)gridDim.x, 0, &a.state->timeout};
  // phase clock of thread 0 of workgroup 0 (100 MHz wall clock)
  const bool timer = a.phase_clock && blockIdx.x == 0 && tid == 0;
  uint64_t ph[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  const uint64_t t_start = timer ? wall_clock64() : 0;
  uint64_t t_prev = t_start;
#define IGM_TICK(k)                      \
  if (timer) {                           \
    const uint64_t t_ = wall_clock64();  \
    ph[k] += t_ - t_prev;                \
    t_prev = t_;                         \
  }

  if (tid == 0) {
    for (int i = 0; i < m; ++i) { sc[i] = 0; ss[i] = 0; }
    for (int i = 0; i <= m; ++i) { sg[i] = 0; col[i] = 0; }
    sg[0] = (int64_t)1 << df;  // g = e_1 in Q.df
    ssh.abort = 0; ssh.flag = 0;
    sh_stop = 0; sh_jstar = m; sh_breakdown = 0; sh_steps = 0;
  }
  __syncthreads();

  // reduction finishers (run once per workgroup, in wavefront 0)
  const int sh_dot = df - a.b_dot;
  auto fin_dot = [&](int64_t S, bool &o) { return asr(S, sh_dot); };
  auto fin_norm = [&](int64_t S, bool &o) { return shl(isqrt64(S), a.b_norm, o); };
  auto no_side = [] {};

  int64_t w[R];
  int64_t carry = 0;  // rotated lower entry of the current column (thread kGivens)
  int64_t hn = 0;     // h_{j+1,j}
  bool lucky = false;
  // earlier rotation i (1-based) on (carry, col[i]); thread kGivens only
  auto rotate = [&](int j, int i) {
    const int64_t x0 = asr(carry, a.b_rot), x1 = asr(col[i], a.b_rot);
    const int64_t c = sc[i - 1], s = ss[i - 1];
    bool o = false;
    const int64_t ms = subc(0, s, o);
    const int64_t top = addc(mulw(x0, c, o), mulw(x1, s, o), o);
    const int64_t bot = addc(mulw(x0, ms, o), mulw(x1, c, o), o);
    col[i - 1] = asr(top, df - a.b_rot);
    carry = asr(bot, df - a.b_rot);
    if (o) atomicMin((long long *)first, (long long)ev_code(j, 6, i));
  };
  // radius, new rotation, rotation of g and H update for column j on (carry, hn); thread kGivens only
  auto givens = [&](int j) {
    col[j - 1] = carry;
    col[j] = hn;
    bool o = false;  // rotation radius t_mp
    const int64_t p0 = asr(col[j - 1], a.b_tmp), p1 = asr(col[j], a.b_tmp);
    const int64_t ssq = addc(sqrc(p0, o), sqrc(p1, o), o);
    const int64_t tmp = shl(isqrt64(ssq), a.b_tmp, o);
    if (o) atomicMin((long long *)first, (long long)ev_code(j, 7, 0));
    const int64_t den2 = asr(tmp, a.b_cs_den);  // new rotation c_j, s_j
    int stop = 0;
    if (den2 == 0) {
      sh_breakdown = 2;
      sh_jstar = j - 1;
      stop = 1;
    } else {
      bool oc = false;
      const int e2 = df - a.b_cs_num - a.b_cs_den;
      const int64_t cj = normalize_elem(col[j - 1], den2, a.b_cs_num, e2, oc);
      const int64_t sj = normalize_elem(col[j], den2, a.b_cs_num, e2, oc);
      if (oc) atomicMin((long long *)first, (long long)ev_code(j, 8, 0));
      sc[j - 1] = cj;
      ss[j - 1] = sj;
      bool og = false;  // rotation of g, both from the old g_j
      const int64_t gj = sg[j - 1];
      const int64_t msj = subc(0, sj, og);
      sg[j - 1] = asr(mulw(gj, cj, og), df);
      sg[j] = asr(mulw(gj, msj, og), df);
      if (og) atomicMin((long long *)first, (long long)ev_code(j, 9, 0));
      col[j - 1] = tmp;  // h_jj = t_mp, h_{j+1,j} = 0
      col[j] = 0;
      if (lucky) {
        sh_breakdown = 1;
        sh_jstar = j;
        stop = 1;
      } else if (a.gtol >= 0) {
        const int64_t gn = sg[j] < 0 ? -sg[j] : sg[j];
        if (gn <= a.gtol) { sh_jstar = j; stop = 1; }
      }
    }
    if (blockIdx.x == 0) {
      for (int i = 0; i <= j; ++i) a.H[(size_t)i * m + (j - 1)] = col[i];
      a.c[j - 1] = sc[j - 1];
      a.s[j - 1] = ss[j - 1];
      a.g[j - 1] = sg[j - 1];
      a.g[j] = sg[j];
    }
    sh_steps = j;
    sh_stop = stop;
  };

  for (int j = 1; j <= m; ++j) {  // Arnoldi step j
    const int64_t *__restrict__ vj = a.V + (size_t)(j - 1) * a.npad;
    // ---- integer SpMV, then the preconditioner apply
    if (PRE != IGM_PRE_ILU0) {
      bool o1 = false, o2 = false;
#pragma unroll
      for (int k = 0; k < R; ++k) {  // padded rows: empty slices (or rows), unit diagonals
        const int64_t row = gt + k * T;
        int64_t z = cycle_spmv<BLOCK, MAP>(a, row, (int64_t)blockIdx.x * BLOCK + k * T, vj,
                                           (char *)smem + a.spmv_lds_off, o1);
        if (PRE == IGM_PRE_JACOBI) z = tdiv_diag(tdiv_diag(z, a.ldiag[row], o2), a.udiag[row], o2);
        w[k] = z;
      }
      note_event(o1, first, ev_code(j, 1, 0));
      note_event(o2, first, ev_code(j, 2, 0));
    } else {
      // z, y and u pass between workgroups through device-coherent stores
      // and loads; the two sweeps run block by block (igm_bsweep.hpp), and
      // three grid barriers per step separate the SpMV, the two sweeps and
      // the read-back of u. The blocks' progress words restart from zero in
      // every step (cleared before the barrier that follows the SpMV; the
      // previous step's sweeps ended at an earlier barrier).
      bool o1 = false, o2 = false, to = false;
#pragma unroll
      for (int k = 0; k < R; ++k) {
        const int64_t row = gt + k * T;
        const int64_t z = cycle_spmv<BLOCK, MAP>(a, row, (int64_t)blockIdx.x * BLOCK + k * T, vj,
                                                 (char *)smem + a.spmv_lds_off, o1);
        st_coh(a.zbuf + row, z);
      }
      for (int64_t i = gt; i < (int64_t)a.bsf.nb + a.bsb.nb; i += T) st_coh(a.bsf.prog + i * kLevStride, 0u);
      note_event(o1, first, ev_code(j, 1, 0));
      grid_barrier_coh(gs, ssh);
      char *slds = (char *)smem + a.sweep_lds_off;
      if (!ssh.abort) ilu_sweep<BLOCK>(a.bsf, (const int64_t *)a.zbuf, a.wbuf, slds, o2, to);
      grid_barrier_coh(gs, ssh);
      if (!ssh.abort) ilu_sweep<BLOCK>(a.bsb, (const int64_t *)a.wbuf, a.wbuf, slds, o2, to);
      if (to) __hip_atomic_store(&a.state->timeout, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      grid_barrier_coh(gs, ssh);
      note_event(o2, first, ev_code(j, 2, 0));
#pragma unroll
      for (int k = 0; k < R; ++k) w[k] = ld_coh(a.wbuf + gt + k * T);  // padded rows hold 0
    }
    IGM_TICK(0)
    // ---- modified Gram-Schmidt, i increasing. v_{i+1} is loaded
    // before waiting for the grid sum of (w, v_i) so its latency overlaps.
    // Earlier rotation i needs only h_{i+1,j}, so thread kGivens
    // applies rotation q-2 while wavefront 0 waits for reduction q.
    int64_t vv[R];
#pragma unroll
    for (int k = 0; k < R; ++k) vv[k] = a.V[gt + k * T];
    for (int i = 1; i <= j; ++i) {
      Acc acc;
      acc.zero();
      bool o = false;
#pragma unroll
      for (int k = 0; k < R; ++k) acc.add(mulw(asr(w[k], a.b_dot), vv[k], o));  // inner product: only w is shifted
      note_event(o, first, ev_code(j, 3, 2 * (i - 1)));
      int64_t vnext[R];
      if (i < j) {
        const int64_t *vi1 = a.V + (size_t)i * a.npad;
#pragma unroll
        for (int k = 0; k < R; ++k) vnext[k] = vi1[gt + k * T];
      }
      IGM_TICK(1)
      bool os = false;
      const int64_t h = grid_sum<BLOCK>(gs, acc, ssh, fin_dot, [&] {
        if (tid == kGivens && i >= 3) rotate(j, i - 2);
      }, os);
      IGM_TICK(2)
      if (os && tid == 0) atomicMin((long long *)first, (long long)ev_code(j, 3, 2 * (i - 1)));
      if (tid == kGivens) {
        col[i - 1] = h;
        if (i == 1) carry = h;
      }
      // update of w: only h is shifted
      const int64_t hs = asr(h, a.b_axpy);
      bool ou = false;
#pragma unroll
      for (int k = 0; k < R; ++k) w[k] = subc(w[k], asr(mulw(hs, vv[k], ou), df - a.b_axpy), ou);
      note_event(ou, first, ev_code(j, 3, 2 * (i - 1) + 1));
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
      for (int k = 0; k < R; ++k) acc.add(sqrc(asr(w[k], a.b_norm), o));
      note_event(o, first, ev_code(j, 4, 0));
      bool os = false;
      hn = grid_sum<BLOCK>(gs, acc, ssh, fin_norm, [&] {
        if (tid == kGivens && j >= 2) rotate(j, j - 1);
      }, os);
      if (os && tid == 0) atomicMin((long long *)first, (long long)ev_code(j, 4, 0));
    }
    IGM_TICK(3)
    // ---- normalisation v_{j+1} = w / h_{j+1,j}
    const int64_t den = asr(hn, a.b_div_den);
    lucky = den == 0;
    if (!lucky) {
      int64_t *__restrict__ vn = a.V + (size_t)j * a.npad;
      const int e = df - a.b_div_num - a.b_div_den;
      bool ov = false;
#pragma unroll
      for (int k = 0; k < R; ++k) st_coh(vn + gt + k * T, normalize_elem(w[k], den, a.b_div_num, e, ov));
      note_event(ov, first, ev_code(j, 5, 0));
    }
    IGM_TICK(4)
    // v_{j+1} becomes visible to every workgroup; the new rotation and the
    // update of g and H (thread kGivens) run while wavefront 0 waits
    grid_barrier_coh(gs, ssh, [&] {
      if (tid == kGivens) givens(j);
    });
    IGM_TICK(6)
    if (sh_stop || ssh.abort) break;
  }
  // publish H, c, s, g of the last step written during the last barrier
  grid_barrier(gs, ssh, no_side);
  IGM_TICK(6)

  if (tid == 0 && blockIdx.x == 0) {
    a.state->jstar = sh_jstar;
    a.state->breakdown = sh_breakdown;
    a.state->steps = sh_steps;
    ph[7] = wall_clock64() - t_start;
    for (int k = 0; k < 8; ++k) a.state->phase[k] = ph[k];
  }
#undef IGM_TICK
  if (!a.update || ssh.abort) return;
  // ---- closing least-squares step and x += gamma x^(k): each thread updates its own rows
  if (tid == 0) {
    const int64_t ev = __hip_atomic_load(first, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    sh_update = (ev == kNoEvent && sh_jstar > 0);
    if (sh_update) {
      const int js = sh_jstar;
      const double rho = a.scal[1];
      for (int i = js - 1; i >= 0; --i) {  // back substitution, inner sum k increasing
        double acc = 0.0;
        for (int k = i + 1; k < js; ++k) acc = acc + ldexp((double)a.H[(size_t)i * m + k], -df) * sy[k];
        sy[i] = (ldexp((double)sg[i], -df) - acc) / ldexp((double)a.H[(size_t)i * m + i], -df);
      }
      for (int i = 0; i < js; ++i) sy[i] = rho * sy[i];
    }
  }
  __syncthreads();
  if (!sh_update) return;
  const int js = sh_jstar;
  const double gamma = a.scal[0];
#pragma unroll
  for (int k = 0; k < R; ++k) {
    const int64_t row = gt + k * T;
    if (row < a.n) {
      double acc = 0.0;
      for (int i = 0; i < js; ++i) acc = acc + sy[i] * ldexp((double)a.V[(size_t)i * a.npad + row], -df);
      a.x[row] = a.x[row] + gamma * (a.cscale ? acc / a.cscale[row] : acc);
    }
  }
}

// The kernel for a workgroup size, rows per thread and preconditioner, with
// SpMV mapping MAP (nullptr for a shape that is not built). Each mapping's
// kernels are instantiated in a source file of their own.
template <int MAP>
const void *cycle_kernel_for(int block, int R, int pre) {
#define IGM_K(BB, RR)                                                           \
  if (block == BB && R == RR) {                                                 \
    if (pre == IGM_PRE_NONE) return (const void *)&k_cycle<BB, RR, 0, MAP>;     \
    if (pre == IGM_PRE_JACOBI) return (const void *)&k_cycle<BB, RR, 1, MAP>;   \
    return (const void *)&k_cycle<BB, RR, 2, MAP>;                              \
  }
  IGM_K(1024, 1)
  IGM_K(1024, 2)
  IGM_K(1024, 4)
  IGM_K(512, 1)
  IGM_K(512, 2)
  IGM_K(512, 4)
  IGM_K(512, 8)
  IGM_K(512, 16)
#undef IGM_K
  return nullptr;
}

}  // namespace igm
