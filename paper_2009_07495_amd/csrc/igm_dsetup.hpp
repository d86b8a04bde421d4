// Setup of a served request on the device, by the request's team of
// workgroups, from its inputs (ahat, bhat) and the structure the host made
// (host_structure in igm_setup.cpp). Every value is computed with the same
// operations in the same order as the host setup (igm_setup.cpp), so the
// results are the same bits, and the first error is the one the host setup
// would report:
//   1. eq. (eq3) / (eq1): dhat_i = max_j |ahat_ij| 2^-alpha_a; a = ahat / dhat_i,
//      b = bhat / dhat_i (IGM_ERR_SINGULAR_ROW, IGM_ERR_RANGE: the first row);
//      two-sided, eq. (eq2): s_i = sqrt(dhat_i) for every row first, then
//      a_ij = ahat_ij / (s_i s_j), b_i = bhat_i / s_i;
//   2. eq. (A) with one term: Abar = trunc(A), written straight into the
//      SELL-64 layout (IGM_ERR_RANGE);
//   3. Sec. VI-A: the FP64 ILU(0) of A in place (rows of one level of the
//      strict lower pattern in parallel, levels in order, each row's updates in
//      CSR order; the position of column j in row i by binary search), in the
//      basis array, which the solve overwrites later (IGM_ERR_ZERO_PIVOT);
//   4. Sec. VI: the cast diagonals |u_ii|^(1/2) (sign on the upper one) and,
//      for ILU(0), the integer factors with their FP64 copies
//      (IGM_ERR_ZERO_PIVOT before any cast, then IGM_ERR_RANGE or
//      IGM_ERR_ZERO_PIVOT of the first row).
#pragma once

#include "igm_team.hpp"

namespace igm {

// FP64 -> int64 truncation with the range test of the host's cast_i64.
__device__ __forceinline__ int64_t dcast_i64(double y, bool &bad) {
  if (!(y >= -9223372036854775808.0 && y < 9223372036854775808.0)) {
    bad = true;
    return 0;
  }
  return (int64_t)y;
}

// Entry of column j in row i (columns sorted), or -1.
__device__ __forceinline__ int64_t find_col(const int32_t *__restrict__ col, int64_t lo, int64_t hi, int32_t j) {
  while (lo < hi) {
    const int64_t mid = (lo + hi) >> 1;
    const int32_t c = col[mid];
    if (c == j) return mid;
    if (c < j) lo = mid + 1;
    else hi = mid;
  }
  return -1;
}

// Returns IGM_OK or the first error. g0, TB: this thread's first row slot and
// the team's thread count. Every thread of every member calls it.
template <int BLOCK>
__device__ igm_status device_setup(Team &tm, TeamShared &tsh, const BatchSys &S, int64_t g0, int64_t TB) {
  const int64_t n = S.n;
  const int64_t *__restrict__ rp = S.row_ptr;
  const int32_t *__restrict__ col = S.col;
  double *a = const_cast<double *>(S.a);
  double *b = const_cast<double *>(S.b);
  // first error: (phase << 56) | (row << 8) | -status; the smallest code wins
  unsigned long long err = ~0ull;
  auto fail = [&](int phase, int64_t row, igm_status st) {
    const unsigned long long c = ((unsigned long long)phase << 56) | ((unsigned long long)row << 8) |
                                 (unsigned long long)(-(int)st);
    if (c < err) err = c;
  };
  auto team_err = [&]() -> igm_status {
    unsigned long long v[1] = {~err};
    team_reduce<BLOCK, 1, true>(tm, tsh, v);
    const unsigned long long c = ~v[0];
    return c == ~0ull ? IGM_OK : (igm_status)(-(int)(c & 0xff));
  };
  igm_status st;

  // 1. scaling
  for (int64_t i = g0; i < n; i += TB) {
    double mu = 0.0;
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
      const double v = fabs(S.ahat[e]);
      mu = mu < v ? v : mu;
    }
    if (mu == 0.0) { fail(1, i, IGM_ERR_SINGULAR_ROW); continue; }
    const double d = ldexp(mu, -S.alpha_a);
    if (d == 0.0 || !isfinite(d)) { fail(1, i, IGM_ERR_RANGE); continue; }
    if (S.cscale) {
      const_cast<double *>(S.cscale)[i] = sqrt(d);
      continue;
    }
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) a[e] = S.ahat[e] / d;
    b[i] = S.bhat[i] / d;
  }
  if ((st = team_err()) != IGM_OK) return st;
  team_barrier(tm, tsh);
  if (S.cscale) {  // every s_j is in place
    const double *__restrict__ cs = S.cscale;
    for (int64_t i = g0; i < n; i += TB) {
      for (int64_t e = rp[i]; e < rp[i + 1]; ++e) a[e] = S.ahat[e] / (cs[i] * cs[col[e]]);
      b[i] = S.bhat[i] / cs[i];
    }
    team_barrier(tm, tsh);
  }

  // 2. the integer matrix in the SELL-64 layout: thread t of the team takes
  // lane t % 64 of slices t / 64, t / 64 + TB / 64, ...
  {
    int64_t *sv = const_cast<int64_t *>(S.sell_val[0]);
    const int64_t ns = (n + kSlice - 1) / kSlice;
    const int lane = (int)(g0 % kSlice);
    bool bad = false;
    for (int64_t sl = g0 / kSlice; sl < ns; sl += TB / kSlice) {
      const int64_t i = sl * kSlice + lane, off = S.sell_off[sl];
      const int w = S.sell_w[sl];
      const int64_t lo = i < n ? rp[i] : 0, len = i < n ? rp[i + 1] - lo : 0;
      for (int k = 0; k < w; ++k) sv[off + (int64_t)k * kSlice + lane] = k < len ? dcast_i64(a[lo + k], bad) : 0;
    }
    if (bad) fail(2, 0, IGM_ERR_RANGE);
  }
  if ((st = team_err()) != IGM_OK) return st;
  if (S.precond == IGM_PRE_NONE) {
    team_barrier(tm, tsh);
    return IGM_OK;
  }

  // a preconditioner needs every diagonal entry
  for (int64_t i = g0; i < n; i += TB)
    if (S.diag_pos[i] < 0) fail(3, i, IGM_ERR_ZERO_PIVOT);
  if ((st = team_err()) != IGM_OK) return st;

  // 3. FP64 ILU(0) in place, in the basis array
  const bool ilu = S.precond == IGM_PRE_ILU0;
  double *lu = ilu ? (double *)S.V : a;
  if (ilu) {
    for (int64_t e = g0; e < rp[n]; e += TB) lu[e] = a[e];
    team_barrier(tm, tsh);
    bool zero = false;
    for (int L = 0; L < S.nflev; ++L) {
      for (int64_t q = S.flev_ptr[L] + g0; q < S.flev_ptr[L + 1]; q += TB) {
        const int64_t i = S.flev_rows[q];
        const int64_t lo = rp[i], hi = rp[i + 1];
        bool ok = true;
        for (int64_t e = lo; e < hi && col[e] < i; ++e) {
          const int64_t k = col[e];
          const int64_t dk = S.diag_pos[k];
          const double piv = lu[dk];
          if (piv == 0.0) { ok = false; break; }
          const double lik = lu[e] / piv;
          lu[e] = lik;
          for (int64_t f = dk + 1; f < rp[k + 1]; ++f) {
            const int64_t t = find_col(col, lo, hi, col[f]);
            if (t >= 0) lu[t] = lu[t] - lik * lu[f];
          }
        }
        if (!ok || lu[S.diag_pos[i]] == 0.0) zero = true;
      }
      team_barrier(tm, tsh);  // the level's rows for the next levels
    }
    if (zero) fail(4, 0, IGM_ERR_ZERO_PIVOT);
    if ((st = team_err()) != IGM_OK) return st;
  }

  // 4. casts: every pivot first, then the rows in order
  double *sq = ilu ? S.fbuf : nullptr;  // |u_jj|^(1/2) of every row, read across rows
  bool zero = false;
  for (int64_t i = g0; i < n; i += TB) {
    const double piv = lu[S.diag_pos[i]];
    if (piv == 0.0 || !isfinite(piv)) zero = true;
    else if (ilu) sq[i] = sqrt(fabs(piv));
  }
  if (zero) fail(5, 0, IGM_ERR_ZERO_PIVOT);
  if ((st = team_err()) != IGM_OK) return st;
  if (ilu) team_barrier(tm, tsh);
  int64_t *ldiag = const_cast<int64_t *>(S.ldiag), *udiag = const_cast<int64_t *>(S.udiag);
  for (int64_t i = g0; i < n; i += TB) {
    const double piv = lu[S.diag_pos[i]];
    const double s = ilu ? sq[i] : sqrt(fabs(piv));
    const double su = piv < 0.0 ? -s : s;
    bool bad = false;
    ldiag[i] = dcast_i64(s, bad);
    udiag[i] = dcast_i64(su, bad);
    if (bad) { fail(6, i, IGM_ERR_RANGE); continue; }
    if (ldiag[i] == 0 || udiag[i] == 0) { fail(6, i, IGM_ERR_ZERO_PIVOT); continue; }
    if (ilu) {
      int64_t pl = S.lptr[i], pu = S.uptr[i];
      int64_t *lval = const_cast<int64_t *>(S.lval), *uval = const_cast<int64_t *>(S.uval);
      double *lf = const_cast<double *>(S.lvalf), *uf = const_cast<double *>(S.uvalf);
      for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
        const int32_t j = col[e];
        if (j < i) {
          const int64_t v = dcast_i64(lu[e] * sq[j], bad);
          lval[pl] = v;
          lf[pl++] = (double)v;
        } else if (j > i) {
          const int64_t v = dcast_i64(su * (lu[e] / piv), bad);
          uval[pu] = v;
          uf[pu++] = (double)v;
        }
      }
      if (bad) fail(6, i, IGM_ERR_RANGE);
    }
  }
  if ((st = team_err()) != IGM_OK) return st;
  team_barrier(tm, tsh);
  return IGM_OK;
}

}  // namespace igm
