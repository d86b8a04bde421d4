// Host setup of a system: initial scaling (Sec. III), integer matrices
// (Sec. IV-B), integer ILU(0)/Jacobi factors (Sec. VI-A), level sets of the
// triangular sweeps and the SELL-64 layout of the integer matrices.
//
// Every FP64 step follows a fixed operation order with no contraction, so the
// products are reproducible bit for bit.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <algorithm>

#include "igm_internal.hpp"

namespace igm {

static bool shift_ok(int32_t b, int32_t hi) { return b >= 0 && b <= hi; }

igm_status check_policy(const igm_policy &p) {
  if (p.df < 1 || p.df > 62 || p.alpha_a < 0 || p.alpha_a > 62) return IGM_ERR_ARG;
  if (p.m < 1 || p.m > 1024 || p.s_terms < 0 || p.s_terms > kMaxTerms - 1) return IGM_ERR_ARG;
  if (p.precond < IGM_PRE_NONE || p.precond > IGM_PRE_ILU0) return IGM_ERR_ARG;
  if (!shift_ok(p.b_dot, p.df) || !shift_ok(p.b_axpy, p.df) || !shift_ok(p.b_rot, p.df)) return IGM_ERR_ARG;
  if (!shift_ok(p.b_norm, p.df) || !shift_ok(p.b_tmp, p.df)) return IGM_ERR_ARG;
  if (!shift_ok(p.b_div_num, 62) || !shift_ok(p.b_div_den, 62)) return IGM_ERR_ARG;
  if (!shift_ok(p.b_cs_num, 62) || !shift_ok(p.b_cs_den, 62)) return IGM_ERR_ARG;
  if (p.max_refine < 0 || !(p.tol >= 0.0) || p.grid_blocks < 0) return IGM_ERR_ARG;
  if (p.phase_clock < 0 || p.phase_clock > 1) return IGM_ERR_ARG;
  return IGM_OK;
}

// C cast to int64 with a range check (|y| < 2^63).
static inline int64_t cast_i64(double y, bool &bad) {
  if (!(y >= -9223372036854775808.0 && y < 9223372036854775808.0)) {
    bad = true;
    return 0;
  }
  return (int64_t)y;
}

// eq. (eq3): dhat_i = max_j |ahat_ij| / 2^alpha_a; eq. (eq1): A = Dhat^-1 Ahat,
// b = Dhat^-1 bhat, one division per entry.
static igm_status scale_rows(int64_t n, const std::vector<int64_t> &rp, const std::vector<double> &ahat,
                             const std::vector<double> &bhat, int alpha, HostSetup &h) {
  h.dhat.resize(n);
  h.a.resize(ahat.size());
  h.b.resize(n);
  for (int64_t i = 0; i < n; ++i) {
    double mu = 0.0;
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) mu = std::max(mu, fabs(ahat[e]));
    if (mu == 0.0) return IGM_ERR_SINGULAR_ROW;
    double d = ldexp(mu, -alpha);
    if (d == 0.0 || !isfinite(d)) return IGM_ERR_RANGE;
    h.dhat[i] = d;
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) h.a[e] = ahat[e] / d;
    h.b[i] = bhat[i] / d;
  }
  return IGM_OK;
}

// Sec. IV-B: A_0 = trunc(A); remainders R_l give alpha_l = alpha_a -
// floor(log2 max|R_l|) (eq. (alpha1)) and A_l = trunc(2^alpha_l R_l).
static igm_status split_terms(const igm_policy &p, HostSetup &h) {
  size_t nnz = h.a.size();
  bool bad = false;
  std::vector<double> rem(nnz);
  h.abar.assign(1, std::vector<int64_t>(nnz));
  h.alpha[0] = 0;
  for (size_t e = 0; e < nnz; ++e) {
    int64_t t = cast_i64(h.a[e], bad);
    h.abar[0][e] = t;
    rem[e] = h.a[e] - (double)t;
  }
  h.nterms = 1;
  for (int l = 1; l <= p.s_terms; ++l) {
    double mu = 0.0;
    for (size_t e = 0; e < nnz; ++e) mu = std::max(mu, fabs(rem[e]));
    if (mu == 0.0) break;
    int ex = 0;
    frexp(mu, &ex);
    int al = p.alpha_a - (ex - 1);
    if (al > 1070) break;
    h.alpha[l] = al;
    h.abar.emplace_back(nnz);
    for (size_t e = 0; e < nnz; ++e) {
      double t = ldexp(rem[e], al);
      int64_t q = cast_i64(t, bad);
      h.abar[l][e] = q;
      rem[e] = ldexp(t - (double)q, -al);
    }
    h.nterms = l + 1;
  }
  return bad ? IGM_ERR_RANGE : IGM_OK;
}

// FP64 ILU(0) on the pattern, row-oriented: for row i and each k < i of the
// row (increasing), l_ik = a_ik / u_kk, then a_ij -= l_ik u_kj for the j > k
// of row k that also occur in row i.
static igm_status ilu0_fp(int64_t n, const std::vector<int64_t> &rp, const std::vector<int32_t> &col,
                          HostSetup &h) {
  h.lu = h.a;
  std::vector<int64_t> where(n, -1);
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) where[col[e]] = e;
    for (int64_t e = rp[i]; e < rp[i + 1] && col[e] < i; ++e) {
      int64_t k = col[e];
      double piv = h.lu[h.diag_pos[k]];
      if (piv == 0.0) return IGM_ERR_ZERO_PIVOT;
      double lik = h.lu[e] / piv;
      h.lu[e] = lik;
      for (int64_t f = h.diag_pos[k] + 1; f < rp[k + 1]; ++f) {
        int64_t t = where[col[f]];
        if (t >= 0) h.lu[t] = h.lu[t] - lik * h.lu[f];
      }
    }
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) where[col[e]] = -1;
    if (h.lu[h.diag_pos[i]] == 0.0) return IGM_ERR_ZERO_PIVOT;
  }
  return IGM_OK;
}

// eqs. (dl), (dl2), (l1), (u1): Lbar = trunc(L |D|^1/2), Ubar = trunc(sgn(D)
// |D|^1/2 U) with U unit upper (stored entries divided by the pivot).
static igm_status cast_factors(int64_t n, const std::vector<int64_t> &rp, const std::vector<int32_t> &col,
                               const std::vector<double> &piv, bool offdiag, HostSetup &h) {
  bool bad = false;
  h.ldiag.resize(n);
  h.udiag.resize(n);
  std::vector<double> sq(n);
  for (int64_t i = 0; i < n; ++i) {
    if (piv[i] == 0.0 || !isfinite(piv[i])) return IGM_ERR_ZERO_PIVOT;
    sq[i] = sqrt(fabs(piv[i]));
  }
  h.lptr.assign(n + 1, 0);
  h.uptr.assign(n + 1, 0);
  h.lcol.clear(); h.ucol.clear(); h.lval.clear(); h.uval.clear();
  for (int64_t i = 0; i < n; ++i) {
    double su = piv[i] < 0.0 ? -sq[i] : sq[i];
    h.ldiag[i] = cast_i64(sq[i], bad);
    h.udiag[i] = cast_i64(su, bad);
    if (bad) return IGM_ERR_RANGE;
    if (h.ldiag[i] == 0 || h.udiag[i] == 0) return IGM_ERR_ZERO_PIVOT;
    if (offdiag) {
      for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
        int32_t j = col[e];
        if (j < i) {
          h.lcol.push_back(j);
          h.lval.push_back(cast_i64(h.lu[e] * sq[j], bad));
        } else if (j > i) {
          h.ucol.push_back(j);
          h.uval.push_back(cast_i64(su * (h.lu[e] / piv[i]), bad));
        }
      }
    }
    h.lptr[i + 1] = (int64_t)h.lcol.size();
    h.uptr[i + 1] = (int64_t)h.ucol.size();
    if (bad) return IGM_ERR_RANGE;
  }
  return IGM_OK;
}

// Level sets: a row's forward level is one more than the largest level of the
// rows its strict lower part reads (rows in increasing order); backward levels
// likewise on the strict upper part in decreasing order.
static void level_sets(int64_t n, HostSetup &h) {
  std::vector<int32_t> lev(n);
  auto group = [&](std::vector<int32_t> &ptr, std::vector<int32_t> &rows, int32_t nlev) {
    ptr.assign(nlev + 1, 0);
    for (int64_t i = 0; i < n; ++i) ptr[lev[i] + 1]++;
    for (int32_t k = 0; k < nlev; ++k) ptr[k + 1] += ptr[k];
    rows.assign(n, 0);
    std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
    for (int64_t i = 0; i < n; ++i) rows[fill[lev[i]]++] = (int32_t)i;
  };
  int32_t nlev = 0;
  for (int64_t i = 0; i < n; ++i) {
    int32_t l = 0;
    for (int64_t e = h.lptr[i]; e < h.lptr[i + 1]; ++e) l = std::max(l, lev[h.lcol[e]] + 1);
    lev[i] = l;
    nlev = std::max(nlev, l + 1);
  }
  group(h.flev_ptr, h.flev_rows, nlev);
  nlev = 0;
  for (int64_t i = n - 1; i >= 0; --i) {
    int32_t l = 0;
    for (int64_t e = h.uptr[i]; e < h.uptr[i + 1]; ++e) l = std::max(l, lev[h.ucol[e]] + 1);
    lev[i] = l;
    nlev = std::max(nlev, l + 1);
  }
  group(h.blev_ptr, h.blev_rows, nlev);
}

// SELL-64: rows in slices of 64, each slice stored column-major with the width
// of its longest row; padding entries have value 0 and point at the row itself.
static void build_sell(int64_t n, const std::vector<int64_t> &rp, const std::vector<int32_t> &col, HostSetup &h) {
  int64_t ns = (n + kSlice - 1) / kSlice;
  h.nslices = ns;
  h.sell_off.assign(ns + 1, 0);
  h.sell_w.assign(ns, 0);
  for (int64_t s = 0; s < ns; ++s) {
    int64_t w = 0;
    for (int64_t i = s * kSlice; i < std::min(n, (s + 1) * kSlice); ++i) w = std::max(w, rp[i + 1] - rp[i]);
    h.sell_w[s] = (int32_t)w;
    h.sell_off[s + 1] = h.sell_off[s] + w * kSlice;
  }
  int64_t tot = h.sell_off[ns];
  h.sell_col.assign(tot, 0);
  h.sell_val.assign(h.nterms, std::vector<int64_t>(tot, 0));
  for (int64_t s = 0; s < ns; ++s) {
    for (int lane = 0; lane < kSlice; ++lane) {
      int64_t i = s * kSlice + lane;
      for (int64_t k = 0; k < h.sell_w[s]; ++k) {
        int64_t pos = h.sell_off[s] + k * kSlice + lane;
        int64_t e = (i < n) ? rp[i] + k : -1;
        if (i < n && e < rp[i + 1]) {
          h.sell_col[pos] = col[e];
          for (int l = 0; l < h.nterms; ++l) h.sell_val[l][pos] = h.abar[l][e];
        } else {
          h.sell_col[pos] = (int32_t)std::min<int64_t>(i, n - 1);
        }
      }
    }
  }
}

igm_status host_setup(int64_t n, const std::vector<int64_t> &rp, const std::vector<int32_t> &col,
                      const std::vector<double> &ahat, const std::vector<double> &bhat, const igm_policy &pol,
                      HostSetup &h) {
  h = HostSetup();
  igm_status st = scale_rows(n, rp, ahat, bhat, pol.alpha_a, h);
  if (st != IGM_OK) return st;
  st = split_terms(pol, h);
  if (st != IGM_OK) return st;
  h.diag_pos.assign(n, -1);
  for (int64_t i = 0; i < n; ++i)
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e)
      if (col[e] == i) h.diag_pos[i] = e;
  if (pol.precond != IGM_PRE_NONE) {
    for (int64_t i = 0; i < n; ++i)
      if (h.diag_pos[i] < 0) return IGM_ERR_ZERO_PIVOT;
    std::vector<double> piv(n);
    if (pol.precond == IGM_PRE_ILU0) {
      st = ilu0_fp(n, rp, col, h);
      if (st != IGM_OK) return st;
      for (int64_t i = 0; i < n; ++i) piv[i] = h.lu[h.diag_pos[i]];
    } else {
      for (int64_t i = 0; i < n; ++i) piv[i] = h.a[h.diag_pos[i]];
    }
    st = cast_factors(n, rp, col, piv, pol.precond == IGM_PRE_ILU0, h);
    if (st != IGM_OK) return st;
    level_sets(n, h);
  }
  build_sell(n, rp, col, h);
  return IGM_OK;
}

int32_t sweep_threads(int block, int grid, int32_t max_level) {
  if (const char *e = std::getenv("IGM_SWEEP_THREADS")) {
    const int v = std::atoi(e);
    if (v >= 64 && v % 64 == 0) return std::min(v, block);
  }
  const int64_t want = (4 * (int64_t)max_level + grid - 1) / std::max(grid, 1);
  const int64_t t = (want + 63) / 64 * 64;
  return (int32_t)std::max<int64_t>(64, std::min<int64_t>(t, block));
}

int32_t max_level_rows(const HostSetup &h) {
  int32_t mx = 0;
  for (size_t L = 0; L + 1 < h.flev_ptr.size(); ++L) mx = std::max(mx, h.flev_ptr[L + 1] - h.flev_ptr[L]);
  for (size_t L = 0; L + 1 < h.blev_ptr.size(); ++L) mx = std::max(mx, h.blev_ptr[L + 1] - h.blev_ptr[L]);
  return mx;
}

// CSR and right-hand side checks shared by every entry point that takes a
// host system: rows and columns in range, columns strictly increasing within a
// row, finite values.
igm_status validate_csr(int64_t n, const int64_t *rp, const int32_t *col, const double *val, const double *b) {
  if (n < 1 || n >= ((int64_t)1 << 31) || !rp || !col || !val || !b) return IGM_ERR_ARG;
  if (rp[0] != 0) return IGM_ERR_ARG;
  for (int64_t i = 0; i < n; ++i) {
    if (rp[i + 1] < rp[i]) return IGM_ERR_ARG;
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
      if (col[e] < 0 || col[e] >= n) return IGM_ERR_ARG;
      if (e > rp[i] && col[e] <= col[e - 1]) return IGM_ERR_ARG;
      if (!isfinite(val[e])) return IGM_ERR_ARG;
    }
    if (!isfinite(b[i])) return IGM_ERR_ARG;
  }
  return IGM_OK;
}

}  // namespace igm
