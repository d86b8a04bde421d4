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
#include "igm_par.hpp"

namespace igm {

namespace {

std::atomic<int> g_setups{0};

// First error in row order over the chunks of a parallel pass: each chunk
// records its first failing row (chunks are in row order, so the smallest
// recorded row is the one the serial loop would have stopped at).
struct FirstError {
  std::vector<int64_t> row;
  std::vector<igm_status> st;
  explicit FirstError(int nt) : row(std::max(nt, 1), INT64_MAX), st(std::max(nt, 1), IGM_OK) {}
  void set(int c, int64_t r, igm_status s) {
    if (r < row[c]) {
      row[c] = r;
      st[c] = s;
    }
  }
  igm_status first() const {
    int64_t best = INT64_MAX;
    igm_status s = IGM_OK;
    for (size_t c = 0; c < row.size(); ++c)
      if (row[c] < best) {
        best = row[c];
        s = st[c];
      }
    return s;
  }
};

}  // namespace

SetupRegion::SetupRegion() { g_setups.fetch_add(1); }
SetupRegion::~SetupRegion() { g_setups.fetch_sub(1); }

int setup_thread_count() {
  int hw = 0;
  if (const char *e = std::getenv("IGM_SETUP_THREADS")) hw = std::atoi(e);
  if (hw < 1 || hw > 64) {
    const unsigned c = std::thread::hardware_concurrency();
    hw = c ? (int)std::min(c, 16u) : 1;
  }
  return std::max(1, hw / std::max(1, g_setups.load()));
}

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
  if (p.shift_retry < 0 || p.shift_retry > 64) return IGM_ERR_ARG;
  if (p.two_sided < 0 || p.two_sided > 1) return IGM_ERR_ARG;
  if (p.gauss_seidel < 0 || p.gauss_seidel > 1) return IGM_ERR_ARG;
  if (p.gauss_seidel && p.precond != IGM_PRE_ILU0) return IGM_ERR_ARG;
  if (p.sweep_rows < 0 || p.sweep_rows % 64 != 0 || p.sweep_rows > (1 << 20)) return IGM_ERR_ARG;
  if (p.sweep_lanes != 0 && p.sweep_lanes != 4 && p.sweep_lanes != 8 && p.sweep_lanes != 16) return IGM_ERR_ARG;
  if (p.s_rule < 0 || p.s_rule > 1) return IGM_ERR_ARG;
  if (p.spmv_lanes < -1 || p.spmv_lanes > 64 || (p.spmv_lanes > 2 && (p.spmv_lanes & (p.spmv_lanes - 1)) != 0))
    return IGM_ERR_ARG;  // -1, 0, 1, 2, or 4, 8, 16, 32, 64 lanes per row
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
// Two-sided (eq. (eq2), D1 = D2 = Dhat^(1/2)): s_i = sqrt(dhat_i), a_ij =
// ahat_ij / (s_i s_j), b_i = bhat_i / s_i; s is kept in h.cscale.
static igm_status scale_rows(int nt, int64_t n, const hvec<int64_t> &rp, const hvec<int32_t> &col,
                             const hvec<double> &ahat, const hvec<double> &bhat, int alpha, bool two_sided,
                             HostSetup &h) {
  h.dhat.resize(n);
  h.a.resize(ahat.size());
  h.b.resize(n);
  if (two_sided) h.cscale.resize(n);
  FirstError fe(nt);
  par_ranges(nt, n, [&](int c, int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi; ++i) {
      double mu = 0.0;
      for (int64_t e = rp[i]; e < rp[i + 1]; ++e) mu = std::max(mu, fabs(ahat[e]));
      if (mu == 0.0) return fe.set(c, i, IGM_ERR_SINGULAR_ROW);
      double d = ldexp(mu, -alpha);
      if (d == 0.0 || !isfinite(d)) return fe.set(c, i, IGM_ERR_RANGE);
      h.dhat[i] = d;
      if (two_sided) {
        h.cscale[i] = sqrt(d);
        continue;
      }
      for (int64_t e = rp[i]; e < rp[i + 1]; ++e) h.a[e] = ahat[e] / d;
      h.b[i] = bhat[i] / d;
    }
  });
  const igm_status st = fe.first();
  if (st != IGM_OK || !two_sided) return st;
  par_ranges(nt, n, [&](int, int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi; ++i) {
      for (int64_t e = rp[i]; e < rp[i + 1]; ++e) h.a[e] = ahat[e] / (h.cscale[i] * h.cscale[col[e]]);
      h.b[i] = bhat[i] / h.cscale[i];
    }
  });
  return IGM_OK;
}

// Sec. IV-B: A_0 = trunc(A); remainders R_l give alpha_l = alpha_a -
// floor(log2 max|R_l|) (eq. (alpha1)) and A_l = trunc(2^alpha_l R_l).
static igm_status split_terms(int nt, const igm_policy &p, HostSetup &h) {
  const int64_t nnz = (int64_t)h.a.size();
  std::atomic<bool> bad{false};
  // the remainders are needed only for terms beyond A_0
  hvec<double> rem(p.s_terms > 0 ? nnz : 0);
  h.abar.clear();
  h.abar.emplace_back(nnz);  // not assign(1, ...): that copies a whole array on one thread
  h.alpha[0] = 0;
  par_ranges(nt, nnz, [&](int, int64_t lo, int64_t hi) {
    bool b = false;
    for (int64_t e = lo; e < hi; ++e) {
      int64_t t = cast_i64(h.a[e], b);
      h.abar[0][e] = t;
      if (p.s_terms > 0) rem[e] = h.a[e] - (double)t;
    }
    if (b) bad = true;
  });
  h.nterms = 1;
  for (int l = 1; l <= p.s_terms; ++l) {
    std::vector<double> cmax(std::max(nt, 1), 0.0);  // the maximum is the same in any order
    par_ranges(nt, nnz, [&](int c, int64_t lo, int64_t hi) {
      double mu = 0.0;
      for (int64_t e = lo; e < hi; ++e) mu = std::max(mu, fabs(rem[e]));
      cmax[c] = mu;
    });
    double mu = 0.0;
    for (double v : cmax) mu = std::max(mu, v);
    if (mu == 0.0) break;
    int ex = 0;
    frexp(mu, &ex);
    int al = p.alpha_a - (ex - 1);
    if (al > 1070) break;
    h.alpha[l] = al;
    h.abar.emplace_back(nnz);
    hvec<int64_t> &q_l = h.abar[l];
    par_ranges(nt, nnz, [&](int, int64_t lo, int64_t hi) {
      bool b = false;
      for (int64_t e = lo; e < hi; ++e) {
        double t = ldexp(rem[e], al);
        int64_t q = cast_i64(t, b);
        q_l[e] = q;
        rem[e] = ldexp(t - (double)q, -al);
      }
      if (b) bad = true;
    });
    h.nterms = l + 1;
  }
  return bad ? IGM_ERR_RANGE : IGM_OK;
}

// FP64 ILU(0) on the pattern, row-oriented: for row i and each k < i of the
// row (increasing), l_ik = a_ik / u_kk, then a_ij -= l_ik u_kj for the j > k
// of row k that also occur in row i. Row i changes only its own entries and
// reads rows k < i of its strict lower part, so the rows of one level set of
// that part (every row one level above the rows it reads) are independent:
// threads share each level, in level order, with the same operations per row.
static igm_status ilu0_fp(int nt, int64_t n, const hvec<int64_t> &rp, const hvec<int32_t> &col,
                          HostSetup &h) {
  const int64_t nnz = rp[n];
  h.lu.resize(nnz);
  par_ranges(nt, nnz, [&](int, int64_t lo, int64_t hi) { std::copy(h.a.begin() + lo, h.a.begin() + hi, h.lu.begin() + lo); });
  // one row: returns false on a zero pivot
  auto row_ilu = [&](int64_t i, std::vector<int64_t> &where) {
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) where[col[e]] = e;
    bool ok = true;
    for (int64_t e = rp[i]; e < rp[i + 1] && col[e] < i; ++e) {
      int64_t k = col[e];
      double piv = h.lu[h.diag_pos[k]];
      if (piv == 0.0) { ok = false; break; }
      double lik = h.lu[e] / piv;
      h.lu[e] = lik;
      for (int64_t f = h.diag_pos[k] + 1; f < rp[k + 1]; ++f) {
        int64_t t = where[col[f]];
        if (t >= 0) h.lu[t] = h.lu[t] - lik * h.lu[f];
      }
    }
    for (int64_t e = rp[i]; e < rp[i + 1]; ++e) where[col[e]] = -1;
    return ok && h.lu[h.diag_pos[i]] != 0.0;
  };
  if (nt <= 1 || n < 32768) {
    std::vector<int64_t> where(n, -1);
    for (int64_t i = 0; i < n; ++i)
      if (!row_ilu(i, where)) return IGM_ERR_ZERO_PIVOT;
    return IGM_OK;
  }
  // level sets of the strict lower pattern, rows increasing inside a level
  std::vector<int32_t> lev(n);
  int32_t nlev = 0;
  for (int64_t i = 0; i < n; ++i) {
    int32_t l = 0;
    for (int64_t e = rp[i]; e < rp[i + 1] && col[e] < i; ++e) l = std::max(l, lev[col[e]] + 1);
    lev[i] = l;
    nlev = std::max(nlev, l + 1);
  }
  std::vector<int64_t> ptr(nlev + 1, 0);
  for (int64_t i = 0; i < n; ++i) ptr[lev[i] + 1]++;
  for (int32_t k = 0; k < nlev; ++k) ptr[k + 1] += ptr[k];
  std::vector<int32_t> rows(n);
  {
    std::vector<int64_t> fill(ptr.begin(), ptr.end() - 1);
    for (int64_t i = 0; i < n; ++i) rows[fill[lev[i]]++] = (int32_t)i;
  }
  std::atomic<int32_t> zero_level{INT32_MAX};  // first level with a zero pivot
  SpinBarrier bar(nt);
  auto work = [&](int t) {
    std::vector<int64_t> where(n, -1);
    for (int32_t L = 0; L < nlev; ++L) {
      const int64_t lo = ptr[L], cnt = ptr[L + 1] - lo, per = (cnt + nt - 1) / nt;
      const int64_t q0 = lo + t * per, q1 = std::min(lo + cnt, q0 + per);
      for (int64_t q = q0; q < q1; ++q)
        if (!row_ilu(rows[q], where)) {
          int32_t z = zero_level.load();
          while (L < z && !zero_level.compare_exchange_weak(z, L)) {
          }
        }
      bar.wait();
      if (zero_level.load() <= L) break;  // set only during levels <= L: every thread stops here
    }
  };
  std::vector<std::thread> th;
  for (int t = 1; t < nt; ++t) th.emplace_back(work, t);
  work(0);
  for (auto &x : th) x.join();
  return zero_level.load() != INT32_MAX ? IGM_ERR_ZERO_PIVOT : IGM_OK;
}

// Gauss-Seidel splitting (policy gauss_seidel): M = D + L_A as L D U with
// L = I + L_A D^-1, U = I: below the diagonal a_ik / a_kk, nothing
// eliminated, nothing above; every row is independent.
static igm_status gs_split_fp(int nt, int64_t n, const hvec<int64_t> &rp, const hvec<int32_t> &col,
                              HostSetup &h) {
  h.lu.resize(rp[n]);
  std::atomic<bool> zero{false};
  par_ranges(nt, n, [&](int, int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi; ++i) {
      for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
        const int64_t k = col[e];
        if (k < i) {
          const double piv = h.a[h.diag_pos[k]];
          if (piv == 0.0) zero = true;
          h.lu[e] = h.a[e] / piv;
        } else {
          h.lu[e] = k == i ? h.a[e] : 0.0;
        }
      }
      if (h.a[h.diag_pos[i]] == 0.0) zero = true;
    }
  });
  return zero ? IGM_ERR_ZERO_PIVOT : IGM_OK;
}

// eqs. (dl), (dl2), (l1), (u1): Lbar = trunc(L |D|^1/2), Ubar = trunc(sgn(D)
// |D|^1/2 U) with U unit upper (stored entries divided by the pivot).
// Patterns of the strict triangles of the integer factors (lptr, lcol, uptr,
// ucol; entries in CSR order): below the diagonal when offdiag, above it too
// when upper.
static void factor_pattern(int nt, int64_t n, const hvec<int64_t> &rp, const hvec<int32_t> &col, bool offdiag,
                           bool upper, HostSetup &h) {
  h.lptr.assign(n + 1, 0);
  h.uptr.assign(n + 1, 0);
  if (offdiag) {
    par_ranges(nt, n, [&](int, int64_t lo, int64_t hi) {
      for (int64_t i = lo; i < hi; ++i) {
        int64_t nl = 0, nu = 0;
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
          nl += col[e] < i;
          nu += upper && col[e] > i;
        }
        h.lptr[i + 1] = nl;
        h.uptr[i + 1] = nu;
      }
    });
    for (int64_t i = 0; i < n; ++i) {
      h.lptr[i + 1] += h.lptr[i];
      h.uptr[i + 1] += h.uptr[i];
    }
  }
  h.lcol.resize(h.lptr[n]);
  h.ucol.resize(h.uptr[n]);
  if (!offdiag) return;
  par_ranges(nt, n, [&](int, int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi; ++i) {
      int64_t pl = h.lptr[i], pu = h.uptr[i];
      for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
        if (col[e] < i) h.lcol[pl++] = col[e];
        else if (upper && col[e] > i) h.ucol[pu++] = col[e];
      }
    }
  });
}

static igm_status cast_factors(int nt, int64_t n, const hvec<int64_t> &rp, const hvec<int32_t> &col,
                               const hvec<double> &piv, bool offdiag, bool upper, HostSetup &h) {
  h.ldiag.resize(n);
  h.udiag.resize(n);
  hvec<double> sq(n);
  std::atomic<bool> zero{false};
  par_ranges(nt, n, [&](int, int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi; ++i) {
      if (piv[i] == 0.0 || !isfinite(piv[i])) { zero = true; return; }
      sq[i] = sqrt(fabs(piv[i]));
    }
  });
  if (zero) return IGM_ERR_ZERO_PIVOT;
  factor_pattern(nt, n, rp, col, offdiag, upper, h);
  h.lval.resize(h.lptr[n]);
  h.uval.resize(h.uptr[n]);
  FirstError fe(nt);
  par_ranges(nt, n, [&](int c, int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi; ++i) {
      bool bad = false;
      double su = piv[i] < 0.0 ? -sq[i] : sq[i];
      h.ldiag[i] = cast_i64(sq[i], bad);
      h.udiag[i] = cast_i64(su, bad);
      if (bad) return fe.set(c, i, IGM_ERR_RANGE);
      if (h.ldiag[i] == 0 || h.udiag[i] == 0) return fe.set(c, i, IGM_ERR_ZERO_PIVOT);
      if (offdiag) {
        int64_t pl = h.lptr[i], pu = h.uptr[i];
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
          int32_t j = col[e];
          if (j < i) {
            h.lval[pl++] = cast_i64(h.lu[e] * sq[j], bad);
          } else if (upper && j > i) {
            h.uval[pu++] = cast_i64(su * (h.lu[e] / piv[i]), bad);
          }
        }
      }
      if (bad) return fe.set(c, i, IGM_ERR_RANGE);
    }
  });
  return fe.first();
}

// Level sets: a row's forward level is one more than the largest level of the
// rows its strict lower part reads (rows in increasing order); backward levels
// likewise on the strict upper part in decreasing order.
static void level_sets(int64_t n, HostSetup &h) {
  // rows grouped by level, rows increasing inside a level
  auto group = [n](const std::vector<int32_t> &lev, int32_t nlev, hvec<int32_t> &ptr, hvec<int32_t> &rows) {
    ptr.assign(nlev + 1, 0);
    for (int64_t i = 0; i < n; ++i) ptr[lev[i] + 1]++;
    for (int32_t k = 0; k < nlev; ++k) ptr[k + 1] += ptr[k];
    rows.assign(n, 0);
    std::vector<int32_t> fill(ptr.begin(), ptr.end() - 1);
    for (int64_t i = 0; i < n; ++i) rows[fill[lev[i]]++] = (int32_t)i;
  };
  // the two scans are independent: the backward one runs on a second thread
  auto forward = [&] {
    std::vector<int32_t> lev(n);
    int32_t nlev = 0;
    for (int64_t i = 0; i < n; ++i) {
      int32_t l = 0;
      for (int64_t e = h.lptr[i]; e < h.lptr[i + 1]; ++e) l = std::max(l, lev[h.lcol[e]] + 1);
      lev[i] = l;
      nlev = std::max(nlev, l + 1);
    }
    group(lev, nlev, h.flev_ptr, h.flev_rows);
  };
  auto backward = [&] {
    std::vector<int32_t> lev(n);
    int32_t nlev = 0;
    for (int64_t i = n - 1; i >= 0; --i) {
      int32_t l = 0;
      for (int64_t e = h.uptr[i]; e < h.uptr[i + 1]; ++e) l = std::max(l, lev[h.ucol[e]] + 1);
      lev[i] = l;
      nlev = std::max(nlev, l + 1);
    }
    group(lev, nlev, h.blev_ptr, h.blev_rows);
  };
  if (setup_thread_count() > 1 && n >= 32768) {
    std::thread tb(backward);
    forward();
    tb.join();
  } else {
    forward();
    backward();
  }
}

// SELL-64: rows in slices of 64, each slice stored column-major with the width
// of its longest row; padding entries have value 0 and point at the row itself.
static void build_sell(int nt, int64_t n, const hvec<int64_t> &rp, const hvec<int32_t> &col,
                       HostSetup &h, bool values = true) {
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
  h.sell_col.resize(tot);
  h.sell_val.assign(values ? h.nterms : 0, hvec<int64_t>());
  for (int l = 0; l < (int)h.sell_val.size(); ++l) h.sell_val[l].resize(tot);
  par_ranges(nt, ns, [&](int, int64_t s0, int64_t s1) {
    for (int64_t s = s0; s < s1; ++s) {
      // written in layout order (entry k of the 64 rows, then k + 1)
      for (int64_t k = 0; k < h.sell_w[s]; ++k) {
        for (int lane = 0; lane < kSlice; ++lane) {
          const int64_t i = s * kSlice + lane;
          const int64_t pos = h.sell_off[s] + k * kSlice + lane;
          const int64_t e = (i < n) ? rp[i] + k : -1;
          if (i < n && e < rp[i + 1]) {
            h.sell_col[pos] = col[e];
            for (int l = 0; l < (int)h.sell_val.size(); ++l) h.sell_val[l][pos] = h.abar[l][e];
          } else {
            h.sell_col[pos] = (int32_t)std::min<int64_t>(i, n - 1);
            for (int l = 0; l < (int)h.sell_val.size(); ++l) h.sell_val[l][pos] = 0;
          }
        }
      }
    }
  }, 64);  // a slice is 64 rows
}

igm_status host_setup(int64_t n, const hvec<int64_t> &rp, const hvec<int32_t> &col,
                      const hvec<double> &ahat, const hvec<double> &bhat, const igm_policy &pol,
                      HostSetup &h) {
  SetupRegion region;
  const int nt = setup_thread_count();
  h = HostSetup();
  igm_status st = scale_rows(nt, n, rp, col, ahat, bhat, pol.alpha_a, pol.two_sided != 0, h);
  if (st != IGM_OK) return st;
  st = split_terms(nt, pol, h);
  if (st != IGM_OK) return st;
  h.diag_pos.assign(n, -1);
  par_ranges(nt, n, [&](int, int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi; ++i)
      for (int64_t e = rp[i]; e < rp[i + 1]; ++e)
        if (col[e] == i) h.diag_pos[i] = e;
  });
  if (pol.precond != IGM_PRE_NONE) {
    for (int64_t i = 0; i < n; ++i)
      if (h.diag_pos[i] < 0) return IGM_ERR_ZERO_PIVOT;
    hvec<double> piv(n);
    if (pol.precond == IGM_PRE_ILU0) {
      st = pol.gauss_seidel ? gs_split_fp(nt, n, rp, col, h) : ilu0_fp(nt, n, rp, col, h);
      if (st != IGM_OK) return st;
      for (int64_t i = 0; i < n; ++i) piv[i] = h.lu[h.diag_pos[i]];
    } else {
      for (int64_t i = 0; i < n; ++i) piv[i] = h.a[h.diag_pos[i]];
    }
    st = cast_factors(nt, n, rp, col, piv, pol.precond == IGM_PRE_ILU0, !pol.gauss_seidel, h);
    if (st != IGM_OK) return st;
    level_sets(n, h);
  }
  build_sell(nt, n, rp, col, h);
  return IGM_OK;
}

igm_status host_structure(int64_t n, const hvec<int64_t> &rp, const hvec<int32_t> &col, const igm_policy &pol,
                          HostSetup &h) {
  SetupRegion region;
  const int nt = setup_thread_count();
  h = HostSetup();
  if (pol.s_terms != 0 || pol.gauss_seidel) return IGM_ERR_UNSUPPORTED;
  h.nterms = 1;
  h.alpha[0] = 0;
  h.diag_pos.assign(n, -1);
  par_ranges(nt, n, [&](int, int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi; ++i)
      for (int64_t e = rp[i]; e < rp[i + 1]; ++e)
        if (col[e] == i) h.diag_pos[i] = e;
  });
  if (pol.precond != IGM_PRE_NONE) {  // a missing diagonal (-1) is reported by the device, in the host's order
    factor_pattern(nt, n, rp, col, pol.precond == IGM_PRE_ILU0, true, h);
    if (pol.precond == IGM_PRE_ILU0) level_sets(n, h);
  }
  build_sell(nt, n, rp, col, h, false);
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
  for (int64_t i = 0; i < n; ++i)
    if (rp[i + 1] < rp[i]) return IGM_ERR_ARG;
  std::atomic<bool> bad{false};
  par_ranges(setup_thread_count(), n, [&](int, int64_t lo, int64_t hi) {
    for (int64_t i = lo; i < hi; ++i) {
      for (int64_t e = rp[i]; e < rp[i + 1]; ++e) {
        if (col[e] < 0 || col[e] >= n || (e > rp[i] && col[e] <= col[e - 1]) || !isfinite(val[e])) {
          bad = true;
          return;
        }
      }
      if (!isfinite(b[i])) {
        bad = true;
        return;
      }
    }
  });
  return bad ? IGM_ERR_ARG : IGM_OK;
}

}  // namespace igm
