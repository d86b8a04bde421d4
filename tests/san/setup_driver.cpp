// Sanitizer run of the library's host setup (test infrastructure): the
// setup of seeded stencil systems above the size where its passes run on
// several threads, with one thread and with four; every product must be the
// same bit for bit. Built with g++ and AddressSanitizer + UndefinedBehavior
// Sanitizer, or ThreadSanitizer. Exit status 0 on success.
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <cmath>
#include <cstdint>
#include <vector>

#include "../../paper_2009_07495_amd/csrc/igm_internal.hpp"

using igm::hvec;

struct Csr {
  int64_t n = 0;
  hvec<int64_t> rp;
  hvec<int32_t> col;
  hvec<double> val, b;
};

// 7-point stencil on an nx x ny x nz grid with seeded nonsymmetric values
// (diagonal = 1.1 x the sum of the off-diagonal magnitudes)
static Csr stencil(int nx, int ny, int nz, uint64_t seed) {
  Csr a;
  a.n = (int64_t)nx * ny * nz;
  a.rp.assign(a.n + 1, 0);
  uint64_t s = seed;
  auto rnd = [&] {  // 53-bit uniform in [0, 1) from a 64-bit LCG
    s = s * 6364136223846793005ull + 1442695040888963407ull;
    return (double)(s >> 11) / 9007199254740992.0;
  };
  for (int z = 0; z < nz; ++z)
    for (int y = 0; y < ny; ++y)
      for (int x = 0; x < nx; ++x) {
        const int64_t r = ((int64_t)z * ny + y) * nx + x;
        const int64_t nb[7] = {r - (int64_t)nx * ny, r - nx, r - 1, r, r + 1, r + nx, r + (int64_t)nx * ny};
        const bool ok[7] = {z > 0, y > 0, x > 0, true, x < nx - 1, y < ny - 1, z < nz - 1};
        double off = 0.0;
        size_t dpos = 0;
        for (int t = 0; t < 7; ++t)
          if (ok[t]) {
            a.col.push_back((int32_t)nb[t]);
            double v = nb[t] == r ? 0.0 : -(0.5 + rnd());
            if (nb[t] == r) dpos = a.val.size();
            off += std::fabs(v);
            a.val.push_back(v);
          }
        a.val[dpos] = 1.1 * off;
        a.rp[r + 1] = (int64_t)a.col.size();
        a.b.push_back(2.0 * rnd() - 1.0);
      }
  return a;
}

// the shift settings of Table IV (no preconditioner) and Table VI (ILU(0);
// also its diagonal-only variant), as in tests/golden/shift_presets.txt
static igm_policy preset_policy(int precond) {
  igm_policy p;
  memset(&p, 0, sizeof(p));
  p.struct_size = sizeof(igm_policy);
  p.df = 30; p.m = 30; p.max_refine = 2000; p.gtol = -1; p.tol = 1e-10;
  p.precond = precond;
  if (precond == IGM_PRE_NONE) {
    p.alpha_a = 16;
    p.b_dot = p.b_axpy = p.b_norm = p.b_rot = p.b_tmp = 16;
    p.b_div_num = p.b_cs_num = 16;
    p.b_div_den = p.b_cs_den = 14;
  } else {
    p.alpha_a = 32;
    p.b_div_num = p.b_cs_num = 30;
  }
  return p;
}

static uint64_t H;
template <class V>
static void mix(const V &v) {
  const unsigned char *p = (const unsigned char *)v.data();
  for (size_t i = 0; i < v.size() * sizeof(v[0]); ++i) H = (H ^ p[i]) * 1099511628211ull;
  H = (H ^ v.size()) * 1099511628211ull;
}

static uint64_t setup_hash(const Csr &a, const igm_policy &p, igm_status &st) {
  igm::HostSetup h;
  st = igm::host_setup(a.n, a.rp, a.col, a.val, a.b, p, h);
  H = 1469598103934665603ull;
  mix(h.dhat); mix(h.a); mix(h.b); mix(h.diag_pos); mix(h.lu); mix(h.ldiag); mix(h.udiag);
  for (auto &v : h.abar) mix(v);
  mix(h.lptr); mix(h.uptr); mix(h.lcol); mix(h.ucol); mix(h.lval); mix(h.uval);
  mix(h.flev_ptr); mix(h.flev_rows); mix(h.blev_ptr); mix(h.blev_rows);
  mix(h.sell_off); mix(h.sell_w); mix(h.sell_col);
  for (auto &v : h.sell_val) mix(v);
  return H;
}

// Slot of entry kk (CSR order) of the row at sorted position k of block q,
// level L: levels are stored column-major.
static int64_t entry_at(const igm::BlockSchedule &b, int32_t q, int32_t L, int32_t k, int64_t kk) {
  const int32_t *lo = b.lvoff.data() + b.lvbase[q];
  return b.levent[b.lvbase[q] + L] + kk * (lo[L + 1] - lo[L]) + (k - lo[L]);
}

// The blocked sweep schedule of a strict triangular factor (igm_bsched.cpp):
// every row appears once; an in-block dependency sits at a lower local level
// of the same block; a dependency on another block is covered by a wait
// record at or before the row's level asking for at least the dependency's
// level + 1 (blocks only wait on earlier blocks); and a serial replay of the
// schedule (exact integer sums, truncating division) equals plain
// substitution in processing order. Returns the number of violations.
static int check_schedule(int64_t n, bool lower, int32_t S, const hvec<int64_t> &ptr, const hvec<int32_t> &col,
                          const hvec<int64_t> &val, const hvec<int64_t> &diag, uint64_t &hash) {
  igm::BlockSchedule b;
  igm::block_schedule(n, lower, S, ptr, col, val, diag, b);
  int bad = 0;
  auto pos_of = [&](int64_t r) { return lower ? r : n - 1 - r; };
  std::vector<int32_t> where(n, -1), level(n, -1);  // sorted position and local level of each row
  for (int32_t q = 0; q < b.nb; ++q) {
    const int32_t *lo = b.lvoff.data() + b.lvbase[q];
    const int32_t nl = b.lvbase[q + 1] - b.lvbase[q] - 1;
    for (int32_t L = 0; L < nl; ++L)
      for (int32_t k = lo[L]; k < lo[L + 1]; ++k) {
        const int64_t r = b.prow[(int64_t)q * S + k];
        if (where[r] >= 0 || pos_of(r) / S != q) ++bad;
        where[r] = (int32_t)((int64_t)q * S + k);
        level[r] = L;
      }
  }
  for (int64_t r = 0; r < n; ++r)
    if (where[r] < 0) ++bad;
  if (bad) return bad;
  // dependencies against the levels and the wait records
  for (int32_t q = 0; q < b.nb; ++q) {
    std::vector<int32_t> req(b.nb, 0);
    int32_t w = b.wbase[q];
    const int32_t *lo = b.lvoff.data() + b.lvbase[q];
    const int32_t nl = b.lvbase[q + 1] - b.lvbase[q] - 1;
    for (int32_t L = 0; L < nl; ++L) {
      for (; w < b.wbase[q + 1] && b.wrec[w].level <= L; ++w) {
        if (b.wrec[w].level != L || b.wrec[w].dep >= q) ++bad;
        req[b.wrec[w].dep] = std::max(req[b.wrec[w].dep], b.wrec[w].need);
      }
      for (int32_t k = lo[L]; k < lo[L + 1]; ++k) {
        const int64_t pk = (int64_t)q * S + k;
        if (b.plen[pk] != ptr[b.prow[pk] + 1] - ptr[b.prow[pk]]) ++bad;
        for (int64_t kk = 0; kk < b.plen[pk]; ++kk) {
          const int64_t e = entry_at(b, q, L, k, kk);
          if (e < b.levent[b.lvbase[q] + L] || e >= b.levent[b.lvbase[q] + L + 1]) ++bad;
          const int32_t c = b.ecode[e];
          if (c >= 0) {
            if (c >= S || level[b.prow[(int64_t)q * S + c]] >= L) ++bad;
          } else {
            const int64_t dr = -(int64_t)c - 1;
            const int32_t dq = (int32_t)(pos_of(dr) / S);
            if (dq >= q || req[dq] < level[dr] + 1) ++bad;
          }
        }
      }
    }
    if (w != b.wbase[q + 1]) ++bad;
  }
  // replay against plain substitution (rhs z_i = 2^40 + 12345 i, varying signs)
  std::vector<int64_t> z(n), ref(n), got(n);
  for (int64_t i = 0; i < n; ++i) z[i] = (i % 3 == 1 ? -1 : 1) * (((int64_t)1 << 40) + 12345 * i);
  auto tdiv = [](__int128 a, int64_t d) { return (int64_t)(a / d); };
  for (int64_t p = 0; p < n; ++p) {
    const int64_t r = lower ? p : n - 1 - p;
    __int128 acc = z[r];
    for (int64_t e = ptr[r]; e < ptr[r + 1]; ++e) acc -= (__int128)val[e] * ref[col[e]];
    ref[r] = tdiv(acc, diag[r]);
  }
  for (int32_t q = 0; q < b.nb; ++q) {
    const int32_t *lo = b.lvoff.data() + b.lvbase[q];
    const int32_t nl = b.lvbase[q + 1] - b.lvbase[q] - 1;
    for (int32_t L = 0; L < nl; ++L)
      for (int32_t k = lo[L]; k < lo[L + 1]; ++k) {
        const int64_t pk = (int64_t)q * S + k;
        const int64_t r = b.prow[pk];
        __int128 acc = z[r];
        for (int64_t kk = 0; kk < b.plen[pk]; ++kk) {
          const int64_t e = entry_at(b, q, L, k, kk);
          const int64_t want = col[ptr[r] + kk];  // CSR order kept
          if (b.ecode[e] >= 0 ? b.prow[(int64_t)q * S + b.ecode[e]] != want : -(int64_t)b.ecode[e] - 1 != want) ++bad;
          const int32_t c = b.ecode[e];
          const int64_t x = c >= 0 ? got[b.prow[(int64_t)q * S + c]] : got[-(int64_t)c - 1];
          acc -= (__int128)b.eval[e] * x;
          if ((double)b.eval[e] != b.evalf[e]) ++bad;
        }
        if (b.pdiag[pk] != diag[r]) ++bad;
        got[r] = tdiv(acc, b.pdiag[pk]);
      }
  }
  for (int64_t r = 0; r < n; ++r)
    if (got[r] != ref[r]) ++bad;
  H = 1469598103934665603ull;
  mix(b.prow); mix(b.plen); mix(b.levent); mix(b.ecode); mix(b.eval); mix(b.pdiag); mix(b.lvbase); mix(b.lvoff);
  mix(b.wbase);
  for (const auto &w : b.wrec) {
    const int32_t f[4] = {w.level, w.slot, w.need, w.dep};
    for (int32_t x : f) H = (H ^ (uint32_t)x) * 1099511628211ull;
  }
  hash = H;
  return bad;
}

int main() {
  int bad = 0;
  const Csr a = stencil(40, 40, 24, 7);  // 38,400 rows
  if (igm::validate_csr(a.n, a.rp.data(), a.col.data(), a.val.data(), a.b.data()) != IGM_OK) ++bad;
  for (int preset : {IGM_PRE_NONE, IGM_PRE_ILU0, IGM_PRE_JACOBI}) {
    igm_policy p = preset_policy(preset);
    if (preset == IGM_PRE_NONE) p.s_terms = 2;  // also the correction terms
    igm_status s1, s4;
    setenv("IGM_SETUP_THREADS", "1", 1);
    const uint64_t h1 = setup_hash(a, p, s1);
    setenv("IGM_SETUP_THREADS", "4", 1);
    const uint64_t h4 = setup_hash(a, p, s4);
    printf("preconditioner %d: status %d / %d, hash %016llx / %016llx\n", preset, (int)s1, (int)s4, (unsigned long long)h1,
           (unsigned long long)h4);
    if (s1 != IGM_OK || s4 != IGM_OK || h1 != h4) ++bad;
  }
  // blocked sweep schedules of the ILU(0) factors: invariants, replay, and
  // the same schedule for one and four setup threads
  {
    igm_policy p = preset_policy(IGM_PRE_ILU0);
    igm::HostSetup h;
    igm_status st = igm::host_setup(a.n, a.rp, a.col, a.val, a.b, p, h);
    if (st != IGM_OK) ++bad;
    for (int32_t S : {64, 640, 4096, 65536}) {
      for (int lower = 0; lower < 2; ++lower) {
        uint64_t h1 = 0, h4 = 0;
        setenv("IGM_SETUP_THREADS", "1", 1);
        int v1 = lower ? check_schedule(a.n, true, S, h.lptr, h.lcol, h.lval, h.ldiag, h1)
                       : check_schedule(a.n, false, S, h.uptr, h.ucol, h.uval, h.udiag, h1);
        setenv("IGM_SETUP_THREADS", "4", 1);
        int v4 = lower ? check_schedule(a.n, true, S, h.lptr, h.lcol, h.lval, h.ldiag, h4)
                       : check_schedule(a.n, false, S, h.uptr, h.ucol, h.uval, h.udiag, h4);
        printf("blocked schedule S=%d %s: %d / %d violations, hash %016llx / %016llx\n", S,
               lower ? "forward" : "backward", v1, v4, (unsigned long long)h1, (unsigned long long)h4);
        if (v1 || v4 || h1 != h4) ++bad;
      }
    }
  }
  // error paths: an all-zero row, a zero ILU pivot
  Csr z = a;
  for (int64_t e = z.rp[100]; e < z.rp[101]; ++e) z.val[e] = 0.0;
  igm_policy p = preset_policy(IGM_PRE_NONE);
  igm_status st;
  setup_hash(z, p, st);
  if (st != IGM_ERR_SINGULAR_ROW) ++bad;
  printf("host setup sanitizer run: %d failures\n", bad);
  return bad ? 1 : 0;
}
