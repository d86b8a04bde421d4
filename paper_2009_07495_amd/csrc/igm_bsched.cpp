// Host construction of the blocked schedule of the ILU(0) triangular sweeps
// (the preconditioner apply of Sec. VI; the device side is igm_bsweep.hpp).
//
// Rows are taken in processing order (increasing for the forward sweep on the
// strict lower factor, decreasing for the backward sweep on the strict upper
// factor) and cut into blocks of S consecutive positions. Inside a block a
// row's local level is one more than the largest local level of the rows of
// the same block it reads; the block's rows are stored sorted by local level
// (then by position), so one workgroup can run the block level by level with
// its values in LDS. A dependency on a row of another block (always an
// earlier block) becomes a wait record: before local level L the other block
// must have finished as many of its own local levels as that row needs.
// Records of one (block, dependency block) pair are kept only where the
// requirement grows, since the other block finishes its levels in order.
//
// The schedule only reorders independent work: every row is still computed
// from the same operands with the same exact sum, so the sweep's bits do not
// depend on S.
#include <algorithm>
#include <thread>

#include "igm_internal.hpp"
#include "igm_par.hpp"

namespace igm {

namespace {

// f(q) for every block q, blocks spread over the setup threads.
template <class F>
void for_blocks(int32_t nb, F &&f) {
  const int nt = std::max(1, std::min<int>(setup_thread_count(), nb));
  if (nt <= 1) {
    for (int32_t q = 0; q < nb; ++q) f(q);
    return;
  }
  std::vector<std::thread> th;
  for (int t = 1; t < nt; ++t)
    th.emplace_back([&f, t, nt, nb] {
      for (int32_t q = t; q < nb; q += nt) f(q);
    });
  for (int32_t q = 0; q < nb; q += nt) f(q);
  for (auto &x : th) x.join();
}

struct CrossDep {
  int32_t dep, level, need;
};

}  // namespace

void block_schedule(int64_t n, bool lower, int32_t S, const hvec<int64_t> &ptr, const hvec<int32_t> &col,
                    const hvec<int64_t> &val, const hvec<int64_t> &diag, BlockSchedule &o) {
  o = BlockSchedule();
  o.S = S;
  o.nb = (int32_t)((n + S - 1) / S);
  const int32_t nb = o.nb;
  auto row_of = [&](int64_t p) { return lower ? p : n - 1 - p; };  // also maps rows to positions
  hvec<int32_t> lv(n), sorted(n);  // local level of each position; sorted index inside its block
  std::vector<int32_t> nl(nb);
  std::vector<int64_t> eslots(nb);  // entry slots of each block (levels padded to their longest row)
  std::vector<int32_t> widest(nb);  // rows of each block's widest level
  for_blocks(nb, [&](int32_t q) {
    const int64_t p0 = (int64_t)q * S, p1 = std::min<int64_t>(n, p0 + S);
    int32_t top = 0;
    for (int64_t p = p0; p < p1; ++p) {
      const int64_t r = row_of(p);
      int32_t l = 0;
      for (int64_t e = ptr[r]; e < ptr[r + 1]; ++e) {
        const int64_t pc = row_of(col[e]);
        if (pc >= p0) l = std::max(l, lv[pc] + 1);  // dependencies precede p: pc < p
      }
      lv[p] = l;
      top = std::max(top, l + 1);
    }
    // counting sort by level, stable in position; widest row of each level
    std::vector<int32_t> fill(top + 1, 0);
    std::vector<int64_t> width(top, 0);
    for (int64_t p = p0; p < p1; ++p) {
      fill[lv[p] + 1]++;
      const int64_t r = row_of(p);
      width[lv[p]] = std::max<int64_t>(width[lv[p]], ptr[r + 1] - ptr[r]);
    }
    int64_t slots = 0;
    int32_t wmax = 0;
    for (int32_t l = 0; l < top; ++l) {
      slots += width[l] * fill[l + 1];
      wmax = std::max(wmax, fill[l + 1]);  // rows of level l
    }
    for (int32_t l = 0; l < top; ++l) fill[l + 1] += fill[l];
    for (int64_t p = p0; p < p1; ++p) sorted[p] = fill[lv[p]]++;
    nl[q] = top;
    eslots[q] = slots;
    widest[q] = wmax;
  });
  o.lvbase.assign(nb + 1, 0);
  std::vector<int64_t> ebase(nb + 1, 0);
  for (int32_t q = 0; q < nb; ++q) {
    o.lvbase[q + 1] = o.lvbase[q] + nl[q] + 1;
    ebase[q + 1] = ebase[q] + eslots[q];
    o.max_levels = std::max(o.max_levels, nl[q]);
    o.max_width = std::max(o.max_width, widest[q]);
  }
  const int64_t nslots = ebase[nb];  // one more slot follows: the padding slot (code 0, value 0)
  o.prow.resize(n);
  o.plen.resize(n);
  o.pdiag.resize(n);
  o.pmag.resize(n);
  o.pshift.resize(n);
  o.ecode.resize(nslots + 1);
  o.eval.resize(nslots + 1);
  o.evalf.resize(nslots + 1);
  o.ecode[nslots] = 0;
  o.eval[nslots] = 0;
  o.evalf[nslots] = 0.0;
  o.pad_slot = nslots;
  o.lvoff.resize(o.lvbase[nb]);
  o.levent.resize(o.lvbase[nb]);
  std::vector<std::vector<WaitRec>> recs(nb);
  std::vector<int32_t> slots(nb), narrow(nb, 1);
  for_blocks(nb, [&](int32_t q) {
    const int64_t p0 = (int64_t)q * S, p1 = std::min<int64_t>(n, p0 + S);
    int32_t *lo = o.lvoff.data() + o.lvbase[q];
    int64_t *le = o.levent.data() + o.lvbase[q];
    for (int32_t l = 0; l <= nl[q]; ++l) lo[l] = 0;
    for (int64_t p = p0; p < p1; ++p) lo[lv[p] + 1]++;
    for (int32_t l = 0; l < nl[q]; ++l) lo[l + 1] += lo[l];
    for (int64_t p = p0; p < p1; ++p) {
      const int64_t r = row_of(p);
      o.prow[p0 + sorted[p]] = (int32_t)r;
      o.plen[p0 + sorted[p]] = (int32_t)(ptr[r + 1] - ptr[r]);
      o.pdiag[p0 + sorted[p]] = diag[r];
      if (diag[r] != 0) div_magic(diag[r], o.pmag[p0 + sorted[p]], o.pshift[p0 + sorted[p]]);
      else o.pmag[p0 + sorted[p]] = 0, o.pshift[p0 + sorted[p]] = 512;  // the device divides the slow way
    }
    // level L's slots: its row count times its widest row
    le[0] = ebase[q];
    for (int32_t l = 0; l < nl[q]; ++l) {
      int64_t w = 0;
      for (int32_t k = lo[l]; k < lo[l + 1]; ++k) w = std::max<int64_t>(w, o.plen[p0 + k]);
      le[l + 1] = le[l] + w * (lo[l + 1] - lo[l]);
    }
    std::fill(o.ecode.begin() + ebase[q], o.ecode.begin() + ebase[q + 1], 0);  // padding: never read
    std::fill(o.eval.begin() + ebase[q], o.eval.begin() + ebase[q + 1], 0);
    std::fill(o.evalf.begin() + ebase[q], o.evalf.begin() + ebase[q + 1], 0.0);
    std::vector<CrossDep> cross;
    for (int32_t l = 0; l < nl[q]; ++l) {
      const int64_t c = lo[l + 1] - lo[l];
      for (int32_t k = lo[l]; k < lo[l + 1]; ++k) {
        const int64_t r = o.prow[p0 + k];
        const int64_t p = row_of(r);
        int64_t kk = 0;
        for (int64_t e = ptr[r]; e < ptr[r + 1]; ++e, ++kk) {
          const int64_t at = le[l] + kk * c + (k - lo[l]);
          const int64_t cl = col[e];
          const int64_t pc = row_of(cl);
          o.eval[at] = val[e];
          o.evalf[at] = (double)val[e];
          if (val[e] < INT32_MIN || val[e] > INT32_MAX) narrow[q] = 0;
          if (pc >= p0) {
            o.ecode[at] = sorted[pc];
          } else {
            o.ecode[at] = (int32_t)(-(cl + 1));
            cross.push_back({(int32_t)(pc / S), lv[p], lv[pc] + 1});
          }
        }
      }
    }
    // keep, per dependency block, the levels where its requirement grows
    std::sort(cross.begin(), cross.end(), [](const CrossDep &a, const CrossDep &b) {
      return a.dep != b.dep ? a.dep < b.dep : a.level != b.level ? a.level < b.level : a.need > b.need;
    });
    std::vector<WaitRec> &rq = recs[q];
    int32_t slot = -1, prev_dep = -1, best = 0;
    for (const CrossDep &d : cross) {
      if (d.dep != prev_dep) {
        prev_dep = d.dep;
        ++slot;
        best = 0;
      }
      if (d.need > best) {
        best = d.need;
        rq.push_back({d.level, slot, d.need, d.dep});
      }
    }
    std::stable_sort(rq.begin(), rq.end(), [](const WaitRec &a, const WaitRec &b) { return a.level < b.level; });
    slots[q] = slot + 1;
  });
  o.wbase.assign(nb + 1, 0);
  o.narrow = true;
  for (int32_t q = 0; q < nb; ++q) {
    o.wbase[q + 1] = o.wbase[q] + (int32_t)recs[q].size();
    o.max_slots = std::max(o.max_slots, slots[q]);
    o.narrow = o.narrow && narrow[q];
  }
  o.wrec.resize(o.wbase[nb]);
  for (int32_t q = 0; q < nb; ++q) std::copy(recs[q].begin(), recs[q].end(), o.wrec.begin() + o.wbase[q]);
}

}  // namespace igm
