// Host-side symbolic setup: partition, algebraic overlap, the coarse maps of
// the two-level variant, the extended patterns A_i = R_i A R_i^T with their
// value sources, block ILU(0) update pairs and level schedules, and the
// device layouts of the triangular solves.
//
// Method (Jackson, Taroni, Ponting, arXiv:1401.7227):
//  - classical additive Schwarz, eq. (3.3)-(3.4): A_i = R_i A R_i^T with
//    R_i restricting to the overlapping subdomain;
//  - two-level variant, Section 4, eq. (4.1)-(4.5): R_i keeps subdomain i
//    (with its overlap) and lumps every other cell by summation (App. B,
//    eq. (B.3)) into near-field boxes on face-neighbour subdomains and
//    far-field boxes elsewhere;
//  - local solver: block ILU(0) (Section 2 and Section 6).
//
// Lumping is done in the shared way Section 4 asks for (matrix elements are
// lumped once and shared, not re-summed per subdomain): cells are grouped
// into atoms that every subdomain sees as wholly fine or wholly inside one
// coarse variable, and each subdomain's coarse entries are sums of
// atom-level lumped blocks.
#include "setup.hpp"

#include <algorithm>
#include <array>
#include <cstring>
#include <map>
#include <numeric>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace asmx {
namespace {


struct Split {
  std::vector<int32_t> part;   // part of each column index
  std::vector<int32_t> start;  // first column of each part, size k+1
};

// Balanced split of n columns into k parts: the first (n mod k) parts are
// one column wider.
Split balanced(int n, int k) {
  Split s;
  s.start.resize(k + 1);
  const int base = n / k, rem = n % k;
  s.start[0] = 0;
  for (int p = 0; p < k; ++p) s.start[p + 1] = s.start[p] + base + (p < rem ? 1 : 0);
  s.part.resize(n);
  for (int p = 0; p < k; ++p)
    for (int i = s.start[p]; i < s.start[p + 1]; ++i) s.part[i] = p;
  return s;
}

struct Csr {
  std::vector<int32_t> ptr, idx;
};

// Undirected block graph (pattern of A plus its transpose, no self loops).
Csr undirected(const HostPattern &A) {
  Csr g;
  g.ptr.assign(A.N + 1, 0);
  for (int r = 0; r < A.N; ++r)
    for (int e = A.rp[r]; e < A.rp[r + 1]; ++e) {
      const int c = A.ci[e];
      if (c == r) continue;
      g.ptr[r + 1]++;
      g.ptr[c + 1]++;
    }
  for (int r = 0; r < A.N; ++r) g.ptr[r + 1] += g.ptr[r];
  g.idx.resize(g.ptr[A.N]);
  std::vector<int32_t> fill(g.ptr.begin(), g.ptr.end() - 1);
  for (int r = 0; r < A.N; ++r)
    for (int e = A.rp[r]; e < A.rp[r + 1]; ++e) {
      const int c = A.ci[e];
      if (c == r) continue;
      g.idx[fill[r]++] = c;
      g.idx[fill[c]++] = r;
    }
  return g;
}

// Column view of A: for column d, the (row, entry) pairs holding it, rows
// ascending.
struct Transpose {
  std::vector<int32_t> ptr, row, ent;
};

Transpose transpose(const HostPattern &A) {
  Transpose t;
  t.ptr.assign(A.N + 1, 0);
  for (int64_t e = 0; e < A.nnzb; ++e) t.ptr[A.ci[e] + 1]++;
  for (int d = 0; d < A.N; ++d) t.ptr[d + 1] += t.ptr[d];
  t.row.resize(A.nnzb);
  t.ent.resize(A.nnzb);
  std::vector<int32_t> fill(t.ptr.begin(), t.ptr.end() - 1);
  for (int r = 0; r < A.N; ++r)
    for (int e = A.rp[r]; e < A.rp[r + 1]; ++e) {
      const int d = A.ci[e];
      t.row[fill[d]] = r;
      t.ent[fill[d]] = e;
      fill[d]++;
    }
  return t;
}

// Per-subdomain result of the symbolic phase (local indices).
struct SubLocal {
  int32_t n = 0, nfine = 0, ncoarse = 0;
  std::vector<int32_t> cells;   // fine rows -> cell
  std::vector<uint8_t> owned;   // fine rows owned by this subdomain
  std::vector<int32_t> rp, ci;  // CSR of A_i
  std::vector<int32_t> sptr, sidx;  // value sources per entry (pool indices)
  std::vector<int32_t> diag;
  std::vector<int32_t> tptr, tdst, tsrc;
  std::vector<int32_t> cptr, cidx;  // coarse rows -> near/far atom sums
  // factorisation steps (forward chunks) and sweep records, local offsets
  std::vector<Step> fst;
  std::vector<int32_t> frow;             // rows in forward order
  std::vector<int32_t> bpos;             // backward position of each row
  std::vector<RecStep> rf, rb;           // rec/pos fields local (rec in bytes)
  std::vector<uint8_t> rec;
  std::vector<int32_t> fsrc;             // per forward position (coarse: local index)
  std::vector<int32_t> rl_src, rl_base, rl_stride;  // base in elements, local
  std::vector<uint8_t> rl_to32;
  int32_t levels = 0;
  int64_t spilled = 0;
  int64_t split_rows = 0;  // rows whose sum runs over several sweep steps (pieces)
  int32_t bad_row = -1;  // missing diagonal
};

// Everything about atoms that the per-subdomain pass needs.
struct Atoms {
  bool on = false;
  int32_t nA = 0, nNa = 0, nFa = 0;
  std::vector<int32_t> cell_atom;            // fine atom of each cell
  std::vector<int32_t> a_near, a_far;        // fine atom -> N-atom, F-atom
  std::vector<int32_t> na_box, na_owner, fa_box, fa_owner;
  Csr na_sig, fa_sig;                         // subdomains for which the atom is fine
  Csr owner_na, owner_fa;                     // owner -> its N-atoms / F-atoms
  // L2 blocks: 4 matrices, CSR over row atoms, pool position of each entry
  struct M {
    std::vector<int32_t> ptr, col, pos;
  } nn, nf, fn, ff;
  std::vector<int32_t> nbox, fbox;            // per cell
  int32_t nbn = 0, nbf = 0;
};

inline bool contains(const Csr &c, int row, int v) {
  for (int t = c.ptr[row]; t < c.ptr[row + 1]; ++t)
    if (c.idx[t] == v) return true;
  return false;
}

// Assigns compact ids to keys (in sorted key order).  keys: (k1, k2) pairs
// with non-negative components.  The pairs are packed into one 64-bit key
// when the range allows, and sorted directly (with their index) rather than
// through an index permutation.
std::vector<int32_t> compact_ids(const std::vector<std::pair<int64_t, int64_t>> &keys, int32_t &nids) {
  const size_t n = keys.size();
  std::vector<int32_t> id(n);
  int64_t max1 = 0, max2 = 0;
  for (const auto &k : keys) {
    max1 = std::max(max1, k.first);
    max2 = std::max(max2, k.second);
  }
  int32_t next = -1;
  if (max2 < INT64_MAX / 2 && max1 < INT64_MAX / (max2 + 1) - 1) {
    std::vector<std::pair<int64_t, int32_t>> s(n);
    for (size_t i = 0; i < n; ++i) s[i] = {keys[i].first * (max2 + 1) + keys[i].second, (int32_t)i};
    std::sort(s.begin(), s.end());
    for (size_t i = 0; i < n; ++i) {
      if (i == 0 || s[i].first != s[i - 1].first) ++next;
      id[s[i].second] = next;
    }
  } else {
    std::vector<int32_t> order(n);
    std::iota(order.begin(), order.end(), 0);
    std::sort(order.begin(), order.end(), [&](int a, int b) { return keys[a] < keys[b]; });
    for (size_t i = 0; i < n; ++i) {
      if (i == 0 || keys[order[i]] != keys[order[i - 1]]) ++next;
      id[order[i]] = next;
    }
  }
  nids = next + 1;
  return id;
}

// Builds a CSR "row -> (col, source)" lumped matrix from (row, col, src)
// triples; returns pattern and gather list (sources in ascending order).
void triples_to_csr(std::vector<std::array<int32_t, 3>> &t, int32_t nrows, std::vector<int32_t> &ptr,
                    std::vector<int32_t> &col, GatherList &g) {
  // bucket by row (counting sort), then sort each row's (col, src) pairs:
  // the same order as sorting the triples, without one large sort
  const size_t n = t.size();
  std::vector<int64_t> rs(nrows + 1, 0);
  for (const auto &x : t) rs[x[0] + 1]++;
  for (int r = 0; r < nrows; ++r) rs[r + 1] += rs[r];
  std::vector<std::pair<int32_t, int32_t>> cs(n);
  {
    std::vector<int64_t> cur(rs.begin(), rs.end() - 1);
    for (const auto &x : t) cs[cur[x[0]]++] = {x[1], x[2]};
  }
  std::vector<int32_t> ndist(nrows, 0);
#pragma omp parallel for schedule(dynamic, 256)
  for (int r = 0; r < nrows; ++r) {
    std::sort(cs.begin() + rs[r], cs.begin() + rs[r + 1]);
    int d = 0;
    for (int64_t i = rs[r]; i < rs[r + 1]; ++i) d += (i == rs[r] || cs[i].first != cs[i - 1].first);
    ndist[r] = d;
  }
  ptr.assign(nrows + 1, 0);
  for (int r = 0; r < nrows; ++r) ptr[r + 1] = ptr[r] + ndist[r];
  col.assign(ptr[nrows], 0);
  const size_t g0 = g.ptr.size() - 1;          // groups already in g
  const int64_t i0 = (int64_t)g.idx.size();   // sources already in g
  g.ptr.resize(g0 + 1 + ptr[nrows]);
  g.idx.resize(i0 + n);
#pragma omp parallel for schedule(dynamic, 256)
  for (int r = 0; r < nrows; ++r) {
    int k = ptr[r] - 1;
    for (int64_t i = rs[r]; i < rs[r + 1]; ++i) {
      if (i == rs[r] || cs[i].first != cs[i - 1].first) col[++k] = cs[i].first;
      g.idx[i0 + i] = cs[i].second;
      g.ptr[g0 + 1 + k] = (int32_t)(i0 + i + 1);
    }
  }
}

inline int32_t align16(int64_t b) { return (int32_t)((b + 15) & ~int64_t(15)); }

// Record section offsets of a step.  total: bytes stored in global memory;
// lds: bytes the record occupies in an LDS buffer (stored part plus the
// rows' inputs).
struct StepShape {
  int n32 = 0, n64 = 0, nlong = 0;  // rows per section
  int e32 = 0, e64 = 0, elong = 0;  // entries per section
  int nrows() const { return n32 + n64 + nlong; }
};
struct RecLayout {
  int32_t slots32, slots64, ldeps, lrptr, vals32, vals64, lvals, dinv32, dinv64, total, lds;
};


RecLayout rec_layout(const StepShape &k, bool fwd) {
  RecLayout L{};
  int64_t at = align16(kRecHead + (int64_t)kRecRowBytes * k.nrows());
  L.slots32 = (int32_t)at;
  at += align16((int64_t)2 * k.e32);
  L.slots64 = (int32_t)at;
  at += align16((int64_t)2 * k.e64);
  L.ldeps = (int32_t)at;
  at += align16((int64_t)4 * k.elong);
  L.lrptr = (int32_t)at;
  if (k.nlong > 0) at += align16((int64_t)4 * (k.nlong + 1));
  L.vals32 = (int32_t)at;
  at += align16((int64_t)36 * k.e32);
  L.vals64 = (int32_t)at;
  at += align16((int64_t)72 * k.e64);
  L.lvals = (int32_t)at;
  at += align16((int64_t)72 * k.elong);
  L.dinv32 = (int32_t)at;
  if (!fwd) at += align16((int64_t)36 * k.n32);
  L.dinv64 = (int32_t)at;
  if (!fwd) at += align16((int64_t)72 * (k.n64 + k.nlong));
  const int64_t lim = (int64_t)1 << 30;
  L.total = (int32_t)std::min(at, lim);
  L.lds = (int32_t)std::min((int64_t)rec_in_offset(at) + rec_in_bytes(k.nrows()), lim);
  return L;
}

// Level steps of both sweeps of one subdomain.  The rows of a level form
// steps of at most kMaxStepRows rows whose record fits one LDS buffer; a
// step holds short FP32 rows, short FP64 rows and long rows (sections in
// that order; short rows sorted by entry count, descending).  A long row
// too big for a buffer on its own becomes one-row pieces.  LDS vector
// slots are assigned by a linear scan over live ranges; rows that get no
// slot pass their values through the global vector and are reloaded by
// fill steps.
void build_sweeps(SubLocal &S, const std::vector<int32_t> &lf, int maxf, const std::vector<int32_t> &lb, int maxb,
                  bool fp32, bool restricted, const std::vector<int32_t> &owner, int sub) {
  struct Chunk {
    std::vector<int32_t> rows;  // section order
    int n32 = 0, n64 = 0;       // short rows of each precision (the rest are long)
    int piece = kPieceWhole;    // split row: which piece
    int e0 = 0, e1 = 0;         // split row: entry range (of the row's entries)
  };
  auto count = [&](int i, bool fwd) {
    int c = 0;
    for (int e = S.rp[i]; e < S.rp[i + 1]; ++e) c += fwd ? (S.ci[e] < i) : (S.ci[e] > i);
    return c;
  };
  // section of a row: 0 short FP32, 1 short FP64, 2 long
  auto section = [&](int i, bool fwd) {
    if (count(i, fwd) > kMaxJdsWidth) return 2;
    return (fp32 && i < S.nfine) ? 0 : 1;
  };
  auto make_chunks = [&](bool fwd, const std::vector<int32_t> &lev, int maxl) {
    std::vector<Chunk> out;
    std::vector<std::vector<int32_t>> bylev(maxl + 1);
    for (int i = 0; i < S.n; ++i) bylev[lev[i]].push_back(i);
    for (int l = 0; l <= maxl; ++l) {
      std::vector<int32_t> rows[3];
      for (int i : bylev[l]) rows[section(i, fwd)].push_back(i);
      for (int sc = 0; sc < 2; ++sc)
        std::stable_sort(rows[sc].begin(), rows[sc].end(), [&](int a, int b) { return count(a, fwd) > count(b, fwd); });
      Chunk cur;
      StepShape shp;
      auto flush = [&]() {
        if (!cur.rows.empty()) out.push_back(cur);
        cur = Chunk{};
        shp = StepShape{};
      };
      for (int sc = 0; sc < 3; ++sc)
        for (int i : rows[sc]) {
          const int c = count(i, fwd);
          StepShape t = shp;
          if (sc == 0) { ++t.n32; t.e32 += c; }
          if (sc == 1) { ++t.n64; t.e64 += c; }
          if (sc == 2) { ++t.nlong; t.elong += c; }
          if (t.nrows() > kMaxStepRows || rec_layout(t, fwd).lds > kRecBytes) {
            flush();
            t = StepShape{};
            if (sc == 0) { t.n32 = 1; t.e32 = c; }
            if (sc == 1) { t.n64 = 1; t.e64 = c; }
            if (sc == 2) { t.nlong = 1; t.elong = c; }
          }
          if (rec_layout(t, fwd).lds > kRecBytes) {
            // a long row too big for one buffer: consecutive one-row pieces
            int per = c;
            StepShape one;
            one.nlong = 1;
            do {
              one.elong = per;
              if (rec_layout(one, fwd).lds <= kRecBytes) break;
              per = (per + 1) / 2;
            } while (true);
            const int np = (c + per - 1) / per;
            for (int k = 0; k < np; ++k) {
              Chunk pc;
              pc.rows = {i};
              pc.piece = (k == 0) ? kPieceFirst : (k == np - 1 ? kPieceLast : kPieceMiddle);
              pc.e0 = k * per;
              pc.e1 = std::min(c, (k + 1) * per);
              out.push_back(pc);
            }
            continue;
          }
          cur.rows.push_back(i);
          if (sc == 0) ++cur.n32;
          if (sc == 1) ++cur.n64;
          shp = t;
        }
      flush();
    }
    return out;
  };
  const std::vector<Chunk> fch0 = make_chunks(true, lf, maxf), bch0 = make_chunks(false, lb, maxb);
  // LDS slots by linear scan over steps
  auto allocate = [&](const std::vector<Chunk> &ch, bool fwd, std::vector<int32_t> &slot, std::vector<int32_t> &last) {
    std::vector<int32_t> stp(S.n);
    for (size_t k = 0; k < ch.size(); ++k)
      for (int i : ch[k].rows) stp[i] = (int32_t)k;
    last.assign(S.n, -1);
    for (int i = 0; i < S.n; ++i)
      for (int e = S.rp[i]; e < S.rp[i + 1]; ++e) {
        const int c = S.ci[e];
        if (fwd ? c < i : c > i) last[c] = std::max(last[c], stp[i]);
      }
    slot.assign(S.n, -1);
    std::vector<std::pair<int32_t, int32_t>> heap;  // (last use, slot), min-heap
    std::vector<int32_t> freel;
    for (int q = kVecSlots - kFillSlots - 1; q >= 0; --q) freel.push_back(q);
    auto cmp = [](const std::pair<int32_t, int32_t> &a, const std::pair<int32_t, int32_t> &b) { return a > b; };
    for (size_t k = 0; k < ch.size(); ++k) {
      while (!heap.empty() && heap.front().first < (int32_t)k) {
        freel.push_back(heap.front().second);
        std::pop_heap(heap.begin(), heap.end(), cmp);
        heap.pop_back();
      }
      for (int i : ch[k].rows) {
        if (last[i] <= (int32_t)k) continue;
        if (freel.empty()) {
          ++S.spilled;
          continue;
        }
        slot[i] = freel.back();
        freel.pop_back();
        heap.push_back({last[i], slot[i]});
        std::push_heap(heap.begin(), heap.end(), cmp);
      }
    }
  };
  std::vector<int32_t> fslot, flast, bslot, blast;
  allocate(fch0, true, fslot, flast);
  allocate(bch0, false, bslot, blast);
  // Entries of a chunk (row-relative CSR entry lists, piece ranges applied).
  auto chunk_entries = [&](const Chunk &c, bool fwd) {
    std::vector<std::vector<int32_t>> ent(c.rows.size());
    for (size_t j = 0; j < c.rows.size(); ++j) {
      const int i = c.rows[j];
      for (int e = S.rp[i]; e < S.rp[i + 1]; ++e)
        if (fwd ? S.ci[e] < i : S.ci[e] > i) ent[j].push_back(e);
      if (c.piece != kPieceWhole) ent[j] = std::vector<int32_t>(ent[j].begin() + c.e0, ent[j].begin() + c.e1);
    }
    return ent;
  };
  // Splits a chunk so that no part reads more than kFillSlots values that
  // have no LDS slot: rows of a step are independent, and a long row splits
  // into further pieces.
  auto split_for_fills = [&](const Chunk &c, bool fwd, const std::vector<int32_t> &slot) {
    auto add_spilled = [&](int e, std::vector<int32_t> &set) {
      const int col = S.ci[e];
      if (slot[col] < 0 && std::find(set.begin(), set.end(), col) == set.end()) set.push_back(col);
    };
    std::vector<Chunk> out;
    auto split_row = [&](const Chunk &c1) {
      const int i = c1.rows[0];
      std::vector<int32_t> all;
      for (int e = S.rp[i]; e < S.rp[i + 1]; ++e)
        if (fwd ? S.ci[e] < i : S.ci[e] > i) all.push_back(e);
      const int lo = c1.piece == kPieceWhole ? 0 : c1.e0;
      const int hi = c1.piece == kPieceWhole ? (int)all.size() : c1.e1;
      std::vector<std::pair<int, int>> ranges;
      std::vector<int32_t> set;
      int start = lo;
      for (int q = lo; q < hi; ++q) {
        std::vector<int32_t> t = set;
        add_spilled(all[q], t);
        if ((int)t.size() > kFillSlots) {
          ranges.push_back({start, q});
          start = q;
          t.clear();
          add_spilled(all[q], t);
        }
        set = t;
      }
      ranges.push_back({start, hi});
      if (ranges.size() == 1) {
        out.push_back(c1);
        return;
      }
      const bool open = (c1.piece == kPieceWhole || c1.piece == kPieceFirst);
      const bool close = (c1.piece == kPieceWhole || c1.piece == kPieceLast);
      for (size_t k = 0; k < ranges.size(); ++k) {
        Chunk p;
        p.rows = c1.rows;
        p.e0 = ranges[k].first;
        p.e1 = ranges[k].second;
        p.piece = (k == 0 && open) ? kPieceFirst : ((k + 1 == ranges.size() && close) ? kPieceLast : kPieceMiddle);
        out.push_back(p);
      }
    };
    const auto ent = chunk_entries(c, fwd);
    std::vector<int32_t> total;
    for (const auto &es : ent)
      for (int e : es) add_spilled(e, total);
    if ((int)total.size() <= kFillSlots) return std::vector<Chunk>{c};
    if (c.rows.size() == 1) {
      Chunk one = c;
      one.n32 = one.n64 = 0;  // a split row is always handled as a long row
      split_row(one);
      return out;
    }
    // several whole rows: greedy groups of consecutive rows
    Chunk cur;
    std::vector<int32_t> set;
    auto flush = [&]() {
      if (cur.rows.size() == 1 && cur.n32 + cur.n64 == 0) split_row(cur);
      else if (!cur.rows.empty()) out.push_back(cur);
      cur = Chunk{};
    };
    for (size_t j = 0; j < c.rows.size(); ++j) {
      std::vector<int32_t> t = set;
      for (int e : ent[j]) add_spilled(e, t);
      if ((int)t.size() > kFillSlots && !cur.rows.empty()) {
        flush();
        t.clear();
        for (int e : ent[j]) add_spilled(e, t);
      }
      cur.rows.push_back(c.rows[j]);
      if ((int)j < c.n32) ++cur.n32;
      else if ((int)j < c.n32 + c.n64) ++cur.n64;
      set = t;
    }
    flush();
    return out;
  };
  std::vector<Chunk> fch, bch;
  for (const Chunk &c : fch0)
    for (Chunk &q : split_for_fills(c, true, fslot)) fch.push_back(std::move(q));
  for (const Chunk &c : bch0)
    for (Chunk &q : split_for_fills(c, false, bslot)) bch.push_back(std::move(q));
  for (const std::vector<Chunk> *ch : {&fch, &bch})
    for (const Chunk &c : *ch) S.split_rows += (c.piece == kPieceFirst);
  // positions: rows of a step are consecutive, in the step's row order
  std::vector<int32_t> fpos(S.n), bpos(S.n);
  int p = 0;
  for (const Chunk &c : fch) {
    if (c.piece != kPieceWhole && c.piece != kPieceFirst) continue;
    S.fst.push_back(Step{p, (int32_t)c.rows.size()});
    for (int i : c.rows) {
      fpos[i] = p++;
      S.frow.push_back(i);
      S.fsrc.push_back(i < S.nfine ? S.cells[i] : -(1 + (i - S.nfine)));
    }
  }
  p = 0;
  for (const Chunk &c : bch) {
    if (c.piece != kPieceWhole && c.piece != kPieceFirst) continue;
    for (int i : c.rows) bpos[i] = p++;
  }
  S.bpos = bpos;
  // Records.  Before a step that reads values without an LDS slot, a fill
  // step reloads them from the global vector into the fill slots; empty
  // steps keep that reload at least two steps after the values' producers.
  auto emit = [&](const std::vector<Chunk> &ch, bool fwd, std::vector<RecStep> &out) {
    const std::vector<int32_t> &slot = fwd ? fslot : bslot;
    const std::vector<int32_t> &last = fwd ? flast : blast;
    std::vector<int32_t> made(S.n, -1);  // emitted step that produced each row
    auto push_record = [&](const RecHead &h, int32_t total, int32_t pos, int32_t nrows) -> uint8_t * {
      RecStep st{};
      st.rec = (int32_t)S.rec.size();
      st.len = total / 16;
      st.pos = pos;
      st.nrows = nrows;
      S.rec.resize(S.rec.size() + total, 0);
      uint8_t *base = S.rec.data() + st.rec;
      std::memcpy(base, &h, sizeof h);
      out.push_back(st);
      return base;
    };
    auto add_slot = [&](int32_t e, int64_t base, int32_t stride, bool f32) {
      S.rl_src.push_back(e);
      S.rl_base.push_back((int32_t)base);
      S.rl_stride.push_back(stride);
      S.rl_to32.push_back((uint8_t)f32);
    };
    std::vector<int32_t> fill_of(S.n, -1);  // fill slot of a value for the current step
    for (const Chunk &c : ch) {
      const int nr = (int)c.rows.size();
      const auto ent = chunk_entries(c, fwd);
      const int32_t pos0 = fwd ? fpos[c.rows[0]] : bpos[c.rows[0]];
      StepShape shp;
      shp.n32 = c.n32;
      shp.n64 = c.n64;
      shp.nlong = nr - c.n32 - c.n64;
      std::vector<int32_t> fills;  // columns to reload, in first-use order
      int32_t newest = -1;
      for (int j = 0; j < nr; ++j) {
        const int ne = (int)ent[j].size();
        if (j < c.n32) shp.e32 += ne;
        else if (j < c.n32 + c.n64) shp.e64 += ne;
        else shp.elong += ne;
        for (int e : ent[j]) {
          const int col = S.ci[e];
          if (slot[col] >= 0 || fill_of[col] >= 0) continue;
          fill_of[col] = (int32_t)fills.size();
          fills.push_back(col);
          newest = std::max(newest, made[col]);
        }
      }
      if (!fills.empty()) {
        // the fill step (index out.size()) must come two steps after the
        // newest producer
        while ((int32_t)out.size() < newest + 2) {
          RecHead e{};
          e.pos = out.empty() ? pos0 : out.back().pos;
          e.in = rec_in_offset(kRecHead);
          push_record(e, kRecHead, e.pos, 0);
        }
        RecHead f{};
        f.pos = out.empty() ? pos0 : out.back().pos;
        f.nfill = (int32_t)fills.size();
        f.fill = kRecHead;
        const int32_t total = kRecHead + align16((int64_t)8 * fills.size());
        f.in = rec_in_offset(total);
        uint8_t *fb = push_record(f, total, f.pos, 0);
        int32_t *fl = reinterpret_cast<int32_t *>(fb + kRecHead);
        for (size_t q = 0; q < fills.size(); ++q) {
          fl[2 * q] = bpos[fills[q]];
          fl[2 * q + 1] = kVecSlots - kFillSlots + (int32_t)q;
        }
      }
      const RecLayout L = rec_layout(shp, fwd);
      RecHead h{};
      h.nrows = nr;
      h.n32 = c.n32;
      h.n64 = c.n64;
      h.piece = c.piece;
      h.nslots32 = shp.e32;
      h.nslots64 = shp.e64;
      h.pos = pos0;
      h.in = rec_in_offset(L.total);
      h.slots32 = L.slots32;
      h.slots64 = L.slots64;
      h.vals32 = L.vals32;
      h.vals64 = L.vals64;
      h.lvals = L.lvals;
      h.ldeps = L.ldeps;
      h.lrptr = L.lrptr;
      h.dinv32 = L.dinv32;
      h.dinv64 = L.dinv64;
      // jagged-diagonal starts of the short sections
      auto diag_starts = [&](int j0, int j1, int32_t *koff) {
        int width = 0;
        for (int j = j0; j < j1; ++j) width = std::max(width, (int)ent[j].size());
        int q = 0;
        for (int k = 0; k <= kMaxJdsWidth; ++k) {
          koff[k] = q;
          if (k < width)
            for (int j = j0; j < j1 && k < (int)ent[j].size(); ++j) ++q;
        }
      };
      diag_starts(0, c.n32, h.koff32);
      diag_starts(c.n32, c.n32 + c.n64, h.koff64);
      uint8_t *base = push_record(h, L.total, h.pos, nr);
      const int32_t rec0 = out.back().rec;
      int32_t *ldeps = reinterpret_cast<int32_t *>(base + L.ldeps);
      int32_t *lrptr = reinterpret_cast<int32_t *>(base + L.lrptr);
      auto dep_of = [&](int col) { return slot[col] >= 0 ? slot[col] : kVecSlots - kFillSlots + fill_of[col]; };
      for (int j = 0; j < nr; ++j) {
        const int i = c.rows[j];
        int32_t *m = reinterpret_cast<int32_t *>(base + kRecHead + (int64_t)kRecRowBytes * j);
        // flags: bit 0 = store to the global vector, bit 1 = the input is a
        // cell value of r (forward fine rows: scaled by the basis scale)
        int flags;
        if (fwd) {
          flags = 1 | (i < S.nfine ? 2 : 0);
          m[1] = bpos[i];
        } else {
          const bool fine = i < S.nfine;
          m[1] = (restricted && fine && owner[S.cells[i]] == sub) ? S.cells[i] : -1;
          flags = ((slot[i] < 0 && last[i] >= 0) || (!restricted && fine)) ? 1 : 0;
        }
        m[0] = (int32_t)((uint32_t)(slot[i] >= 0 ? slot[i] : kRecNoSlot) | ((uint32_t)flags << 16) |
                         ((uint32_t)ent[j].size() << 18));
        if (j < c.n32 + c.n64) {
          // dependency slots in the order of the section's values
          const bool f32 = j < c.n32;
          const int32_t *koff = f32 ? h.koff32 : h.koff64;
          uint16_t *dp = reinterpret_cast<uint16_t *>(base + (f32 ? L.slots32 : L.slots64));
          const int i_sec = f32 ? j : j - c.n32;
          for (size_t k = 0; k < ent[j].size(); ++k) dp[koff[k] + i_sec] = (uint16_t)dep_of(S.ci[ent[j][k]]);
        }
        if (c.piece == kPieceWhole || c.piece == kPieceLast) made[i] = (int)out.size() - 1;
      }
      // short sections: jagged diagonals, structure of arrays
      // (granule layout: the relayout stride packs the entry count and the entry)
      auto short_vals = [&](int j0, int j1, const int32_t *koff, int32_t off, int nslots, bool f32) {
        const int sz = f32 ? 4 : 8;
        const int64_t vbase = (rec0 + off) / sz;
        for (int k = 0; k < kMaxJdsWidth; ++k)
          for (int j = j0; j < j1 && k < (int)ent[j].size(); ++j) {
            const int32_t q = koff[k] + (j - j0);
            S.rl_src.push_back(ent[j][k]);
            S.rl_base.push_back((int32_t)vbase);
            S.rl_stride.push_back(nslots | (q << 16));
            S.rl_to32.push_back((uint8_t)((f32 ? 1 : 0) | 2));
          }
      };
      short_vals(0, c.n32, h.koff32, L.vals32, shp.e32, true);
      short_vals(c.n32, c.n32 + c.n64, h.koff64, L.vals64, shp.e64, false);
      // long section: 9 values per entry
      {
        const int64_t vbase = (rec0 + L.lvals) / 8;
        int q = 0;
        for (int j = c.n32 + c.n64; j < nr; ++j) {
          lrptr[j - c.n32 - c.n64] = q;
          for (int e : ent[j]) {
            ldeps[q] = dep_of(S.ci[e]);
            add_slot(e, vbase + 9 * q, 1, false);
            ++q;
          }
        }
        if (shp.nlong > 0) lrptr[shp.nlong] = q;
      }
      for (int col : fills) fill_of[col] = -1;
      if (!fwd) {
        const int64_t d32 = (rec0 + L.dinv32) / 4, d64 = (rec0 + L.dinv64) / 8;
        for (int j = 0; j < nr; ++j) {
          const int32_t dg = S.diag[c.rows[j]];
          if (j < c.n32) add_slot(dg, d32 + j, c.n32, true);
          else add_slot(dg, d64 + (j - c.n32), nr - c.n32, false);
        }
      }
    }
  };
  emit(fch, true, S.rf);
  emit(bch, false, S.rb);
}

}  // namespace

asm_status build_plan(const HostPattern &A, const asm_precond_opts &o, PlanHost &P, std::string &err) {
  const int nx = A.nx, ny = A.ny, nz = A.nz, N = A.N;
  const bool two = (o.kind == ASM_KIND_TWO_LEVEL);
  const int sx = o.sx, sy = o.sy, nsub = sx * sy;
  const int delta = o.overlap;
  const bool restricted = (o.combine == ASM_COMBINE_RESTRICTED);
  const bool fp32 = (o.precision == ASM_PREC_FP32);

  const Split xs = balanced(nx, sx), ys = balanced(ny, sy);
  std::vector<int32_t> owner(N);
  for (int c = 0; c < N; ++c) {
    const int ix = c / (ny * nz), iy = (c / nz) % ny;
    owner[c] = xs.part[ix] * sy + ys.part[iy];
  }
  auto face_nbr = [&](int a, int b) {
    const int ax = a / sy, ay = a % sy, bx = b / sy, by = b % sy;
    return std::abs(ax - bx) + std::abs(ay - by) == 1;
  };
  // Outside cells owned by a face neighbour form the near region, the rest
  // the far region; the far-field-only variant treats all as far, the
  // near-field-only variant drops the far region (Section 5).
  auto near_rel = [&](int a, int b) { return o.field != ASM_FIELD_FAR && face_nbr(a, b); };
  const bool keep_far = (o.field != ASM_FIELD_NEAR);

  const Csr G = undirected(A);

  // ---------------------------------------------------------------- fine sets
  std::vector<std::vector<int32_t>> F(nsub);
#pragma omp parallel
  {
    std::vector<int32_t> dist(N, -1), queue;
#pragma omp for schedule(dynamic)
    for (int s = 0; s < nsub; ++s) {
      const int px = s / sy, py = s % sy;
      queue.clear();
      for (int ix = xs.start[px]; ix < xs.start[px + 1]; ++ix)
        for (int iy = ys.start[py]; iy < ys.start[py + 1]; ++iy)
          for (int iz = 0; iz < nz; ++iz) {
            const int c = (ix * ny + iy) * nz + iz;
            dist[c] = 0;
            queue.push_back(c);
          }
      for (size_t h = 0; h < queue.size(); ++h) {
        const int c = queue[h];
        if (dist[c] >= delta) continue;
        for (int t = G.ptr[c]; t < G.ptr[c + 1]; ++t) {
          const int d = G.idx[t];
          if (dist[d] < 0) {
            dist[d] = dist[c] + 1;
            queue.push_back(d);
          }
        }
      }
      F[s] = queue;
      std::sort(F[s].begin(), F[s].end());
      for (int c : queue) dist[c] = -1;
    }
  }

  // ---------------------------------------------------------------- atoms
  Atoms at;
  const Transpose T = two ? transpose(A) : Transpose{};
  if (two) {
    at.on = true;
    const int *nb = o.near_box, *fb = o.far_box;
    const int nbny = (ny + nb[1] - 1) / nb[1], nbnz = (nz + nb[2] - 1) / nb[2];
    const int fbny = (ny + fb[1] - 1) / fb[1], fbnz = (nz + fb[2] - 1) / fb[2];
    at.nbn = ((nx + nb[0] - 1) / nb[0]) * nbny * nbnz;
    at.nbf = ((nx + fb[0] - 1) / fb[0]) * fbny * fbnz;
    at.nbox.resize(N);
    at.fbox.resize(N);
    for (int c = 0; c < N; ++c) {
      const int ix = c / (ny * nz), iy = (c / nz) % ny, iz = c % nz;
      at.nbox[c] = ((ix / nb[0]) * nbny + iy / nb[1]) * nbnz + iz / nb[2];
      at.fbox[c] = ((ix / fb[0]) * fbny + iy / fb[1]) * fbnz + iz / fb[2];
    }
    // membership of each cell in the fine sets of subdomains other than its owner
    Csr sig;
    sig.ptr.assign(N + 1, 0);
    for (int s = 0; s < nsub; ++s)
      for (int c : F[s])
        if (owner[c] != s) sig.ptr[c + 1]++;
    for (int c = 0; c < N; ++c) sig.ptr[c + 1] += sig.ptr[c];
    sig.idx.resize(sig.ptr[N]);
    {
      std::vector<int32_t> fill(sig.ptr.begin(), sig.ptr.end() - 1);
      for (int s = 0; s < nsub; ++s)
        for (int c : F[s])
          if (owner[c] != s) sig.idx[fill[c]++] = s;
    }
    // ids of the full / near-part / far-part signature lists
    std::map<std::vector<int32_t>, int32_t> sig_ids;
    sig_ids[{}] = 0;
    std::vector<std::vector<int32_t>> sig_list{{}};
    auto sig_id = [&](const std::vector<int32_t> &v) {
      auto it = sig_ids.find(v);
      if (it != sig_ids.end()) return it->second;
      const int32_t id = (int32_t)sig_list.size();
      sig_ids.emplace(v, id);
      sig_list.push_back(v);
      return id;
    };
    std::vector<int32_t> sfull(N), snear(N), sfar(N);
    std::vector<int32_t> tmp, tn, tf;
    for (int c = 0; c < N; ++c) {
      if (sig.ptr[c] == sig.ptr[c + 1]) {
        sfull[c] = snear[c] = sfar[c] = 0;
        continue;
      }
      tmp.assign(sig.idx.begin() + sig.ptr[c], sig.idx.begin() + sig.ptr[c + 1]);
      tn.clear();
      tf.clear();
      for (int s : tmp) (near_rel(s, owner[c]) ? tn : tf).push_back(s);
      sfull[c] = sig_id(tmp);
      snear[c] = sig_id(tn);
      sfar[c] = sig_id(tf);
    }
    const int64_t ns = nsub;
    std::vector<std::pair<int64_t, int64_t>> kA(N), kN(N), kF(N);
    for (int c = 0; c < N; ++c) {
      kA[c] = {((int64_t)at.nbox[c] * at.nbf + at.fbox[c]) * ns + owner[c], sfull[c]};
      kN[c] = {(int64_t)at.nbox[c] * ns + owner[c], snear[c]};
      kF[c] = {(int64_t)at.fbox[c] * ns + owner[c], sfar[c]};
    }
    std::vector<int32_t> cN, cF;
#pragma omp parallel sections
    {
#pragma omp section
      at.cell_atom = compact_ids(kA, at.nA);
#pragma omp section
      cN = compact_ids(kN, at.nNa);
#pragma omp section
      cF = compact_ids(kF, at.nFa);
    }
    at.a_near.assign(at.nA, -1);
    at.a_far.assign(at.nA, -1);
    at.na_box.assign(at.nNa, 0);
    at.na_owner.assign(at.nNa, 0);
    at.fa_box.assign(at.nFa, 0);
    at.fa_owner.assign(at.nFa, 0);
    std::vector<int32_t> na_sigid(at.nNa, 0), fa_sigid(at.nFa, 0);
    for (int c = 0; c < N; ++c) {
      const int a = at.cell_atom[c];
      at.a_near[a] = cN[c];
      at.a_far[a] = cF[c];
      at.na_box[cN[c]] = at.nbox[c];
      at.na_owner[cN[c]] = owner[c];
      na_sigid[cN[c]] = snear[c];
      at.fa_box[cF[c]] = at.fbox[c];
      at.fa_owner[cF[c]] = owner[c];
      fa_sigid[cF[c]] = sfar[c];
    }
    auto sig_csr = [&](const std::vector<int32_t> &ids, Csr &out) {
      out.ptr.assign(ids.size() + 1, 0);
      for (size_t i = 0; i < ids.size(); ++i) out.ptr[i + 1] = out.ptr[i] + (int32_t)sig_list[ids[i]].size();
      out.idx.resize(out.ptr.back());
      for (size_t i = 0; i < ids.size(); ++i)
        std::copy(sig_list[ids[i]].begin(), sig_list[ids[i]].end(), out.idx.begin() + out.ptr[i]);
    };
    sig_csr(na_sigid, at.na_sig);
    sig_csr(fa_sigid, at.fa_sig);
    auto by_owner = [&](const std::vector<int32_t> &own, Csr &out) {
      out.ptr.assign(nsub + 1, 0);
      for (int32_t o2 : own) out.ptr[o2 + 1]++;
      for (int s = 0; s < nsub; ++s) out.ptr[s + 1] += out.ptr[s];
      out.idx.resize(own.size());
      std::vector<int32_t> fill(out.ptr.begin(), out.ptr.end() - 1);
      for (size_t i = 0; i < own.size(); ++i) out.idx[fill[own[i]]++] = (int32_t)i;
    };
    by_owner(at.na_owner, at.owner_na);
    by_owner(at.fa_owner, at.owner_fa);

    // L1: fine-atom lumped matrix, sources = A blocks
    std::vector<std::array<int32_t, 3>> t1;
    t1.reserve(A.nnzb);
    for (int r = 0; r < N; ++r)
      for (int e = A.rp[r]; e < A.rp[r + 1]; ++e) t1.push_back({at.cell_atom[r], at.cell_atom[A.ci[e]], e});
    std::vector<int32_t> l1ptr, l1col;
    triples_to_csr(t1, at.nA, l1ptr, l1col, P.l1);
    t1.clear();
    t1.shrink_to_fit();
    // L2: near/far atom matrices, sources = L1 entries.  Pool order NN, NF, FN, FF.
    Atoms::M *mats[4] = {&at.nn, &at.nf, &at.fn, &at.ff};
    int32_t pool = 0;
    for (int m = 0; m < 4; ++m) {
      const bool rn = (m < 2), cn = (m % 2 == 0);
      std::vector<std::array<int32_t, 3>> t2;
      for (int a = 0; a < at.nA; ++a)
        for (int q = l1ptr[a]; q < l1ptr[a + 1]; ++q) {
          const int b = l1col[q];
          t2.push_back({rn ? at.a_near[a] : at.a_far[a], cn ? at.a_near[b] : at.a_far[b], q});
        }
      GatherList g;
      triples_to_csr(t2, rn ? at.nNa : at.nFa, mats[m]->ptr, mats[m]->col, g);
      mats[m]->pos.resize(mats[m]->col.size());
      for (size_t i = 0; i < mats[m]->col.size(); ++i) mats[m]->pos[i] = pool + (int32_t)i;
      pool += (int32_t)mats[m]->col.size();
      for (int32_t d = 0; d < g.size(); ++d) {
        for (int q = g.ptr[d]; q < g.ptr[d + 1]; ++q) P.l2.idx.push_back(g.idx[q]);
        P.l2.ptr.push_back((int32_t)P.l2.idx.size());
      }
    }
    // right-hand side lumping: fine-atom sums of cells, then N/F atoms
    {
      // cells of each fine atom, ascending
      P.c1.ptr.assign(at.nA + 1, 0);
      for (int c = 0; c < N; ++c) P.c1.ptr[at.cell_atom[c] + 1]++;
      for (int a = 0; a < at.nA; ++a) P.c1.ptr[a + 1] += P.c1.ptr[a];
      P.c1.idx.resize(N);
      {
        std::vector<int32_t> cur(P.c1.ptr.begin(), P.c1.ptr.end() - 1);
        for (int c = 0; c < N; ++c) P.c1.idx[cur[at.cell_atom[c]]++] = c;
      }
      // c2 destinations: [N-atoms | F-atoms]
      std::vector<std::vector<int32_t>> nsrc(at.nNa), fsrc(at.nFa);
      for (int a = 0; a < at.nA; ++a) {
        nsrc[at.a_near[a]].push_back(a);
        fsrc[at.a_far[a]].push_back(a);
      }
      for (auto &v : nsrc) {
        P.c2.idx.insert(P.c2.idx.end(), v.begin(), v.end());
        P.c2.ptr.push_back((int32_t)P.c2.idx.size());
      }
      P.c2.split = at.nNa;
      for (auto &v : fsrc) {
        P.c2.idx.insert(P.c2.idx.end(), v.begin(), v.end());
        P.c2.ptr.push_back((int32_t)P.c2.idx.size());
      }
    }
  }

  // ---------------------------------------------------------------- per subdomain
  std::vector<SubLocal> L(nsub);
  const int64_t nnzbA = A.nnzb;
#pragma omp parallel
  {
    std::vector<int32_t> loc(N, -1);
    std::vector<int32_t> nvar(two ? at.nbn : 0, -1), fvar(two ? at.nbf : 0, -1);
    std::vector<int32_t> pos;
    std::vector<std::array<int32_t, 3>> trip;
#pragma omp for schedule(dynamic)
    for (int s = 0; s < nsub; ++s) {
      SubLocal &S = L[s];
      S.cells = F[s];
      S.nfine = (int32_t)S.cells.size();
      S.owned.resize(S.nfine);
      for (int u = 0; u < S.nfine; ++u) {
        loc[S.cells[u]] = u;
        S.owned[u] = (owner[S.cells[u]] == s);
      }
      std::vector<int32_t> near_boxes, far_boxes;
      std::vector<std::vector<int32_t>> near_members, far_members;  // atoms per var
      if (two) {
        // coarse variables: near boxes of face-neighbour owners, far boxes
        // elsewhere, each restricted to atoms not fine for s
        for (int o2 = 0; o2 < nsub; ++o2) {
          if (o2 == s) continue;
          if (near_rel(o2, s)) {
            for (int t = at.owner_na.ptr[o2]; t < at.owner_na.ptr[o2 + 1]; ++t) {
              const int a = at.owner_na.idx[t];
              if (!contains(at.na_sig, a, s)) near_boxes.push_back(at.na_box[a]);
            }
          } else if (keep_far) {
            for (int t = at.owner_fa.ptr[o2]; t < at.owner_fa.ptr[o2 + 1]; ++t) {
              const int a = at.owner_fa.idx[t];
              if (!contains(at.fa_sig, a, s)) far_boxes.push_back(at.fa_box[a]);
            }
          }
        }
        std::sort(near_boxes.begin(), near_boxes.end());
        near_boxes.erase(std::unique(near_boxes.begin(), near_boxes.end()), near_boxes.end());
        std::sort(far_boxes.begin(), far_boxes.end());
        far_boxes.erase(std::unique(far_boxes.begin(), far_boxes.end()), far_boxes.end());
        for (size_t i = 0; i < near_boxes.size(); ++i) nvar[near_boxes[i]] = S.nfine + (int32_t)i;
        for (size_t i = 0; i < far_boxes.size(); ++i)
          fvar[far_boxes[i]] = S.nfine + (int32_t)near_boxes.size() + (int32_t)i;
        S.ncoarse = (int32_t)(near_boxes.size() + far_boxes.size());
        near_members.assign(near_boxes.size(), {});
        far_members.assign(far_boxes.size(), {});
      }
      S.n = S.nfine + S.ncoarse;
      auto is_fine = [&](int c) { return loc[c] >= 0; };
      auto label = [&](int c) -> int32_t {
        if (loc[c] >= 0) return loc[c];
        if (!two) return -1;
        const int o2 = owner[c];
        return near_rel(o2, s) ? nvar[at.nbox[c]] : keep_far ? fvar[at.fbox[c]] : -1;
      };
      trip.clear();
      // (a) fine rows: every block of the cell's row
      for (int u = 0; u < S.nfine; ++u) {
        const int a = S.cells[u];
        for (int e = A.rp[a]; e < A.rp[a + 1]; ++e) {
          const int v = label(A.ci[e]);
          if (v >= 0) trip.push_back({u, v, e});
        }
      }
      if (two) {
        // (b) coarse rows against fine columns, from A's blocks
        for (int u = 0; u < S.nfine; ++u) {
          const int d = S.cells[u];
          for (int t = T.ptr[d]; t < T.ptr[d + 1]; ++t) {
            const int a = T.row[t];
            if (is_fine(a)) continue;
            const int32_t la = label(a);
            if (la >= 0) trip.push_back({la, u, T.ent[t]});
          }
        }
        // (c) coarse against coarse, from the shared lumped atom matrices
        auto near_ok = [&](int na) { return near_rel(at.na_owner[na], s) && !contains(at.na_sig, na, s); };
        auto far_ok = [&](int fa) {
          const int o2 = at.fa_owner[fa];
          return keep_far && o2 != s && !near_rel(o2, s) && !contains(at.fa_sig, fa, s);
        };
        for (int o2 = 0; o2 < nsub; ++o2) {
          if (o2 == s) continue;
          if (near_rel(o2, s)) {
            for (int t = at.owner_na.ptr[o2]; t < at.owner_na.ptr[o2 + 1]; ++t) {
              const int a = at.owner_na.idx[t];
              if (!near_ok(a)) continue;
              const int u = nvar[at.na_box[a]];
              near_members[u - S.nfine].push_back(a);
              for (int q = at.nn.ptr[a]; q < at.nn.ptr[a + 1]; ++q)
                if (near_ok(at.nn.col[q])) trip.push_back({u, nvar[at.na_box[at.nn.col[q]]], (int32_t)(nnzbA + at.nn.pos[q])});
              for (int q = at.nf.ptr[a]; q < at.nf.ptr[a + 1]; ++q)
                if (far_ok(at.nf.col[q])) trip.push_back({u, fvar[at.fa_box[at.nf.col[q]]], (int32_t)(nnzbA + at.nf.pos[q])});
            }
          } else {
            for (int t = at.owner_fa.ptr[o2]; t < at.owner_fa.ptr[o2 + 1]; ++t) {
              const int a = at.owner_fa.idx[t];
              if (!far_ok(a)) continue;
              const int u = fvar[at.fa_box[a]];
              far_members[u - S.nfine - near_boxes.size()].push_back(a);
              for (int q = at.fn.ptr[a]; q < at.fn.ptr[a + 1]; ++q)
                if (near_ok(at.fn.col[q])) trip.push_back({u, nvar[at.na_box[at.fn.col[q]]], (int32_t)(nnzbA + at.fn.pos[q])});
              for (int q = at.ff.ptr[a]; q < at.ff.ptr[a + 1]; ++q)
                if (far_ok(at.ff.col[q])) trip.push_back({u, fvar[at.fa_box[at.ff.col[q]]], (int32_t)(nnzbA + at.ff.pos[q])});
            }
          }
        }
        // coarse right-hand sides: sums of the member atoms' lumped values
        S.cptr.assign(1, 0);
        for (auto &m : near_members) {
          std::sort(m.begin(), m.end());
          S.cidx.insert(S.cidx.end(), m.begin(), m.end());
          S.cptr.push_back((int32_t)S.cidx.size());
        }
        for (auto &m : far_members) {
          std::sort(m.begin(), m.end());
          for (int a : m) S.cidx.push_back(at.nNa + a);
          S.cptr.push_back((int32_t)S.cidx.size());
        }
      }
      // CSR of A_i with value sources
      std::sort(trip.begin(), trip.end());
      S.rp.assign(S.n + 1, 0);
      S.sptr.assign(1, 0);
      for (size_t i = 0; i < trip.size(); ++i) {
        if (i == 0 || trip[i][0] != trip[i - 1][0] || trip[i][1] != trip[i - 1][1]) {
          S.ci.push_back(trip[i][1]);
          S.rp[trip[i][0] + 1]++;
          S.sptr.push_back(S.sptr.back());
        }
        S.sidx.push_back(trip[i][2]);
        S.sptr.back()++;
      }
      for (int u = 0; u < S.n; ++u) S.rp[u + 1] += S.rp[u];
      // diagonal positions
      S.diag.assign(S.n, -1);
      for (int u = 0; u < S.n; ++u)
        for (int e = S.rp[u]; e < S.rp[u + 1]; ++e)
          if (S.ci[e] == u) S.diag[u] = e;
      for (int u = 0; u < S.n; ++u)
        if (S.diag[u] < 0 && S.bad_row < 0) S.bad_row = u;
      // ILU(0) update pairs: row i, lower entry (i,k), upper entry (k,j)
      // with j in row i
      const int nnz = S.rp[S.n];
      pos.assign(S.n, -1);
      S.tptr.assign(nnz + 1, 0);
      for (int i = 0; i < S.n && S.bad_row < 0; ++i) {
        for (int e = S.rp[i]; e < S.rp[i + 1]; ++e) pos[S.ci[e]] = e;
        for (int e = S.rp[i]; e < S.rp[i + 1]; ++e) {
          const int k = S.ci[e];
          if (k >= i) break;
          for (int ek = S.diag[k] + 1; ek < S.rp[k + 1]; ++ek) {
            const int dst = pos[S.ci[ek]];
            if (dst < 0) continue;
            S.tdst.push_back(dst);
            S.tsrc.push_back(ek);
          }
          S.tptr[e + 1] = (int32_t)S.tdst.size();
        }
        for (int e = S.rp[i]; e < S.rp[i + 1]; ++e) pos[S.ci[e]] = -1;
      }
      // entries without pairs still need a monotone pointer
      for (int e = 0; e < nnz; ++e) S.tptr[e + 1] = std::max(S.tptr[e + 1], S.tptr[e]);
      // level schedules
      std::vector<int32_t> lf(S.n, 0), lb(S.n, 0);
      int maxf = 0, maxb = 0;
      for (int i = 0; i < S.n; ++i) {
        for (int e = S.rp[i]; e < S.rp[i + 1]; ++e)
          if (S.ci[e] < i) lf[i] = std::max(lf[i], lf[S.ci[e]] + 1);
        maxf = std::max(maxf, lf[i]);
      }
      for (int i = S.n - 1; i >= 0; --i) {
        for (int e = S.rp[i]; e < S.rp[i + 1]; ++e)
          if (S.ci[e] > i) lb[i] = std::max(lb[i], lb[S.ci[e]] + 1);
        maxb = std::max(maxb, lb[i]);
      }
      S.levels = std::max(maxf, maxb) + 1;
      build_sweeps(S, lf, maxf, lb, maxb, fp32, restricted, owner, s);
      for (int u = 0; u < S.nfine; ++u) loc[S.cells[u]] = -1;
      if (two) {
        for (int b : near_boxes) nvar[b] = -1;
        for (int b : far_boxes) fvar[b] = -1;
      }
    }
  }

  // ---------------------------------------------------------------- checks
  for (int s = 0; s < nsub; ++s)
    if (L[s].bad_row >= 0) {
      err = "subdomain " + std::to_string(s) + " local row " + std::to_string(L[s].bad_row) +
            " has no diagonal block";
      return ASM_ERR_INVALID;
    }

  // ---------------------------------------------------------------- concatenate
  P.nsub = nsub;
  P.sub.resize(nsub);
  std::vector<int64_t> o_ext(nsub), o_ent(nsub), o_t(nsub), o_as(nsub), o_coarse(nsub), o_cs(nsub), o_fst(nsub),
      o_rf(nsub), o_rb(nsub), o_rec(nsub), o_rl(nsub);
  int64_t ext = 0, ent = 0, tcount = 0, asrc = 0, coarse = 0, csrc = 0, fst = 0, nrf = 0, nrb = 0, recb = 0, nrl = 0;
  for (int s = 0; s < nsub; ++s) {
    const SubLocal &S = L[s];
    o_ext[s] = ext; o_ent[s] = ent; o_t[s] = tcount; o_as[s] = asrc; o_coarse[s] = coarse; o_cs[s] = csrc;
    o_fst[s] = fst; o_rf[s] = nrf; o_rb[s] = nrb; o_rec[s] = recb; o_rl[s] = nrl;
    ext += S.n; ent += S.rp[S.n]; tcount += (int64_t)S.tdst.size(); asrc += (int64_t)S.sidx.size();
    coarse += S.ncoarse; csrc += (int64_t)S.cidx.size(); fst += (int64_t)S.fst.size();
    nrf += (int64_t)S.rf.size(); nrb += (int64_t)S.rb.size(); recb += (int64_t)S.rec.size();
    nrl += (int64_t)S.rl_src.size();
    P.max_levels = std::max(P.max_levels, S.levels);
    P.fine_row_entries += S.rp[S.nfine];
    P.lds_spilled_rows += S.spilled;
    P.split_rows += S.split_rows;
  }
  const int64_t lim = (int64_t)1 << 31;
  if (ext >= lim || ent >= lim || tcount >= lim || asrc >= lim || recb / 4 >= lim || nrl >= lim) {
    err = "preconditioner too large for 32-bit indexing";
    return ASM_ERR_INVALID;
  }
  P.total_ext = ext;
  P.total_coarse = coarse;
  P.total_entries = ent;
  P.total_pos = ext;
  P.sweep_steps = nrf + nrb;
  P.fstep.resize(fst);
  P.frow.resize(ext);
  P.rf.resize(nrf);
  P.rb.resize(nrb);
  P.rec.assign(recb + kRecPadBytes, 0);
  P.fsrc.assign(ext + kSrcPad, 0);
  P.rhs_src.resize(ext);
  P.arp.resize(ext + 1);
  P.aci.resize(ent);
  P.adiag.resize(ext);
  P.tptr.resize(ent + 1);
  P.tdst.resize(tcount);
  P.tsrc.resize(tcount);
  P.asm_src.ptr.resize(ent + 1);
  P.asm_src.idx.resize(asrc);
  P.c3.ptr.resize(coarse + 1);
  P.c3.idx.resize(csrc);
  P.rl.src.resize(nrl);
  P.rl.base.resize(nrl);
  P.rl.stride.resize(nrl);
  P.rl.to32.resize(nrl);
#pragma omp parallel for schedule(dynamic)
  for (int s = 0; s < nsub; ++s) {
    SubLocal &S = L[s];
    SubDesc &d = P.sub[s];
    const int32_t pos_off = (int32_t)o_ext[s];  // forward / backward positions share the ext range
    d.ext_off = (int32_t)o_ext[s];
    d.n = S.n;
    d.nfine = S.nfine;
    d.fstep0 = (int32_t)o_fst[s];
    d.fstep1 = (int32_t)(o_fst[s] + S.fst.size());
    d.rf0 = (int32_t)o_rf[s];
    d.rf1 = (int32_t)(o_rf[s] + S.rf.size());
    d.rb0 = (int32_t)o_rb[s];
    d.rb1 = (int32_t)(o_rb[s] + S.rb.size());
    for (size_t k = 0; k < S.fst.size(); ++k) P.fstep[o_fst[s] + k] = Step{S.fst[k].pos + pos_off, S.fst[k].nrows};
    for (int q = 0; q < S.n; ++q) {
      P.frow[pos_off + q] = S.frow[q];
      const int32_t f = S.fsrc[q];
      P.fsrc[pos_off + q] = f >= 0 ? f : -(int32_t)(1 + o_coarse[s] + (-f - 1));
    }
    // records: shift positions (rows and reloads) by the subdomain offset
    uint8_t *rb = P.rec.data() + o_rec[s];
    std::copy(S.rec.begin(), S.rec.end(), rb);
    auto place = [&](const std::vector<RecStep> &loc, std::vector<RecStep> &glob, int64_t off, bool fwd) {
      for (size_t k = 0; k < loc.size(); ++k) {
        RecStep st = loc[k];
        RecHead h;
        std::memcpy(&h, rb + st.rec, sizeof h);
        // forward rows name their backward position (backward rows an
        // output cell, already global)
        if (fwd)
          for (int j = 0; j < h.nrows; ++j)
            reinterpret_cast<int32_t *>(rb + st.rec + kRecHead + (int64_t)kRecRowBytes * j)[1] += pos_off;
        int32_t *fl = reinterpret_cast<int32_t *>(rb + st.rec + h.fill);
        for (int q = 0; q < h.nfill; ++q) fl[2 * q] += pos_off;
        h.pos += pos_off;
        std::memcpy(rb + st.rec, &h, sizeof h);
        st.rec = (int32_t)((o_rec[s] + st.rec) / 16);
        st.pos += pos_off;
        glob[off + k] = st;
      }
    };
    place(S.rf, P.rf, o_rf[s], true);
    place(S.rb, P.rb, o_rb[s], false);
    // each record names the one kHeadAhead steps later in its sweep (the
    // last one past the end), where the streaming waves look it up
    auto link = [&](const std::vector<RecStep> &loc, const std::vector<RecStep> &glob, int64_t off) {
      const size_t n = loc.size();
      for (size_t k = 0; k < n; ++k) {
        RecHead h;
        std::memcpy(&h, rb + loc[k].rec, sizeof h);
        h.ahead = glob[off + std::min(k + kHeadAhead, n - 1)];
        std::memcpy(rb + loc[k].rec, &h, sizeof h);
      }
    };
    link(S.rf, P.rf, o_rf[s]);
    link(S.rb, P.rb, o_rb[s]);
    for (size_t t = 0; t < S.rl_src.size(); ++t) {
      const int sz = (S.rl_to32[t] & 1) ? 4 : 8;
      P.rl.src[o_rl[s] + t] = (int32_t)(o_ent[s] + S.rl_src[t]);
      P.rl.base[o_rl[s] + t] = (int32_t)(S.rl_base[t] + o_rec[s] / sz);
      P.rl.stride[o_rl[s] + t] = S.rl_stride[t];
      P.rl.to32[o_rl[s] + t] = S.rl_to32[t];
    }
    for (int u = 0; u < S.n; ++u) {
      const int64_t g = o_ext[s] + u;
      P.rhs_src[g] = (u < S.nfine) ? S.cells[u] : -(int32_t)(1 + o_coarse[s] + (u - S.nfine));
      P.arp[g] = (int32_t)(o_ent[s] + S.rp[u]);
      P.adiag[g] = (int32_t)(o_ent[s] + S.diag[u]);
    }
    const int nnz = S.rp[S.n];
    for (int e = 0; e < nnz; ++e) {
      P.aci[o_ent[s] + e] = S.ci[e];
      P.tptr[o_ent[s] + e] = (int32_t)(o_t[s] + S.tptr[e]);
      P.asm_src.ptr[o_ent[s] + e] = (int32_t)(o_as[s] + S.sptr[e]);
    }
    for (size_t t = 0; t < S.tdst.size(); ++t) {
      P.tdst[o_t[s] + t] = (int32_t)(o_ent[s] + S.tdst[t]);
      P.tsrc[o_t[s] + t] = (int32_t)(o_ent[s] + S.tsrc[t]);
    }
    std::copy(S.sidx.begin(), S.sidx.end(), P.asm_src.idx.begin() + o_as[s]);
    for (int q = 0; q < S.ncoarse; ++q) P.c3.ptr[o_coarse[s] + q] = (int32_t)(o_cs[s] + S.cptr[q]);
    std::copy(S.cidx.begin(), S.cidx.end(), P.c3.idx.begin() + o_cs[s]);
    // free the local copies early
    std::vector<uint8_t>().swap(S.rec);
  }
  if (o.local == ASM_LOCAL_EXACT) {
    P.xdoff.assign(nsub + 1, 0);
    for (int s = 0; s < nsub; ++s) {
      const int64_t n3 = 3 * (int64_t)L[s].n;
      if (n3 > ASM_EXACT_MAX_UNKNOWNS) {
        err = "exact local solve of subdomain " + std::to_string(s) + " has " + std::to_string(n3) +
              " unknowns, more than " + std::to_string(ASM_EXACT_MAX_UNKNOWNS);
        return ASM_ERR_INVALID;
      }
      P.xmaxn3 = std::max<int32_t>(P.xmaxn3, (int32_t)n3);
      P.xdoff[s + 1] = P.xdoff[s] + n3 * n3;
    }
    if (P.xdoff[nsub] * 8 > ((int64_t)8 << 30)) {
      err = "exact local solves need more than 8 GiB of dense inverses";
      return ASM_ERR_INVALID;
    }
    P.xlpos.resize(ext);
    P.xpsub.resize(ext);
    P.xout.resize(ext);
    P.xbpos.resize(ext);
    for (int s = 0; s < nsub; ++s) {
      const SubLocal &S = L[s];
      for (int q = 0; q < S.n; ++q) {
        const int u = S.frow[q];
        const int64_t g = o_ext[s];
        P.xlpos[g + u] = q;
        P.xpsub[g + q] = s;
        P.xout[g + q] = (u < S.nfine && S.owned[u]) ? S.cells[u] : -1;
        P.xbpos[g + q] = (int32_t)(g + S.bpos[u]);
      }
    }
  }
  P.arp[ext] = (int32_t)ent;
  P.tptr[ent] = (int32_t)tcount;
  P.asm_src.ptr[ent] = (int32_t)asrc;
  P.c3.ptr[coarse] = (int32_t)csrc;
  // additive combine: backward positions of each cell's fine rows, in subdomain order
  P.cptr.assign(N + 1, 0);
  for (int s = 0; s < nsub; ++s)
    for (int c : L[s].cells) P.cptr[c + 1]++;
  for (int c = 0; c < N; ++c) P.cptr[c + 1] += P.cptr[c];
  P.cidx.resize(P.cptr[N]);
  {
    std::vector<int32_t> fill(P.cptr.begin(), P.cptr.end() - 1);
    for (int s = 0; s < nsub; ++s)
      for (int u = 0; u < L[s].nfine; ++u) P.cidx[fill[L[s].cells[u]]++] = (int32_t)(o_ext[s] + L[s].bpos[u]);
  }
  P.any_fp32 = fp32;
  // ---------------------------------------------------------------- global coarse grid
  if (o.coarse != ASM_COARSE_NONE) {
    const int *cb = o.coarse_box;
    const int cby = (ny + cb[1] - 1) / cb[1], cbz = (nz + cb[2] - 1) / cb[2];
    const int64_t ncv = (int64_t)((nx + cb[0] - 1) / cb[0]) * cby * cbz;  // clipped boxes are never empty
    if (3 * ncv > ASM_COARSE_MAX_UNKNOWNS) {
      err = "global coarse grid has " + std::to_string(3 * ncv) + " unknowns, more than " +
            std::to_string(ASM_COARSE_MAX_UNKNOWNS);
      return ASM_ERR_INVALID;
    }
    P.ncv = (int32_t)ncv;
    P.cvar.resize(N);
    for (int c = 0; c < N; ++c) {
      const int ix = c / (ny * nz), iy = (c / nz) % ny, iz = c % nz;
      P.cvar[c] = ((ix / cb[0]) * cby + iy / cb[1]) * cbz + iz / cb[2];
    }
    P.cbox_cells.ptr.assign(ncv + 1, 0);
    for (int c = 0; c < N; ++c) P.cbox_cells.ptr[P.cvar[c] + 1]++;
    for (int64_t k = 0; k < ncv; ++k) P.cbox_cells.ptr[k + 1] += P.cbox_cells.ptr[k];
    P.cbox_cells.idx.resize(N);
    {
      std::vector<int32_t> cur(P.cbox_cells.ptr.begin(), P.cbox_cells.ptr.end() - 1);
      for (int c = 0; c < N; ++c) P.cbox_cells.idx[cur[P.cvar[c]]++] = c;
    }
    std::vector<std::array<int32_t, 3>> t;
    t.reserve(A.nnzb);
    for (int a = 0; a < N; ++a)
      for (int e = A.rp[a]; e < A.rp[a + 1]; ++e) t.push_back({P.cvar[a], P.cvar[A.ci[e]], e});
    triples_to_csr(t, P.ncv, P.acp, P.acc, P.ac_src);
  }
  return ASM_OK;
}

}  // namespace asmx
