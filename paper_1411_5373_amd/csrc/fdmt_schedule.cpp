// Pass schedule of the fused FDMT (host).
//
// A pass fuses iterations l0+1 .. l1. Its work item ("block") is a range of
// consecutive rows of one sub-band of plane l1 over one time tile
// [T0, T0 + W). Walking the delay tables down from the block gives, at every
// fused iteration, the rows each sub-band must supply: because d_lo, d_hi and
// s are non-decreasing in dt, they are the contiguous range between the
// children of the block's first and last rows. The lower half is read at the
// same times as its parent; the upper half t - s back, so its time window is
// the parent's widened by the spread of s over the block.
#include "fdmt_schedule.h"

#include <algorithm>

namespace fdmt {

namespace {

struct Tree {
  std::vector<Node> nodes;  // level by level, leaves first
  int need[2] = {0, 0};     // elements of LDS buffers A (even levels) and B (odd levels)
};

// Builds the tree of a block and its LDS layout; levels i = 0..k of the pass.
Tree build_tree(const Tables &t, bool from_input, int l0, int l1, int sub, int r0, int nr, int tile) {
  const int k = l1 - l0;
  std::vector<std::vector<Node>> lv(k + 1);
  lv[k].push_back(Node{static_cast<int32_t>(t.row_off[l1][sub] + r0), nr, 0, tile, 0, sub, 0, 0});
  for (int i = k; i >= 1; --i) {
    const int l = l0 + i;
    lv[i - 1].resize(lv[i].size() * 2);
    for (size_t j = 0; j < lv[i].size(); ++j) {
      const Node &n = lv[i][j];
      const MergeRow &a = t.merge[l][n.row0];
      const MergeRow &b = t.merge[l][n.row0 + n.nrows - 1];
      lv[i - 1][2 * j] = Node{a.lo, b.lo - a.lo + 1, n.win, n.width, 0, 2 * n.sub, 0, 0};
      lv[i - 1][2 * j + 1] =
          Node{a.hi, b.hi - a.hi + 1, n.win + b.s, n.width + (b.s - a.s), 0, 2 * n.sub + 1, 0, 0};
    }
  }
  if (from_input) {
    // Leaves become staged input rows: the Option-1 chain of partial-sum row d
    // reads d samples further back, so the window grows by the largest d.
    for (Node &n : lv[0]) {
      const int ch = n.sub;
      const int d_last = n.row0 + n.nrows - 1 - t.leaf_off[ch];
      n.win += d_last;
      n.width += d_last;
      n.row0 = t.leaf_off[ch];
      n.nrows = 1;
    }
  }
  Tree tr;
  for (int i = 0; i <= k; ++i) {
    int off = 0, cum = 0;
    for (Node &n : lv[i]) {
      n.lds = i < k ? off : 0;
      n.rowcum = cum;
      off += n.nrows * n.width;
      cum += n.nrows;
    }
    if (i < k) tr.need[i & 1] = std::max(tr.need[i & 1], off);
    tr.nodes.insert(tr.nodes.end(), lv[i].begin(), lv[i].end());
  }
  return tr;
}

// Checks, for every block, that each merge reads only rows its children hold
// and only columns inside their windows, and that every node fits its LDS
// buffer: the bounds the fused kernel relies on.
std::string audit_pass(const Tables &t, const Pass &ps, const Node *nodes) {
  const int k = ps.l1 - ps.l0;
  for (int b = 0; b < ps.nblocks; ++b) {
    const Node *nd = nodes + static_cast<int64_t>(b) * ps.nodes_per_block;
    int base = 0;
    std::vector<int> level_base(k + 2);
    for (int i = 0; i <= k; ++i) {
      level_base[i] = base;
      base += 1 << (k - i);
    }
    level_base[k + 1] = base;
    for (int i = 0; i < k; ++i) {
      const int cap = (i & 1) ? ps.lds_b : ps.lds_a;
      for (int j = level_base[i]; j < level_base[i + 1]; ++j)
        if (nd[j].lds < 0 || nd[j].lds + static_cast<int64_t>(nd[j].nrows) * nd[j].width > cap)
          return "node outside its LDS buffer";
    }
    const Node &top = nd[level_base[k]];
    if (top.win != 0 || top.width != ps.tile) return "top node window";
    for (int i = 1; i <= k; ++i) {
      const int l = ps.l0 + i;
      for (int j = level_base[i]; j < level_base[i + 1]; ++j) {
        const Node &n = nd[j];
        const Node &lo = nd[level_base[i - 1] + 2 * (j - level_base[i])];
        const Node &hi = nd[level_base[i - 1] + 2 * (j - level_base[i]) + 1];
        if (n.row0 < 0 || n.row0 + n.nrows > t.total[l]) return "node rows outside plane";
        for (int r = 0; r < n.nrows; ++r) {
          const MergeRow &m = t.merge[l][n.row0 + r];
          const int dl = m.lo - lo.row0, dh = m.hi - hi.row0;
          if (ps.from_input && i == 1) {
            // chain over the staged input row: columns c + lo.win - n.win - d, d <= dl
            if (dl < 0 || dh < 0) return "partial-sum row below the channel";
            if (lo.win - n.win - dl < 0 || n.width - 1 + lo.win - n.win > lo.width - 1)
              return "lower input window";
            if (hi.win - n.win - m.s - dh < 0 || n.width - 1 - m.s + hi.win - n.win > hi.width - 1)
              return "upper input window";
            if (t.leaf_rows[lo.sub] <= dl || t.leaf_rows[hi.sub] <= dh) return "partial-sum row";
          } else {
            if (dl < 0 || dl >= lo.nrows || dh < 0 || dh >= hi.nrows) return "child row outside node";
            if (lo.win != n.win || lo.width < n.width) return "lower window";
            if (hi.win - n.win - m.s < 0 || n.width - 1 - m.s + hi.win - n.win > hi.width - 1)
              return "upper window";
          }
        }
      }
    }
  }
  return "";
}

// Flattens a block's tree into kernel records (see Rec).
void emit_records(const Tables &t, bool from_input, int l0, int k, const Node *nd,
                  std::vector<Rec> &recs, int32_t *head) {
  std::vector<int> level_base(k + 2);
  int base = 0;
  for (int i = 0; i <= k; ++i) {
    level_base[i] = base;
    base += 1 << (k - i);
  }
  level_base[k + 1] = base;
  const int32_t first = static_cast<int32_t>(recs.size());
  head[0] = first;
  for (int j = level_base[0]; j < level_base[1]; ++j) {
    const Node &n = nd[j];
    for (int r = 0; r < n.nrows; ++r)
      recs.push_back(Rec{from_input ? n.sub : n.row0 + r, 0, n.lds + r * n.width, n.win, n.width, 0, 0, 0});
  }
  head[1] = static_cast<int32_t>(recs.size()) - first;
  for (int i = 1; i <= k; ++i) {
    const int l = l0 + i;
    for (int j = level_base[i]; j < level_base[i + 1]; ++j) {
      const Node &n = nd[j];
      const Node &lo = nd[level_base[i - 1] + 2 * (j - level_base[i])];
      const Node &hi = nd[level_base[i - 1] + 2 * (j - level_base[i]) + 1];
      for (int r = 0; r < n.nrows; ++r) {
        const MergeRow &m = t.merge[l][n.row0 + r];
        Rec e{};
        if (from_input && i == 1) {
          e.a = lo.lds + (lo.win - n.win);
          e.b = hi.lds + (hi.win - n.win) - m.s;
          e.g = m.lo - lo.row0;
          e.h = m.hi - hi.row0;
        } else {
          e.a = lo.lds + (m.lo - lo.row0) * lo.width + (lo.win - n.win);
          e.b = hi.lds + (m.hi - hi.row0) * hi.width + (hi.win - n.win) - m.s;
        }
        e.c = i == k ? n.row0 + r : n.lds + r * n.width;
        e.d = m.s + n.win;
        e.e = n.width;
        e.f = n.win;
        recs.push_back(e);
      }
    }
    head[1 + i] = static_cast<int32_t>(recs.size()) - first;
  }
}

// Bounds of every record as the kernel will use it: LDS reads and writes
// inside their buffers, source rows inside the consumed plane (or channel
// range), destination rows inside the produced plane.
std::string audit_records(const Tables &t, const Pass &ps, const Rec *recs, const int32_t *heads) {
  const int k = ps.l1 - ps.l0;
  const int64_t src_rows = ps.from_input ? t.slots : t.total[ps.l0];
  for (int b = 0; b < ps.nblocks; ++b) {
    const int32_t *h = heads + static_cast<int64_t>(b) * kRecHeader;
    const Rec *r = recs + h[0];
    if (h[1 + k] > ps.max_recs) return "record count";
    for (int q = 0; q < h[1]; ++q) {
      if (r[q].a < 0 || r[q].a >= src_rows) return "staged row outside source";
      if (r[q].c < 0 || r[q].c + r[q].e > ps.lds_a || r[q].e < 1) return "staged row outside LDS";
    }
    for (int i = 1; i <= k; ++i) {
      const int64_t src_cap = (i & 1) ? ps.lds_a : ps.lds_b;  // level i-1 buffer
      const int64_t dst_cap = (i & 1) ? ps.lds_b : ps.lds_a;
      for (int q = h[i]; q < h[1 + i]; ++q) {
        const Rec &e = r[q];
        const int back_lo = (ps.from_input && i == 1) ? e.g : 0;
        const int back_hi = (ps.from_input && i == 1) ? e.h : 0;
        if (e.e < 1 || e.a - back_lo < 0 || e.a + e.e > src_cap) return "lower operand outside LDS";
        if (e.b - back_hi < 0 || e.b + e.e > src_cap) return "upper operand outside LDS";
        if (i == k) {
          if (e.c < 0 || e.c >= t.total[ps.l1] || e.e != ps.tile) return "top row";
        } else if (e.c < 0 || e.c + e.e > dst_cap) {
          return "merged row outside LDS";
        }
      }
    }
  }
  return "";
}

// Staged pass layout of one block. Leaves are packed in LDS with row
// strides padded to 4 elements. In the first pass a leaf is one staged input
// row per channel plus, after all of them, the channel's Option-1 partial-sum
// rows 0 .. d_last computed from it in LDS.
struct StagedLayout {
  int64_t stage_elems = 0;  // staged rows (input or plane rows)
  int64_t psum_elems = 0;   // partial-sum rows (first pass)
  std::vector<int> psum_lds;
};

StagedLayout staged_layout(const Tables &t, bool from_input, std::vector<Node> &leaves,
                           const std::vector<Node> &generic) {
  StagedLayout lay;
  int64_t off = 0;
  for (Node &n : leaves) {
    n.lds = static_cast<int32_t>(off);
    off += static_cast<int64_t>(n.nrows) * ((n.width + 3) / 4 * 4);
  }
  lay.stage_elems = off;
  if (from_input) {
    for (size_t j = 0; j < leaves.size(); ++j) {
      const Node &g = generic[j];  // partial-sum rows and window before widening
      const int d_last = g.row0 + g.nrows - 1 - t.leaf_off[g.sub];
      lay.psum_lds.push_back(static_cast<int>(off));
      off += static_cast<int64_t>(d_last + 1) * ((g.width + 3) / 4 * 4);
    }
    lay.psum_elems = off - lay.stage_elems;
  }
  return lay;
}

// Emits the staging records, partial-sum records, terms and header of one
// staged block and checks every LDS access the kernel will make for it.
std::string emit_staged(const Tables &t, bool from_input, int l0, int l1, int sub, int r0, int nr,
                        int tile, const std::vector<Node> &leaves, const std::vector<Node> &generic,
                        const StagedLayout &lay, Schedule &s, const Pass &ps) {
  const int k = l1 - l0;
  const int n_terms = 1 << k;
  const int64_t lds_total = lay.stage_elems + lay.psum_elems;
  int32_t head[kStagedHeader] = {};
  head[0] = static_cast<int32_t>(s.stage.size() - ps.rec_offset);
  int max_w4 = 0;
  for (const Node &n : leaves) {
    const int w4 = (n.width + 3) / 4 * 4;
    max_w4 = std::max(max_w4, w4);
    for (int r = 0; r < n.nrows; ++r) {
      if (n.lds + static_cast<int64_t>(r + 1) * w4 > lay.stage_elems) return "staged row outside LDS";
      s.stage.push_back(Rec{from_input ? n.sub : n.row0 + r, 0, n.lds + r * w4, n.win, w4, 0, 0, 0});
    }
  }
  head[1] = static_cast<int32_t>(s.stage.size() - ps.rec_offset) - head[0];
  head[2] = static_cast<int32_t>(s.sterms.size() - ps.term_offset);
  head[3] = nr;
  head[4] = static_cast<int32_t>(t.row_off[l1][sub] + r0);
  const int qpr = max_w4 / 4;  // quads per staged row
  head[5] = qpr;
  head[6] = static_cast<int32_t>((0x100000000ull + qpr - 1) / qpr);  // ceil(2^32 / qpr)
  if (static_cast<int64_t>(head[1]) * qpr >= 65536) return "staged block too large";
  head[7] = static_cast<int32_t>(s.psums.size() - ps.psum_offset);
  head[8] = from_input ? static_cast<int32_t>(leaves.size()) : 0;
  if (from_input) {
    for (size_t j = 0; j < leaves.size(); ++j) {
      const Node &x = leaves[j], &g = generic[j];
      const int d_last = g.row0 + g.nrows - 1 - t.leaf_off[g.sub];
      const int w4 = (g.width + 3) / 4 * 4;
      // input column of time T0 - g.win + c is c + (x.win - g.win); the chain
      // reads d_last samples back from there
      const int ahead = x.win - g.win;
      if (ahead != d_last || x.width != g.width + d_last) return "partial-sum window";
      if (lay.psum_lds[j] + static_cast<int64_t>(d_last + 1) * w4 > lds_total) return "partial sums outside LDS";
      s.psums.push_back(Rec{lay.psum_lds[j], x.lds, d_last, w4, g.width, ahead, 0, 0});
    }
  }
  std::vector<Term> cur, nxt;
  for (int r = 0; r < nr; ++r) {
    cur.assign(1, Term{static_cast<int32_t>(t.row_off[l1][sub] + r0 + r), 0});
    for (int l = l1; l > l0; --l) {
      nxt.clear();
      for (const Term &x : cur) {
        const MergeRow &m = t.merge[l][x.row];
        nxt.push_back(Term{m.lo, x.shift});
        nxt.push_back(Term{m.hi, x.shift + m.s});
      }
      cur.swap(nxt);
    }
    for (int j = 0; j < n_terms; ++j) {
      StagedTerm st{};
      int64_t row_start, row_end;
      int col0;
      if (from_input) {
        const Node &g = generic[j];
        const int d = cur[j].row - t.leaf_off[g.sub];  // partial-sum row of the channel
        const int d_last = g.row0 + g.nrows - 1 - t.leaf_off[g.sub];
        if (d < 0 || d > d_last) return "partial-sum row of a term";
        const int w4 = (g.width + 3) / 4 * 4;
        col0 = g.win - cur[j].shift;
        if (col0 < 0 || col0 + tile > g.width) return "partial-sum term window";
        row_start = lay.psum_lds[j] + static_cast<int64_t>(d) * w4;
        row_end = row_start + w4;
      } else {
        const Node &n = leaves[j];
        const int w4 = (n.width + 3) / 4 * 4;
        const int rl = cur[j].row - n.row0;
        if (rl < 0 || rl >= n.nrows) return "staged term row outside leaf";
        col0 = n.win - cur[j].shift;  // column of time T0 - sigma
        if (col0 < 0 || col0 + tile > n.width) return "staged term window";
        row_start = n.lds + static_cast<int64_t>(rl) * w4;
        row_end = row_start + w4;
      }
      st.lds = static_cast<int32_t>(row_start + col0);
      if (row_start < 0 || row_end > lds_total || st.lds + tile > row_end) return "staged term outside LDS";
      s.sterms.push_back(st);
    }
  }
  s.sheads.insert(s.sheads.end(), head, head + kStagedHeader);
  return "";
}

} // namespace

// Builds one pass of k iterations starting at plane l0 and appends it.
std::string build_pass(Schedule &s, const Tables &t, const ScheduleParams &p, int l0, int k_req,
                       bool from_input) {
  const int L = t.levels;
  const int64_t budget = p.lds_bytes / p.acc_bytes;
  {
    const bool first = from_input;
    const PassKind kind = first ? p.first_kind : p.later_kind;
    // The d_min pre-shift enters through the input terms of a register pass
    // (and the initialisation kernels); passes that stage input rows in LDS do
    // not apply it.
    if (first && kind != PassKind::Register)
      for (int k = 0; k < t.nf; ++k)
        if (t.pre[k] != 0) return "the d_min pre-shift needs the first pass to gather from the input";
    if (kind == PassKind::Staged) {
      const int k = std::min(k_req, L - l0);
      // five would hold 32 terms of 4 runs per thread: past the register
      // budget of its workgroup (it spilled)
      if (k > 4) return "at most 4 iterations per staged pass";
      if (p.tile % 256 != 0) return "staged passes need a tile that is a multiple of 256";
      Pass ps;
      ps.kind = PassKind::Staged;
      ps.from_input = first;
      ps.l0 = l0;
      ps.l1 = l0 + k;
      ps.tile = p.tile;
      ps.rows_in = first ? t.slots : t.total[l0];
      ps.rows_out = t.total[ps.l1];
      ps.rec_offset = static_cast<int64_t>(s.stage.size());
      ps.term_offset = static_cast<int64_t>(s.sterms.size());
      ps.head_offset = static_cast<int64_t>(s.sheads.size());
      ps.psum_offset = static_cast<int64_t>(s.psums.size());
      int max_stage = 0, max_rows = 0;
      int64_t leaf_max = 0, psum_max = 0;
      for (int sub = 0; sub < (t.slots >> ps.l1); ++sub) {
        const int n = t.rows[ps.l1][sub];
        int r0 = 0;
        while (r0 < n) {
          int nr = std::min(p.max_block_rows, n - r0);
          std::vector<Node> leaves, generic;
          StagedLayout lay;
          int nstage = 0;
          for (;;) {
            Tree tr = build_tree(t, first, l0, ps.l1, sub, r0, nr, p.tile);
            leaves.assign(tr.nodes.begin(), tr.nodes.begin() + (1 << k));
            if (first) {
              Tree g = build_tree(t, false, l0, ps.l1, sub, r0, nr, p.tile);
              generic.assign(g.nodes.begin(), g.nodes.begin() + (1 << k));
            }
            lay = staged_layout(t, first, leaves, generic);
            nstage = 0;
            for (const Node &x : leaves) nstage += x.nrows;
            // LDS: leaves, partial sums, staging records (4 ints each),
            // partial-sum records (4 ints per channel), terms (2 ints each)
            int max_w4 = 0;
            for (const Node &x : leaves) max_w4 = std::max(max_w4, (x.width + 3) / 4 * 4);
            const int64_t quads = static_cast<int64_t>(nstage) * (max_w4 / 4);
            const int64_t need = lay.stage_elems + lay.psum_elems + 4LL * nstage +
                                 (first ? 8LL * (1 << k) : 0) + 2LL * nr * (1 << k);
            if (need <= budget && quads <= kMaxStagedQuads) break;
            if (nr == 1) return "LDS budget too small for one row of pass " + std::to_string(l0);
            nr = std::max(1, nr * 3 / 4);
          }
          ps.staged_rows += nstage;
          const std::string err =
              emit_staged(t, first, l0, ps.l1, sub, r0, nr, p.tile, leaves, generic, lay, s, ps);
          if (!err.empty()) return "audit of pass " + std::to_string(l0) + ": " + err;
          leaf_max = std::max(leaf_max, lay.stage_elems);
          psum_max = std::max(psum_max, lay.psum_elems);
          max_stage = std::max(max_stage, nstage);
          max_rows = std::max(max_rows, nr);
          ++ps.nblocks;
          r0 += nr;
        }
      }
      // LDS areas (4-byte units): staged rows | partial sums | staging records |
      // partial-sum records | terms. Partial-sum offsets are relative to the
      // start of LDS, so the partial-sum area follows the largest staged area.
      ps.lds_a = static_cast<int>((leaf_max + 3) / 4 * 4);
      ps.lds_p = static_cast<int>((psum_max + 3) / 4 * 4);
      ps.stage_ints = 4 * max_stage;
      ps.lds_b = ps.stage_ints + (first ? 8 * (1 << k) : 0);
      ps.max_recs = 2 * max_rows * (1 << k);
      s.passes.push_back(ps);
      return "";
    }
    if (kind == PassKind::Register) {
      // Iterations as register gathers: walking the tables down from each
      // output row gives its 2^k (row, shift) terms of plane l0, in the order
      // the recursion adds them (lower half before upper half). From the
      // input, a plane-0 term is channel ch's Option-1 partial-sum row d:
      // the chain of input samples at shifts sigma .. sigma + d.
      const int k = std::min(k_req, L - l0);
      if (k > 4) return "at most 4 iterations per register pass";
      Pass ps;
      ps.gather = true;
      ps.kind = PassKind::Register;
      ps.from_input = first;
      ps.l0 = l0;
      ps.l1 = l0 + k;
      ps.rows_in = first ? t.slots : t.total[l0];
      ps.rows_out = t.total[ps.l1];
      ps.term_offset = static_cast<int64_t>(first ? s.iterms.size() : s.terms.size());
      std::vector<int32_t> channel_of;
      if (first) {
        channel_of.resize(t.total[0]);
        for (int ch = 0; ch < t.slots; ++ch)
          for (int d = 0; d < t.leaf_rows[ch]; ++d) channel_of[t.leaf_off[ch] + d] = ch;
      }
      std::vector<Term> cur, nxt;
      for (int64_t r = 0; r < ps.rows_out; ++r) {
        cur.assign(1, Term{static_cast<int32_t>(r), 0});
        for (int l = ps.l1; l > l0; --l) {
          nxt.clear();
          for (const Term &x : cur) {
            const MergeRow &m = t.merge[l][x.row];
            nxt.push_back(Term{m.lo, x.shift});
            nxt.push_back(Term{m.hi, x.shift + m.s});
          }
          cur.swap(nxt);
        }
        for (const Term &x : cur)
          if (x.row < 0 || x.row >= t.total[l0] || x.shift < 0) return "gather term out of range";
        if (first) {
          for (const Term &x : cur) {
            const int ch = channel_of[x.row];
            const int d = x.row - t.leaf_off[ch];
            // a position without a channel reads a zero row of the padded input
            s.iterms.push_back(InTerm{ch, x.shift + (ch < t.nf ? t.pre[ch] : 0), d, 0});
            ps.staged_rows += d + 1;
            ps.max_chain = std::max(ps.max_chain, d);
          }
        } else {
          s.terms.insert(s.terms.end(), cur.begin(), cur.end());
          ps.staged_rows += static_cast<int64_t>(cur.size());
        }
      }
      ps.nblocks = static_cast<int>(ps.rows_out);
      s.passes.push_back(ps);
      return "";
    }
    const int k = std::min(k_req, L - l0);
    if (k > 8) return "at most 8 iterations per pass";
    Pass ps;
    ps.kind = PassKind::Recursive;
    ps.from_input = first;
    ps.l0 = l0;
    ps.l1 = l0 + k;
    ps.tile = p.tile;
    ps.nodes_per_block = (1 << (k + 1)) - 1;
    ps.node_offset = static_cast<int64_t>(s.nodes.size());
    ps.rec_offset = static_cast<int64_t>(s.recs.size());
    ps.head_offset = static_cast<int64_t>(s.heads.size());
    ps.rows_in = first ? t.slots : t.total[l0];
    ps.rows_out = t.total[ps.l1];
    for (int sub = 0; sub < (t.slots >> ps.l1); ++sub) {
      const int n = t.rows[ps.l1][sub];
      int r0 = 0;
      while (r0 < n) {
        int nr = std::min(p.max_block_rows, n - r0);
        Tree tr;  // level-by-level LDS pass
        for (;;) {
          tr = build_tree(t, first, l0, ps.l1, sub, r0, nr, p.tile);
          if (tr.need[0] + tr.need[1] + 2 * kLdsSlack <= budget) break;
          if (nr == 1) return "LDS budget too small for one row of pass " + std::to_string(l0);
          nr = std::max(1, nr * 3 / 4);
        }
        ps.lds_a = std::max(ps.lds_a, tr.need[0]);
        ps.lds_b = std::max(ps.lds_b, tr.need[1]);
        for (int j = 0; j < (1 << k); ++j) ps.staged_rows += tr.nodes[j].nrows;
        s.nodes.insert(s.nodes.end(), tr.nodes.begin(), tr.nodes.end());
        int32_t head[kRecHeader] = {};
        const size_t before = s.recs.size();
        emit_records(t, first, l0, k, tr.nodes.data(), s.recs, head);
        head[0] -= static_cast<int32_t>(ps.rec_offset);
        ps.max_recs = std::max(ps.max_recs, static_cast<int>(s.recs.size() - before));
        s.heads.insert(s.heads.end(), head, head + kRecHeader);
        ++ps.nblocks;
        r0 += nr;
      }
    }
    ps.lds_a = (ps.lds_a + 3) / 4 * 4;  // keeps the record area 16-byte aligned
    ps.lds_b = (ps.lds_b + 3) / 4 * 4;
    std::string err = audit_pass(t, ps, s.nodes.data() + ps.node_offset);
    if (err.empty())
      err = audit_records(t, ps, s.recs.data() + ps.rec_offset, s.heads.data() + ps.head_offset);
    if (!err.empty()) return "audit of pass " + std::to_string(l0) + ": " + err;
    s.passes.push_back(ps);
  }
  return "";
}

std::string build_schedule(Schedule &s, const Tables &t, const ScheduleParams &p) {
  s = Schedule();
  const int L = t.levels;
  if (L == 0) return "";
  if (p.tile < 1 || p.first_levels < 1 || p.later_levels < 1) return "bad schedule parameters";
  int l0 = 0;
  while (l0 < L) {
    const bool first = l0 == 0 && !s.init_separate;
    const bool automatic = first ? p.first_auto : p.later_auto;
    int k = std::min(first ? p.first_levels : p.later_levels, L - l0);
    for (;;) {
      // Remember the sizes so a pass that does not fit can be taken back.
      const size_t n_nodes = s.nodes.size(), n_recs = s.recs.size(), n_heads = s.heads.size(),
                   n_terms = s.terms.size(), n_iterms = s.iterms.size(), n_sterms = s.sterms.size(),
                   n_stage = s.stage.size(),
                   n_psums = s.psums.size(), n_sheads = s.sheads.size();
      const std::string err = build_pass(s, t, p, l0, k, first);
      if (err.empty()) break;
      s.nodes.resize(n_nodes);
      s.recs.resize(n_recs);
      s.heads.resize(n_heads);
      s.terms.resize(n_terms);
      s.iterms.resize(n_iterms);
      s.sterms.resize(n_sterms);
      s.stage.resize(n_stage);
      s.psums.resize(n_psums);
      s.sheads.resize(n_sheads);
      const bool too_big = err.find("LDS budget too small") != std::string::npos ||
                           err.find("at most") != std::string::npos;
      if (!automatic || !too_big) return err;
      if (k == 1) {
        // Not even one fused iteration fits: run the Option-1 initialisation
        // as its own step (writing plane 0) and fuse from plane 0 on.
        if (!first) return err;
        s.init_separate = true;
        break;
      }
      --k;
    }
    if (!s.passes.empty()) l0 = s.passes.back().l1;
  }
  return "";
}

namespace {

// Depth-first walk of one adjoint output row (see AdjLeaf).
struct AdjWalker {
  const Tables &t;
  int l_hi;
  std::vector<AdjLeaf> &out;

  // Row r of plane l at accumulated shift sigma, tree depth d; `branch` is
  // the branch depth handed to the first leaf below this node.
  void visit(int l, int r, int sigma, int d, int branch) {
    if (l == l_hi) {
      out.push_back(AdjLeaf{r, sigma, branch, 0});
      return;
    }
    const AdjRow &a = t.adj[l + 1][r];
    for (int q = 0; q < a.count; ++q) {
      const int p = a.first + q;
      const int s = a.upper ? t.merge[l + 1][p].s : 0;
      visit(l + 1, p, sigma + s, d + 1, q == 0 ? branch : d);
    }
  }
};

} // namespace

std::string build_adjoint_schedule(AdjSchedule &s, const Tables &t, int levels_per_pass, int last_levels,
                                   bool lag_reuse) {
  s = AdjSchedule();
  const int L = t.levels;
  if (L == 0) return "";
  if (levels_per_pass < 1 || last_levels < 1) return "bad adjoint schedule parameters";
  // Fold the init transpose into the last pass only while its fan-out (the
  // (d, i) pairs of a channel, quadratic in its partial-sum rows) is small;
  // otherwise the passes stop at plane 0 and the transpose runs on its own.
  int fan = 0, rows_max = 0;
  for (int k = 0; k < t.nf; ++k) {
    fan = std::max(fan, t.leaf_rows[k] * (t.leaf_rows[k] + 1) / 2);
    rows_max = std::max(rows_max, t.leaf_rows[k]);
  }
  s.init_separate = fan > 16;
  int l_hi = L;
  while (l_hi > 0) {
    AdjPass ps;
    ps.l_hi = l_hi;
    // The last pass (down to the channels) takes the init transpose too.
    if (l_hi <= last_levels && !s.init_separate) {
      ps.l_lo = 0;
      ps.to_input = true;
      ps.depth = l_hi + 1;
      ps.nrows = t.nf;
      ps.lagged = lag_reuse && rows_max > 1 && rows_max <= kMaxLags;
    } else {
      ps.l_lo = std::max(l_hi - levels_per_pass, s.init_separate ? 0 : last_levels);
      ps.depth = l_hi - ps.l_lo;
      ps.nrows = static_cast<int>(t.total[ps.l_lo]);
    }
    if (ps.depth > 5) return "adjoint pass deeper than 5";
    ps.leaf_offset = static_cast<int64_t>(s.leaves.size());
    ps.start_offset = static_cast<int64_t>(s.starts.size());
    ps.order_offset = static_cast<int64_t>(s.order.size());
    // Leaves of every output row, then the rows ordered by the first plane-l_hi
    // row they read.
    std::vector<std::vector<AdjLeaf>> per_row(ps.nrows);
    for (int r = 0; r < ps.nrows; ++r) {
      AdjWalker w{t, l_hi, per_row[r]};
      if (ps.lagged) {
        // channel r: the subtree of each partial-sum row d once, at lag 0
        // (plus the channel's pre-shift), its first leaf carrying the d + 1
        // lags it is added at
        for (int d = 0; d < t.leaf_rows[r]; ++d) {
          const size_t first = per_row[r].size();
          w.visit(0, t.leaf_off[r] + d, t.pre[r], 1, 0);
          per_row[r][first].lags = (d + 1) | static_cast<int32_t>(per_row[r].size() - first) << 3;
        }
      } else if (ps.to_input) {
        // channel r: partial-sum rows d at lags i (plus the channel's
        // pre-shift), in (d, i) order; each starts a new child of the root
        // (branch depth 0)
        for (int d = 0; d < t.leaf_rows[r]; ++d)
          for (int i = 0; i <= d; ++i) w.visit(0, t.leaf_off[r] + d, t.pre[r] + i, 1, 0);
      } else {
        w.visit(ps.l_lo, r, 0, 0, 0);
      }
    }
    std::vector<int32_t> ord(ps.nrows);
    for (int r = 0; r < ps.nrows; ++r) ord[r] = r;
    std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) {
      return per_row[a].front().row < per_row[b].front().row;
    });
    for (int i = 0; i < ps.nrows; ++i) {
      s.starts.push_back(static_cast<int32_t>(s.leaves.size() - ps.leaf_offset));
      s.order.push_back(ord[i]);
      const std::vector<AdjLeaf> &lv = per_row[ord[i]];
      s.leaves.insert(s.leaves.end(), lv.begin(), lv.end());
    }
    s.starts.push_back(static_cast<int32_t>(s.leaves.size() - ps.leaf_offset));
    ps.leaves = static_cast<int64_t>(s.leaves.size()) - ps.leaf_offset;
    if (s.leaves.size() > static_cast<size_t>(INT32_MAX)) return "adjoint schedule too large";
    // Audit: rows inside plane l_hi, shifts non-negative, branch depths valid.
    for (int64_t x = ps.leaf_offset; x < static_cast<int64_t>(s.leaves.size()); ++x) {
      const AdjLeaf &e = s.leaves[x];
      if (e.row < 0 || e.row >= t.total[l_hi] || e.shift < 0 || e.branch < 0 || e.branch >= ps.depth)
        return "adjoint leaf out of range";
      if (!ps.lagged && e.lags != 0) return "adjoint leaf lags";
      ps.max_shift = std::max(ps.max_shift, e.shift);
    }
    // A lagged pass: each row is a sequence of subtrees, each opened by a leaf
    // at branch 0 that holds its lags (1..kMaxLags) and leaf count, the other
    // leaves below the root.
    if (ps.lagged) {
      for (int i = 0; i < ps.nrows; ++i) {
        const int64_t end = ps.leaf_offset + s.starts[ps.start_offset + i + 1];
        for (int64_t x = ps.leaf_offset + s.starts[ps.start_offset + i]; x < end;) {
          const AdjLeaf &e = s.leaves[x];
          const int lags = e.lags & 7, count = e.lags >> 3;
          if (e.branch != 0 || lags < 1 || lags > kMaxLags || count < 1 || x + count > end)
            return "adjoint leaf lags";
          for (int64_t y = x + 1; y < x + count; ++y)
            if (s.leaves[y].branch == 0 || s.leaves[y].lags != 0) return "adjoint leaf lags";
          x += count;
        }
      }
    }
    s.passes.push_back(ps);
    l_hi = ps.l_lo;
  }
  return "";
}

} // namespace fdmt
