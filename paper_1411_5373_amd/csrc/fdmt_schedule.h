// Pass schedule of the fused FDMT: which iterations each kernel launch runs
// and, per work block, the tree of (row range, time window) nodes it needs.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "fdmt_tables.h"

namespace fdmt {

// One node of a block's dependency tree. Its rows are row0 .. row0+nrows-1 of
// its iteration's plane (for input-channel leaves: one staged input row and
// row0 = the channel's first partial-sum row); it holds times
// [T0 - win, T0 - win + width) of a tile that starts at T0.
struct Node {
  int32_t row0, nrows, win, width;
  int32_t lds;    // element offset inside its LDS buffer
  int32_t sub;    // sub-band (leaf of the first pass: channel) index
  int32_t rowcum; // rows of the nodes before it at the same level
  int32_t pad;
};

// One row of one level of a block, ready for the kernel (all offsets in
// elements). Level 0 ("staging") rows copy global data into LDS:
//   a = source row (plane row, or channel for the first pass), c = LDS row,
//   d = win (column 0 holds time T0 - win), e = width.
// Merge rows compute, for columns col < e,
//   LDS[c + col] (or global row c at the top level)
//     = LDS[a + col] (+ chain) + (col >= d - T0 ? LDS[b + col] (+ chain) : 0)
// where a/b already include the child row, window alignment and shift s,
// d = s + win (so col >= d - T0 exactly when t - s >= 0), f = win,
// g/h = Option-1 chain lengths of the two halves (first pass, first level).
struct Rec {
  int32_t a, b, c, d, e, f, g, h;
};

constexpr int kRecHeader = 12;  // per block: first record, then level ends (k+1 values)
// Elements past each level buffer of a level-by-level pass: a merge reads its
// operands in whole 64-column groups, up to 63 columns past a row's end.
constexpr int kLdsSlack = 64;

// How a pass evaluates its iterations.
enum class PassKind {
  Staged,     // leaves staged in LDS once, each output the tree sum of its 2^k terms
  Recursive,  // leaves staged in LDS, iterations merged level by level in LDS
  Register    // each output the tree sum of its 2^k terms loaded through the caches
};

// A term of a staged pass: LDS offset of the term's sample at the block's
// first output time, and the Option-1 chain length (first pass; else 0).
struct StagedTerm {
  int32_t lds, chain;
};

// Per staged block: [0] first staging record, [1] staged rows, [2] first term,
// [3] output rows, [4] first output row (plane l1), [5] quads per staged row,
// [6] ceil(2^32 / quads per row), [7] first partial-sum record, [8] channels
// with partial sums (first pass).
constexpr int kStagedHeader = 12;
constexpr int kMaxStagedQuads = 8192;  // staged 4-sample quads per block (held in registers)

struct Pass {
  bool from_input = false;  // leaves are input channels (first pass)
  PassKind kind = PassKind::Staged;
  bool gather = false;      // kind == Register
  int64_t term_offset = 0;  // Register: index of this pass's first Term in Schedule::terms
                            // (from the input: first InTerm in Schedule::iterms);
                            // Staged: first StagedTerm in Schedule::sterms
  int l0 = 0, l1 = 0;       // consumes plane l0 (or the input), produces plane l1
  int tile = 0;             // W: output samples per block
  int nblocks = 0;
  int nodes_per_block = 0;  // 2^(l1-l0+1) - 1, level by level, leaves first
  int lds_a = 0, lds_b = 0; // elements of the two LDS buffers
  int64_t node_offset = 0;  // index of this pass's first node in Schedule::nodes
  int64_t rec_offset = 0;   // index of this pass's first record in Schedule::recs
  int64_t head_offset = 0;  // index of this pass's first block header in Schedule::heads
  int max_recs = 0;         // most records of any block (staged passes keep them in LDS)
  int64_t rows_in = 0;      // unique rows of the consumed plane (input: channels)
  int64_t rows_out = 0;     // rows of the produced plane
  int64_t staged_rows = 0;  // leaf rows staged, summed over blocks (overlap included)
  int64_t psum_offset = 0;  // staged first pass: index of the first Schedule::psums record
  int lds_p = 0;            // staged first pass: LDS elements of the partial-sum rows
  int stage_ints = 0;       // staged: LDS ints of the staging-record area
  int max_chain = 0;        // register pass from the input: longest Option-1 chain of its terms
};

struct ScheduleParams {
  int first_levels = 4;      // iterations fused with the initialisation
  int later_levels = 3;      // iterations per later pass
  bool first_auto = true;    // fewer first-pass iterations if they do not fit the budget
  bool later_auto = true;    // likewise for later passes
  int tile = 256;            // W (a multiple of 256 for staged passes)
  int lds_bytes = 64 * 1024; // per-block LDS budget
  int max_block_rows = 64;   // cap on rows of the top node
  int acc_bytes = 4;
  PassKind first_kind = PassKind::Recursive;
  PassKind later_kind = PassKind::Register;
};

// A term of a gather pass: plane-l0 row and accumulated shift.
struct Term {
  int32_t row, shift;
};

// A term of a register gather from the input: channel ch's Option-1 partial
// sum of chain length `chain` (samples t - shift, t - shift - 1, ...).
struct InTerm {
  int32_t ch, shift, chain, pad;
};

struct Schedule {
  bool init_separate = false;   // the initialisation runs as its own step (writes plane 0)
  std::vector<Pass> passes;
  std::vector<Node> nodes;
  std::vector<Rec> recs;        // per block, level by level
  std::vector<int32_t> heads;   // kRecHeader per block: record base (pass-relative), level ends
  std::vector<Term> terms;      // register passes: 2^k terms per output row, recursion order
  std::vector<InTerm> iterms;   // register pass from the input: 2^k terms per output row
  std::vector<StagedTerm> sterms;  // staged passes: 2^k terms per block row, recursion order
  std::vector<Rec> stage;       // staged passes: leaf rows (a = source row, c = LDS, d = win, e = width)
  std::vector<Rec> psums;       // staged first pass, per channel: a = LDS of partial-sum row 0,
                                // b = LDS of the staged input row, c = last partial-sum row,
                                // d = partial-sum row stride, e = width, f = input columns ahead
  std::vector<int32_t> sheads;  // staged passes: kStagedHeader per block
};

// Builds the pass list and every block's node tree. Returns "" on success.
std::string build_schedule(Schedule &s, const Tables &t, const ScheduleParams &p);

// ---------------------------------------------------------------------------
// Adjoint schedule. Each pass maps plane l_hi (the gradient of the output when
// l_hi = levels) to plane l_lo, or to the input channels when `to_input`, in
// which case it also applies the transpose of the Option-1 sums. Every output
// row is a nested sum: a row of plane l adds, in ascending dt, the rows of
// plane l+1 that read it (shifted by s when it is their upper half); a channel
// adds its partial-sum rows d at lags i = 0..d, in (d, i) order. A leaf is a
// row of plane l_hi with its accumulated shift and the depth of the deepest
// tree node it shares with the previous leaf.
//
// In a `lagged` pass (into the channels, some channel with two or more
// partial-sum rows) the subtree of partial-sum row d is listed once, at lag 0,
// and its first leaf carries lags = d + 1 and its leaf count: the kernel adds
// the finished subtree to the channel at t, t + 1, ..., t + d, taking the
// later samples from neighbouring lanes. The value at t + i is the lag-i
// subtree's, so the sums and their order are those of the full list.
struct AdjLeaf {
  int32_t row, shift, branch;
  int32_t lags;  // lagged pass, a subtree's first leaf: its lags | its leaf count << 3; else 0
};
// Leaf records readable past the end of the list (zeros): the adjoint gather
// loads the records of its next chunk before it knows whether there is one.
constexpr int kAdjLeafPad = 16;

struct AdjPass {
  int l_hi = 0, l_lo = 0;
  bool to_input = false;
  int depth = 0;              // tree depth: l_hi - l_lo, plus 1 with the init transpose
  int nrows = 0;              // output rows (plane l_lo rows, or channels)
  int64_t leaf_offset = 0;    // first leaf in AdjSchedule::leaves
  int64_t start_offset = 0;   // first entry in AdjSchedule::starts (nrows + 1 per pass)
  int64_t order_offset = 0;   // first entry in AdjSchedule::order (nrows per pass)
  int64_t leaves = 0;         // leaves of this pass
  int32_t max_shift = 0;      // largest leaf shift of this pass
  bool lagged = false;        // subtrees listed once with their lag count (see AdjLeaf)
};

struct AdjSchedule {
  bool init_separate = false;   // passes end at plane 0; the init transpose runs on its own
  std::vector<AdjPass> passes;
  std::vector<AdjLeaf> leaves;
  std::vector<int32_t> starts;  // per pass: leaf index (pass-relative) of each row, then the end
  std::vector<int32_t> order;   // per pass: output row of each position (rows that share
                                // leaves are neighbours, so they meet in one XCD's L2)
};

// Largest lag count of a lagged pass: a channel's partial-sum rows are then
// at most this many.
constexpr int kMaxLags = 4;

// Passes of at most `levels_per_pass` iterations from the output down to the
// channels; the last pass includes the init transpose. With `lag_reuse`, a
// last pass whose channels have several partial-sum rows (at most kMaxLags)
// is lagged.
std::string build_adjoint_schedule(AdjSchedule &s, const Tables &t, int levels_per_pass, int last_levels,
                                   bool lag_reuse = true);

} // namespace fdmt
