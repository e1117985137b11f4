// Host-side delay tables of the FDMT (Zackay & Ofek, Sec. 4, Eq. Cf2f0 and
// Algorithm 1) in the flat, device-friendly form the kernels consume.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

namespace fdmt {

// One output row of an iteration: out[t] = plane[lo][t] + plane[hi][t - s]
// (the second term only for t >= s). lo/hi are rows of the previous
// iteration's plane (all sub-bands concatenated), s the upper half's shift.
struct MergeRow {
  int32_t lo, hi, s, sub;
};

// One row of the previous iteration's plane seen from the adjoint: it is the
// lower (upper = 0) or upper (upper = 1) half of `count` consecutive output
// rows starting at `first` in this iteration's plane.
struct AdjRow {
  int32_t first, count, upper, pad;
};

// Pre-shift of a channel position that holds no channel (Nf not a power of
// two): its input lies past the end of every record, so it reads as zero.
constexpr int32_t kNoChannelPre = INT32_MAX;

struct Tables {
  int nf = 0, nd = 0, levels = 0;
  int slots = 0;  // 2^levels channel positions; positions nf .. slots-1 hold no channel
  double f_min = 0, f_max = 0;
  double gamma = -2.0;  // delay law dt ~ f^gamma
  int32_t d_min = 0;    // smallest total delay searched; row dt is delay d_min + dt
  int rule = 0;         // 0: one C at the border frequency; 1: two C's (channel labels)
  // rows[l][j]: dt rows of sub-band j after iteration l (l = 0: channel j's
  // Option-1 partial sums; l = levels: the single output sub-band, nd rows).
  std::vector<std::vector<int32_t>> rows;
  // first row of sub-band j inside iteration l's plane
  std::vector<std::vector<int64_t>> row_off;
  // total rows of iteration l's plane
  std::vector<int64_t> total;
  // per iteration l >= 1: the sub-band delays of each plane row
  std::vector<std::vector<int32_t>> d_lo, d_hi, shift;
  // per iteration l >= 1: one MergeRow per row of plane l
  std::vector<std::vector<MergeRow>> merge;
  // per iteration l >= 1: one AdjRow per row of plane l - 1
  std::vector<std::vector<AdjRow>> adj;
  // per channel position: first row of its partial sums in plane 0 and their count
  std::vector<int32_t> leaf_off, leaf_rows;
  // per channel position: the d_min pre-shift, the samples its input is
  // delayed by before the transform (all 0 when d_min = 0; kNoChannelPre
  // where there is no channel)
  std::vector<int32_t> pre;
};

// Builds every table for the delay law dt ~ f^gamma (-2: cold plasma), the
// pre-shift for delays from d_min on and the table rule (0: one C per merge
// at the border frequency; 1: two C's from the channel labels either side).
// Returns "" on success or a description of the problem.
std::string build_tables(Tables &t, int nf, int nd, double f_min, double f_max, double gamma = -2.0,
                         int d_min = 0, int rule = 0);

} // namespace fdmt
