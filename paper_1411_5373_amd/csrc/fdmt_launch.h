// Host launchers of the register-gather kernels (fdmt_gather.hip,
// fdmt_adjoint.hip), called by the step glue in fdmt_kernels.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "fdmt_boxcar.h"
#include "fdmt_device.h"

namespace fdmt {

// Boxcar search fused into the last forward pass: where its tile partials
// go (null: no search), the widths (2^0 .. 2^max_log2) and the tiles per row.
struct SearchTile {
  BoxPartial *part = nullptr;
  int32_t max_log2 = 0;
  int32_t ntiles = 0;
  int32_t rows = 0;     // rows per workgroup of the pass (0: the plan's)
  int32_t threads = 0;  // workgroup size of the pass (0: the plan's)
};

// Geometry of one gather launch: grid, stream, ragged map (used when
// `ragged`), k or tree depth, runs of 4 samples per lane, rows per workgroup.
struct GatherLaunch {
  dim3 grid;
  hipStream_t stream;
  RaggedMap rg;
  bool ragged;
  int depth, vecs, rows_per_wg;
  bool lagged = false;  // adjoint: lagged leaf list (subtrees listed once)
  int tiles_fastest = 0;  // adjoint: run each row group's time tiles back to back (uniform launches)
  int threads = kGatherThreads;  // workgroup size: 64 .. 1024, a multiple of 64 * rows_per_wg
  SearchTile search;             // forward gathers: the fused boxcar search (last pass only)
  bool streaming = false;        // output not read again by this call: non-temporal stores
  int max_chain = -1;            // first pass from the input: longest Option-1 chain (-1: not known)
};

// The register-gather kernels place their waves with shifts: the workgroup
// size and the rows per workgroup must be powers of two, with 64 threads or
// more per row.
inline bool gather_shape_ok(const GatherLaunch &g) {
  const auto pow2 = [](int v) { return v > 0 && (v & (v - 1)) == 0; };
  return pow2(g.threads) && pow2(g.rows_per_wg) && g.threads <= 1024 && 64 * g.rows_per_wg <= g.threads;
}

// Output samples per wave of the adjoint gather: 4 per lane in `cv` runs,
// less the last lane's last run in a lagged pass (it only feeds the lane
// exchange of its neighbour).
constexpr int adjoint_wave_span(int cv, bool lagged) { return 256 * cv - (lagged ? 4 : 0); }

// Register gather of 2^depth plane-l0 terms per output row: loads Tsrc,
// adds in Tacc, stores Tdst (uint16 planes hold exact integer sums).
template <typename Tsrc, typename Tacc, typename Tdst>
hipError_t launch_gather(const GatherLaunch &g, const Tsrc *src, Tdst *dst, const int2 *terms, int32_t nt,
                         int64_t src_stride, int64_t src_bstride, int64_t dst_stride, int64_t dst_bstride,
                         int32_t nrows);

// Register gather of 2^depth Option-1 chain terms straight from the input.
template <typename Tin, typename Tacc, typename Tdst>
hipError_t launch_input_gather(const GatherLaunch &g, const Tin *src, Tdst *dst, const int4 *terms, int32_t nt,
                               int64_t src_bstride, int64_t dst_stride, int64_t dst_bstride, int32_t nrows);

// The same two gathers over uint8 input or uint16 planes when every partial
// sum is an integer below 2^24: int32 sums in any order, a lane owning 4 * vecs
// consecutive samples (vecs 1 or 2). Tdst: uint16_t, int32_t or float from the
// input; uint16_t from a plane.
template <typename Tdst>
hipError_t launch_narrow_input_gather(const GatherLaunch &g, const uint8_t *src, Tdst *dst, const int4 *terms,
                                      int32_t nt, int64_t src_bstride, int64_t dst_stride, int64_t dst_bstride,
                                      int32_t nrows);
template <typename Tdst>
hipError_t launch_narrow_gather(const GatherLaunch &g, const uint16_t *src, Tdst *dst, const int2 *terms,
                                int32_t nt, int64_t src_stride, int64_t src_bstride, int64_t dst_stride,
                                int64_t dst_bstride, int32_t nrows);

// Adjoint register gather over a depth-first leaf list; max_shift bounds the
// shifts of every leaf.
template <typename Tacc>
hipError_t launch_adjoint_gather(const GatherLaunch &g, const Tacc *src, Tacc *dst, const int4 *leaves,
                                 const int32_t *starts, const int32_t *order, int32_t nt, int32_t max_shift,
                                 int64_t src_stride, int64_t src_bstride, int64_t dst_stride, int64_t dst_bstride,
                                 int32_t nrows);

} // namespace fdmt
