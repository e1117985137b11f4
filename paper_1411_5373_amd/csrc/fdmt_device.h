// Device helpers shared by the FDMT kernel translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "fdmt_schedule.h"

namespace fdmt {

template <typename Tacc, typename Tin>
__device__ __forceinline__ Tacc widen(Tin x) {
  return static_cast<Tacc>(x);
}
template <>
__device__ __forceinline__ float widen<float, _Float16>(_Float16 x) {
  return static_cast<float>(x);
}

// Where a workgroup's beam lives. Uniform batches take the beam from
// blockIdx.z and share one Nt; ragged batches look the tile (blockIdx.y) up in
// host-built maps: beam b has its own Nt, its input/output start at
// rows * (samples of the beams before it) and its workspace planes at
// rows * (padded samples before it).
struct RaggedMap {
  const int4 *beam;   // per beam: {nt, padded nt, first sample, first padded sample}
  const int2 *tiles;  // per tile of the launch: {beam, tile within the beam}
  int32_t src_rows, dst_rows;      // rows per beam of the source / destination buffer
  int32_t src_padded, dst_padded;  // 1: workspace plane (row stride = padded nt)
  int32_t reverse;                 // uniform launches: run the time tiles last to first
};

struct BeamSpan {
  int nt, tile;                    // samples of the beam; tile index within the beam
  int beam;                        // uniform batches: the beam (grid z, reversed with the tiles)
  int64_t src_off, dst_off;        // element offsets of the beam in src / dst
  int64_t src_stride, dst_stride;  // row strides (elements)
};

template <bool RAGGED>
__device__ __forceinline__ BeamSpan beam_span(const RaggedMap &rg, int nt, int64_t src_stride,
                                              int64_t src_bstride, int64_t dst_stride,
                                              int64_t dst_bstride) {
  BeamSpan b;
  if constexpr (RAGGED) {
    const int2 tb = rg.tiles[blockIdx.y];
    const int4 bm = rg.beam[tb.x];
    b.nt = bm.x;
    b.tile = tb.y;
    b.beam = 0;
    b.src_off = static_cast<int64_t>(rg.src_rows) * (rg.src_padded ? bm.w : bm.z);
    b.dst_off = static_cast<int64_t>(rg.dst_rows) * (rg.dst_padded ? bm.w : bm.z);
    b.src_stride = rg.src_padded ? bm.y : bm.x;
    b.dst_stride = rg.dst_padded ? bm.y : bm.x;
  } else {
    b.nt = nt;
    b.tile = blockIdx.y;
    b.beam = rg.reverse ? static_cast<int>(gridDim.z - 1 - blockIdx.z) : static_cast<int>(blockIdx.z);
    b.src_off = b.beam * src_bstride;
    b.dst_off = b.beam * dst_bstride;
    b.src_stride = src_stride;
    b.dst_stride = dst_stride;
  }
  return b;
}

__device__ __forceinline__ int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

// The 32-bit word at p, an address the same for every lane, through the scalar
// data cache (a read of data that earlier kernels wrote; caches are
// invalidated at each launch).
__device__ __forceinline__ uint32_t scalar_word(const void *p) {
  const uint64_t a = reinterpret_cast<uint64_t>(p);
  const uint64_t u = static_cast<uint64_t>(static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(a >> 32))))
                         << 32 |
                     static_cast<uint32_t>(__builtin_amdgcn_readfirstlane(static_cast<int>(a)));
  return *reinterpret_cast<const __attribute__((address_space(4))) uint32_t *>(u);
}

// Element offset of row `row` (>= 0) of rows `stride` (< 2^32) elements
// apart: one 32 x 32 -> 64-bit product (two scalar instructions, where a
// signed 64-bit product takes six).
__device__ __forceinline__ int64_t row_offset(int row, int64_t stride) {
  return static_cast<int64_t>(static_cast<uint64_t>(static_cast<uint32_t>(row)) * static_cast<uint32_t>(stride));
}

// Workgroups are dealt round-robin to the 8 XCDs; renumber them so each XCD
// runs a contiguous range of work items (neighbouring blocks share leaf rows
// and time halos through that XCD's L2).
__device__ __forceinline__ int xcd_local_order(int id, int n) {
  const int q = n >> 3, r = n & 7;
  const int x = id & 7, slot = id >> 3;
  return x * q + (x < r ? x : r) + slot;
}



// Place of a wave in a register-gather workgroup of blockDim.x threads that
// holds rows_per_wg rows side by side, col_waves waves along time per row.
// Workgroup sizes and rows per workgroup are powers of two (the launchers
// check), so shifts stand in for the divisions, each of which would cost the
// scalar unit about twenty instructions per wave.
struct WaveLayout {
  int col_waves;  // waves per row
  int groups;     // row groups over nrows rows
  int row;        // the wave's row within the workgroup
  int col;        // the wave's place along time within its row
};

__device__ __forceinline__ WaveLayout wave_layout(int wave, int rows_per_wg, int nrows) {
  const int lr = __builtin_ctz(static_cast<unsigned>(rows_per_wg));
  const int lc = __builtin_ctz(blockDim.x) - 6 - lr;
  WaveLayout w;
  w.col_waves = 1 << lc;
  w.groups = (nrows + rows_per_wg - 1) >> lr;
  w.row = wave >> lc;
  w.col = wave & (w.col_waves - 1);
  return w;
}

// Work item (row group, time tile) of a register-gather launch over
// groups x tiles workgroups. By default (and always for ragged launches,
// whose tile comes from their map: blockIdx.y, returned as -1 here) row
// groups are spread over the XCDs as above and all groups of a tile run
// together, so rows that share terms meet in L2. With `tiles_fastest`, a
// uniform launch deals the whole grid so that each XCD runs a contiguous
// range of row groups with every group's time tiles back to back: a term row
// read at a large shift straddles neighbouring tiles, and the second tile
// finds it in that XCD's L2.
template <bool RAGGED>
__device__ __forceinline__ int2 gather_item(int groups, bool tiles_fastest) {
  if (RAGGED || !tiles_fastest) {
    return make_int2(xcd_local_order(blockIdx.x, groups), RAGGED ? -1 : static_cast<int>(blockIdx.y));
  } else {
    // 32-bit arithmetic: the launcher keeps groups x tiles below 2^31
    const unsigned tiles = gridDim.y;
    const unsigned n = static_cast<unsigned>(groups) * tiles;
    const unsigned id = blockIdx.y * gridDim.x + blockIdx.x;  // dispatch order
    const unsigned q = n >> 3, r = n & 7, x = id & 7, slot = id >> 3;
    const unsigned item = x * q + (x < r ? x : r) + slot;
    return make_int2(static_cast<int>(item / tiles), static_cast<int>(item % tiles));
  }
}

// Block records and headers are read-only for the whole launch and the same
// for every lane of a wave: reading them through the constant address space
// makes them scalar loads.
typedef const __attribute__((address_space(4))) int32_t *ConstInts;

// Largest workgroup of the register-gather kernels (their register budget is
// set for it); a launch may use 64 .. 1024 threads, a power of two.
constexpr int kGatherThreads = 1024;

// Four consecutive elements at 4-byte alignment: one 16-byte global access.
template <typename T>
struct Vec4;
template <>
struct Vec4<float> {
  typedef float type __attribute__((ext_vector_type(4), aligned(4)));
};
template <>
struct Vec4<uint16_t> {
  typedef uint16_t type __attribute__((ext_vector_type(4), aligned(2)));
};
template <>
struct Vec4<int32_t> {
  typedef int type __attribute__((ext_vector_type(4), aligned(4)));
};


} // namespace fdmt
