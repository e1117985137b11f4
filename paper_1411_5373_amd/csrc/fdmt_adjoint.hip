// Register-gather kernel of the adjoint transform.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "fdmt_launch.h"
#include "fdmt_schedule.h"

namespace fdmt {

namespace {

// ---------------------------------------------------------------------------
// Adjoint over several iterations as a register gather. An output row (of
// plane l_lo, or an input channel in the last pass) is a nested sum whose
// leaves are rows of plane l_hi at accumulated shifts (AdjLeaf, host-built in
// depth-first order). One accumulator per tree depth reproduces the order of
// the level-by-level transpose exactly: before a leaf whose path leaves the
// previous one below depth b, the finished nodes deeper than b are added to
// their parents (deepest first) and restarted from zero; each leaf is added
// to its parent at depth K-1. A leaf sample at or past nt is zero, which is
// the transpose's "t + s < nt" rule.
//
// Leaves are loaded a chunk at a time, all eight runs of four samples in
// flight before any is used (four leaves of one run: a longer unrolled chunk
// of single runs needs more registers than the 1024-thread budget allows).
// A wave whose samples, at every shift of the pass, stay below nt (all but
// the last tile of a row) takes the interior path, whose loads need no
// checks; the edge path checks every access.
constexpr int kAdjChunk = 8;
constexpr int adjoint_chunk(int cv) { return cv == 1 ? kAdjChunk / 2 : kAdjChunk / cv; }

// Four lanes' worth of accumulator in registers (naturally aligned; memory
// accesses go through the 4-byte-aligned Vec4).
template <typename T>
using Reg4 = T __attribute__((ext_vector_type(4)));

// Running sums of one output row: one accumulator per tree depth, CV runs of
// 4 samples per lane.
template <typename Tacc, int K, int CV>
struct DepthSums {
  typedef Reg4<Tacc> R;
  R acc[K][CV];

  __device__ __forceinline__ DepthSums() {
#pragma unroll
    for (int d = 0; d < K; ++d)
#pragma unroll
      for (int c = 0; c < CV; ++c) acc[d][c] = R(0);
  }

  // Finished nodes deeper than b into their parents, deepest first; restart them.
  __device__ __forceinline__ void flush_below(int b) {
#pragma unroll
    for (int d = K - 1; d >= 1; --d)
      if (d > b)
#pragma unroll
        for (int c = 0; c < CV; ++c) acc[d - 1][c] = acc[d - 1][c] + acc[d][c];
#pragma unroll
    for (int d = 1; d < K; ++d)
      if (d > b)
#pragma unroll
        for (int c = 0; c < CV; ++c) acc[d][c] = R(0);
  }

  // One leaf whose path branches off the previous leaf's at depth b.
  __device__ __forceinline__ void add(const R (&v)[CV], int b, bool first) {
    if (!first) flush_below(b);
#pragma unroll
    for (int c = 0; c < CV; ++c) acc[K - 1][c] = acc[K - 1][c] + v[c];
  }

  static __device__ __forceinline__ Tacc exchange(int addr, Tacc x) {
    return __builtin_bit_cast(Tacc, __builtin_amdgcn_ds_bpermute(addr, __builtin_bit_cast(int, x)));
  }

  // Lagged pass: the subtree of one partial-sum row (depth 1) is complete;
  // add its values at t + i, i = 0..L-1, to the channel (acc[0]) in lag
  // order. Sample t + q + i of run c is this lane's component q + i, or for
  // q + i >= 4 the next lane's component q + i - 4 (lane 63: lane 0's of run
  // c + 1; lane 63 of the last run is not stored). All 64 lanes take part.
  template <int L>
  __device__ __forceinline__ void add_lags(int lane) {
    const int addr = ((lane + 1) & 63) << 2;
    Tacc next[L > 1 ? L - 1 : 1];
#pragma unroll
    for (int k = 0; k < L - 1; ++k) next[k] = exchange(addr, acc[1][0][k]);
#pragma unroll
    for (int c = 0; c < CV; ++c) {
      Tacc nb[L > 1 ? L - 1 : 1];
#pragma unroll
      for (int k = 0; k < L - 1; ++k) {
        nb[k] = next[k];
        if (c + 1 < CV) {
          next[k] = exchange(addr, acc[1][c + 1][k]);
          if (lane == 63) nb[k] = next[k];
        }
      }
#pragma unroll
      for (int i = 0; i < L; ++i) {
        R sh;
#pragma unroll
        for (int q = 0; q < 4; ++q) sh[q] = q + i < 4 ? acc[1][c][q + i] : nb[q + i - 4];
        acc[0][c] = acc[0][c] + sh;
      }
    }
  }

  __device__ __forceinline__ void finish_subtree(int lags, int lane) {
    if constexpr (K >= 2) {
      flush_below(1);
      switch (lags) {
        case 1: add_lags<1>(lane); break;
        case 2: add_lags<2>(lane); break;
        case 3: add_lags<3>(lane); break;
        default: add_lags<4>(lane); break;
      }
#pragma unroll
      for (int c = 0; c < CV; ++c) acc[1][c] = R(0);
    }
  }
};

// Adds leaves x0 .. x1-1 (the first one flushes nothing), kChunk at a time.
// INTERIOR: t + 256 * CV + max_shift <= nt for the whole wave, so no access
// needs a check; otherwise every run is checked against nt.
template <bool INTERIOR, typename Tacc, int K, int CV>
__device__ __forceinline__ void gather_range(DepthSums<Tacc, K, CV> &sums, const Tacc *base, int64_t stride,
                                             const int4 *__restrict__ leaves, int x0, int x1, int t, int nt) {
  typedef typename Vec4<Tacc>::type V;
  typedef Reg4<Tacc> R;
  constexpr int kChunk = adjoint_chunk(CV);
  static_assert(2 * kChunk <= kAdjLeafPad, "leaf records are read up to two chunks past a list");
  // A chunk's leaf records are one scalar load, issued a chunk ahead (records
  // past the list are read, not used: the list is padded)
  struct Chunk {
    int4 e[kChunk];
  };
  const auto load = [&](R (&v)[CV], const int4 &e) {
    const Tacc *row = base + row_offset(e.x, stride);
    const Tacc *p = row + (t + e.y);  // the runs at constant offsets from one address
#pragma unroll
    for (int c = 0; c < CV; ++c) {
      const int ts = t + 256 * c + e.y;
      if (INTERIOR || ts + 4 <= nt) {
        v[c] = *reinterpret_cast<const V *>(p + 256 * c);
      } else {
#pragma unroll
        for (int i = 0; i < 4; ++i) v[c][i] = ts + i < nt ? row[ts + i] : Tacc(0);
      }
    }
  };
  Chunk cur = *reinterpret_cast<const Chunk *>(leaves + x0);
  int x = x0;
  // Whole chunks load and add every leaf unconditionally: with per-leaf
  // conditions the compiler cannot tell a skipped leaf's load from a pending
  // one, and waited for the first leaf's loads before issuing the second's.
  for (; x + kChunk <= x1; x += kChunk) {
    R v[kChunk][CV];
#pragma unroll
    for (int j = 0; j < kChunk; ++j) load(v[j], cur.e[j]);
    const Chunk next = *reinterpret_cast<const Chunk *>(leaves + x + kChunk);
#pragma unroll
    for (int j = 0; j < kChunk; ++j) sums.add(v[j], cur.e[j].z, x + j == x0);
    cur = next;
  }
  if (x < x1) {
    const int n = x1 - x;
    R v[kChunk][CV];
#pragma unroll
    for (int j = 0; j < kChunk; ++j)
      if (j < n) load(v[j], cur.e[j]);
#pragma unroll
    for (int j = 0; j < kChunk; ++j)
      if (j < n) sums.add(v[j], cur.e[j].z, x + j == x0);
  }
}

// A wave covers 256 * CV consecutive samples (4 per lane, CV runs 256 apart)
// and stores them all, or in a lagged pass all but the last lane's last run:
// those 4 samples only feed the lane exchange, and the next wave starts there.
// NT: the output is not read again by this call (the pass into the channels),
// so its full-run stores are non-temporal.
template <typename Tacc, int K, int CV, bool RAGGED, bool LAG, bool NT>
__global__ __launch_bounds__(kGatherThreads) void adjoint_gather_kernel(
    const Tacc *__restrict__ src, Tacc *__restrict__ dst, const int4 *__restrict__ leaves,
    const int32_t *__restrict__ starts, const int32_t *__restrict__ order, int32_t nt_u, int32_t max_shift,
    int64_t src_stride_u, int64_t src_bstride, int64_t dst_stride_u, int64_t dst_bstride, int32_t nrows,
    int32_t rows_per_wg, int32_t tiles_fastest, RaggedMap rg) {
  typedef typename Vec4<Tacc>::type V;
  constexpr int kSpan = adjoint_wave_span(CV, LAG);
  const int wave = uniform(threadIdx.x / 64), lane = threadIdx.x % 64;
  const WaveLayout wl = wave_layout(wave, rows_per_wg, nrows);
  const int col_waves = wl.col_waves;
  const int2 item = gather_item<RAGGED>(wl.groups, tiles_fastest != 0);
  const int g = item.x;
  const int r = g * rows_per_wg + wl.row;
  if (r >= nrows) return;
  BeamSpan bs = beam_span<RAGGED>(rg, nt_u, src_stride_u, src_bstride, dst_stride_u, dst_bstride);
  if (!RAGGED) bs.tile = rg.reverse ? static_cast<int>(gridDim.y) - 1 - item.y : item.y;
  const int nt = bs.nt;
  const int t_wave = (bs.tile * col_waves + wl.col) * kSpan;
  const int t = t_wave + lane * 4;
  if (LAG ? t_wave >= nt : t >= nt) return;
  const Tacc *base = src + bs.src_off;
  const int x_begin = starts[r], x_end = starts[r + 1];
  const int out_row = order[r];
  DepthSums<Tacc, K, CV> sums;
  auto run = [&](auto interior) {
    constexpr bool kInterior = decltype(interior)::value;
    if constexpr (LAG) {
      // one subtree (a partial-sum row) at a time: its first leaf holds
      // lags | leaves << 3
      for (int x = x_begin; x < x_end;) {
        const int w = leaves[x].w;
        gather_range<kInterior>(sums, base, bs.src_stride, leaves, x, x + (w >> 3), t, nt);
        sums.finish_subtree(w & 7, lane);
        x += w >> 3;
      }
    } else {
      gather_range<kInterior>(sums, base, bs.src_stride, leaves, x_begin, x_end, t, nt);
      sums.flush_below(0);
    }
  };
  if (static_cast<int64_t>(t_wave) + 256 * CV + max_shift <= nt)
    run(std::true_type());
  else
    run(std::false_type());
#pragma unroll
  for (int c = 0; c < CV; ++c) {
    const int tc = t + 256 * c;
    if (LAG && c == CV - 1 && lane == 63) continue;
    Tacc *o = dst + bs.dst_off + out_row * bs.dst_stride + tc;
    if (tc + 4 <= nt) {
      if constexpr (NT)
        __builtin_nontemporal_store(sums.acc[0][c], reinterpret_cast<V *>(o));
      else
        *reinterpret_cast<V *>(o) = sums.acc[0][c];
    } else {
      for (int i = 0; i < 4 && tc + i < nt; ++i) o[i] = sums.acc[0][c][i];
    }
  }
}

} // namespace

template <typename Tacc>
hipError_t launch_adjoint_gather(const GatherLaunch &g, const Tacc *src, Tacc *dst, const int4 *leaves,
                                 const int32_t *starts, const int32_t *order, int32_t nt, int32_t max_shift,
                                 int64_t src_stride, int64_t src_bstride, int64_t dst_stride, int64_t dst_bstride,
                                 int32_t nrows) {
  if (!gather_shape_ok(g)) return hipErrorInvalidValue;
  // the tile-major work order numbers the grid's workgroups in 32 bits
  if (g.tiles_fastest && static_cast<uint64_t>(g.grid.x) * g.grid.y >= (1ull << 31)) return hipErrorInvalidValue;
#define FDMT_ADJ_NT(KK, CC, RR, LL, NN)                                                                       \
  hipLaunchKernelGGL((adjoint_gather_kernel<Tacc, KK, CC, RR, LL, NN>), g.grid, dim3(g.threads), 0, g.stream, \
                     src, dst, leaves, starts, order, nt, max_shift, src_stride, src_bstride, dst_stride,          \
                     dst_bstride, nrows, g.rows_per_wg, g.tiles_fastest, g.rg)
#define FDMT_ADJ(KK, CC, RR, LL)                           \
  if (g.streaming) {                                       \
    FDMT_ADJ_NT(KK, CC, RR, LL, true);                     \
  } else {                                                 \
    FDMT_ADJ_NT(KK, CC, RR, LL, false);                    \
  }
#define FDMT_ADJ_K(CC, RR)                                    \
  if (g.lagged) {                                             \
    switch (g.depth) {                                        \
      case 2: FDMT_ADJ(2, CC, RR, true); break;               \
      case 3: FDMT_ADJ(3, CC, RR, true); break;               \
      case 4: FDMT_ADJ(4, CC, RR, true); break;               \
      case 5: FDMT_ADJ(5, CC, RR, true); break;               \
      default: return hipErrorInvalidValue;                   \
    }                                                         \
  } else {                                                    \
    switch (g.depth) {                                        \
      case 1: FDMT_ADJ(1, CC, RR, false); break;              \
      case 2: FDMT_ADJ(2, CC, RR, false); break;              \
      case 3: FDMT_ADJ(3, CC, RR, false); break;              \
      case 4: FDMT_ADJ(4, CC, RR, false); break;              \
      case 5: FDMT_ADJ(5, CC, RR, false); break;              \
      default: return hipErrorInvalidValue;                   \
    }                                                         \
  }
  if (g.ragged) {
    if (g.vecs == 4) { FDMT_ADJ_K(4, true) } else if (g.vecs == 2) { FDMT_ADJ_K(2, true) } else { FDMT_ADJ_K(1, true) }
  } else {
    if (g.vecs == 4) { FDMT_ADJ_K(4, false) } else if (g.vecs == 2) { FDMT_ADJ_K(2, false) } else { FDMT_ADJ_K(1, false) }
  }
#undef FDMT_ADJ_K
#undef FDMT_ADJ
#undef FDMT_ADJ_NT
  return hipGetLastError();
}

template hipError_t launch_adjoint_gather<float>(const GatherLaunch &, const float *, float *, const int4 *,
                                                 const int32_t *, const int32_t *, int32_t, int32_t, int64_t,
                                                 int64_t, int64_t, int64_t, int32_t);
template hipError_t launch_adjoint_gather<int32_t>(const GatherLaunch &, const int32_t *, int32_t *,
                                                   const int4 *, const int32_t *, const int32_t *, int32_t, int32_t,
                                                   int64_t, int64_t, int64_t, int64_t, int32_t);

} // namespace fdmt
