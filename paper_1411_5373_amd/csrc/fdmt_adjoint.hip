// Register-gather kernel of the adjoint transform.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fdmt_launch.h"

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
// Leaves are loaded kChunk at a time, all eight runs of four samples in
// flight before any is used. A wave whose samples, at every shift of the
// pass, stay below nt (all but the last tile of a row) takes the interior
// path, whose loads need no checks; the edge path checks every access.
constexpr int kAdjChunk = 8;

// Four lanes' worth of accumulator in registers (naturally aligned; memory
// accesses go through the 4-byte-aligned Vec4).
template <typename T>
using Reg4 = T __attribute__((ext_vector_type(4)));

// Adds one leaf (CV runs of 4 samples) whose path branches off the previous
// leaf's at depth b.
template <typename V, int K, int CV>
__device__ __forceinline__ void add_leaf(V (&acc)[K][CV], const V (&v)[CV], int b, bool first) {
  if (!first) {
#pragma unroll
    for (int d = K - 1; d >= 1; --d)
      if (d > b)
#pragma unroll
        for (int c = 0; c < CV; ++c) acc[d - 1][c] = acc[d - 1][c] + acc[d][c];
#pragma unroll
    for (int d = 1; d < K; ++d)
      if (d > b)
#pragma unroll
        for (int c = 0; c < CV; ++c) acc[d][c] = V(0);
  }
#pragma unroll
  for (int c = 0; c < CV; ++c) acc[K - 1][c] = acc[K - 1][c] + v[c];
}

// Interior path: t + 256 * CV + max_shift <= nt for the whole wave.
template <typename Tacc, int K, int CV>
__device__ __forceinline__ void gather_interior(Reg4<Tacc> (&acc)[K][CV], const Tacc *base,
                                                int64_t stride, const int4 *__restrict__ leaves, int x_begin,
                                                int x_end, int t) {
  typedef typename Vec4<Tacc>::type V;
  typedef Reg4<Tacc> R;
  constexpr int kChunk = kAdjChunk / CV;
  for (int x0 = x_begin; x0 < x_end; x0 += kChunk) {
    const int n = x_end - x0 < kChunk ? x_end - x0 : kChunk;
    int br[kChunk];
    R v[kChunk][CV];
#pragma unroll
    for (int j = 0; j < kChunk; ++j) {
      if (j < n) {
        const int4 e = leaves[x0 + j];
        br[j] = e.z;
        const Tacc *row = base + e.x * stride + t + e.y;
#pragma unroll
        for (int c = 0; c < CV; ++c) v[j][c] = *reinterpret_cast<const V *>(row + 256 * c);
      }
    }
#pragma unroll
    for (int j = 0; j < kChunk; ++j)
      if (j < n) add_leaf<R, K, CV>(acc, v[j], br[j], x0 + j == x_begin);
  }
}

// Edge path: every run checked against nt.
template <typename Tacc, int K, int CV>
__device__ __forceinline__ void gather_edge(Reg4<Tacc> (&acc)[K][CV], const Tacc *base,
                                            int64_t stride, const int4 *__restrict__ leaves, int x_begin,
                                            int x_end, int t, int nt) {
  typedef typename Vec4<Tacc>::type V;
  typedef Reg4<Tacc> R;
  constexpr int kChunk = kAdjChunk / CV;
  for (int x0 = x_begin; x0 < x_end; x0 += kChunk) {
    const int n = x_end - x0 < kChunk ? x_end - x0 : kChunk;
    int4 e[kChunk];
    R v[kChunk][CV];
#pragma unroll
    for (int j = 0; j < kChunk; ++j) {
      if (j < n) {
        e[j] = leaves[x0 + j];
        const Tacc *row = base + e[j].x * stride;
#pragma unroll
        for (int c = 0; c < CV; ++c) {
          const int ts = t + 256 * c + e[j].y;
          if (ts + 4 <= nt) {
            v[j][c] = *reinterpret_cast<const V *>(row + ts);
          } else {
#pragma unroll
            for (int i = 0; i < 4; ++i) v[j][c][i] = ts + i < nt ? row[ts + i] : Tacc(0);
          }
        }
      }
    }
#pragma unroll
    for (int j = 0; j < kChunk; ++j)
      if (j < n) add_leaf<R, K, CV>(acc, v[j], e[j].z, x0 + j == x_begin);
  }
}

template <typename Tacc, int K, int CV, bool RAGGED>
__global__ __launch_bounds__(kGatherThreads) void adjoint_gather_kernel(
    const Tacc *__restrict__ src, Tacc *__restrict__ dst, const int4 *__restrict__ leaves,
    const int32_t *__restrict__ starts, const int32_t *__restrict__ order, int32_t nt_u, int32_t max_shift,
    int64_t src_stride_u, int64_t src_bstride, int64_t dst_stride_u, int64_t dst_bstride, int32_t nrows,
    int32_t rows_per_wg, RaggedMap rg) {
  typedef typename Vec4<Tacc>::type V;
  typedef Reg4<Tacc> R;
  const int waves = kGatherThreads / 64;
  const int wave = uniform(threadIdx.x / 64), lane = threadIdx.x % 64;
  const int col_waves = waves / rows_per_wg;
  const int groups = (nrows + rows_per_wg - 1) / rows_per_wg;
  const int g = xcd_local_order(blockIdx.x, groups);
  const int r = g * rows_per_wg + wave / col_waves;
  if (r >= nrows) return;
  const BeamSpan bs = beam_span<RAGGED>(rg, nt_u, src_stride_u, src_bstride, dst_stride_u, dst_bstride);
  const int nt = bs.nt;
  const int t_wave = (bs.tile * col_waves + wave % col_waves) * 256 * CV;
  const int t = t_wave + lane * 4;
  if (t >= nt) return;
  const Tacc *base = src + bs.src_off;
  const int x_begin = starts[r], x_end = starts[r + 1];
  const int out_row = order[r];
  R acc[K][CV];
#pragma unroll
  for (int d = 0; d < K; ++d)
#pragma unroll
    for (int c = 0; c < CV; ++c) acc[d][c] = R(0);
  if (t_wave + 256 * CV + max_shift <= nt)
    gather_interior<Tacc, K, CV>(acc, base, bs.src_stride, leaves, x_begin, x_end, t);
  else
    gather_edge<Tacc, K, CV>(acc, base, bs.src_stride, leaves, x_begin, x_end, t, nt);
#pragma unroll
  for (int d = K - 1; d >= 1; --d)
#pragma unroll
    for (int c = 0; c < CV; ++c) acc[d - 1][c] = acc[d - 1][c] + acc[d][c];
#pragma unroll
  for (int c = 0; c < CV; ++c) {
    const int tc = t + 256 * c;
    Tacc *o = dst + bs.dst_off + out_row * bs.dst_stride + tc;
    if (tc + 4 <= nt) {
      *reinterpret_cast<V *>(o) = acc[0][c];
    } else {
      for (int i = 0; i < 4 && tc + i < nt; ++i) o[i] = acc[0][c][i];
    }
  }
}

} // namespace

template <typename Tacc>
hipError_t launch_adjoint_gather(const GatherLaunch &g, const Tacc *src, Tacc *dst, const int4 *leaves,
                                 const int32_t *starts, const int32_t *order, int32_t nt, int32_t max_shift,
                                 int64_t src_stride, int64_t src_bstride, int64_t dst_stride, int64_t dst_bstride,
                                 int32_t nrows) {
#define FDMT_ADJ(KK, CC, RR)                                                                              \
  hipLaunchKernelGGL((adjoint_gather_kernel<Tacc, KK, CC, RR>), g.grid, dim3(kGatherThreads), 0, g.stream, src, \
                     dst, leaves, starts, order, nt, max_shift, src_stride, src_bstride, dst_stride, dst_bstride, \
                     nrows, g.rows_per_wg, g.rg)
#define FDMT_ADJ_K(CC, RR)             \
  switch (g.depth) {                   \
    case 1: FDMT_ADJ(1, CC, RR); break; \
    case 2: FDMT_ADJ(2, CC, RR); break; \
    case 3: FDMT_ADJ(3, CC, RR); break; \
    case 4: FDMT_ADJ(4, CC, RR); break; \
    case 5: FDMT_ADJ(5, CC, RR); break; \
    default: return hipErrorInvalidValue; \
  }
  if (g.ragged) {
    if (g.vecs == 4) { FDMT_ADJ_K(4, true) } else if (g.vecs == 2) { FDMT_ADJ_K(2, true) } else { FDMT_ADJ_K(1, true) }
  } else {
    if (g.vecs == 4) { FDMT_ADJ_K(4, false) } else if (g.vecs == 2) { FDMT_ADJ_K(2, false) } else { FDMT_ADJ_K(1, false) }
  }
#undef FDMT_ADJ_K
#undef FDMT_ADJ
  return hipGetLastError();
}

template hipError_t launch_adjoint_gather<float>(const GatherLaunch &, const float *, float *, const int4 *,
                                                 const int32_t *, const int32_t *, int32_t, int32_t, int64_t,
                                                 int64_t, int64_t, int64_t, int32_t);
template hipError_t launch_adjoint_gather<int32_t>(const GatherLaunch &, const int32_t *, int32_t *,
                                                   const int4 *, const int32_t *, const int32_t *, int32_t, int32_t,
                                                   int64_t, int64_t, int64_t, int64_t, int32_t);

} // namespace fdmt
