// FDMT kernels for gfx950 (CDNA4): Option-1 initialisation, the iteration
// merges of Algorithm 1 and their transposes.
//
// Data layout: a plane holds every sub-band of one iteration, rows of a
// sub-band consecutive, sub-bands in frequency order, time contiguous, row
// stride `ntp` (padded to 64 samples) inside the workspace, `nt` in user
// buffers. The work is a gather-add along time: no contraction, so no MFMA;
// every kernel streams rows with coalesced loads (lane i reads sample base+i).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <type_traits>

#include "fdmt_launch.h"
#include "fdmt_plan.h"

namespace fdmt {

namespace {

constexpr int kThreads = 256;
constexpr int kPerThread = 4;
constexpr int kTile = kThreads * kPerThread;  // samples per workgroup

// ---------------------------------------------------------------------------
// Option-1 initialisation (Sec. 4): row d of channel k holds
// sum_{i=0}^{d} I[k][t - i], zero before t = 0. Grid: (channel position, time
// tile, beam); a position without a channel has its input delayed past every
// record and writes its row as zeros.
template <typename Tin, typename Tacc, bool RAGGED>
__global__ __launch_bounds__(kThreads) void init_kernel(
    const Tin *__restrict__ in, Tacc *__restrict__ out, const int32_t *__restrict__ leaf_off,
    const int32_t *__restrict__ leaf_rows, const int32_t *__restrict__ pre, int64_t nt_u, int64_t in_bstride,
    int64_t out_stride_u, int64_t out_bstride, RaggedMap rg) {
  const int k = blockIdx.x;
  const BeamSpan bs = beam_span<RAGGED>(rg, static_cast<int>(nt_u), nt_u, in_bstride, out_stride_u, out_bstride);
  const int64_t nt = bs.nt, out_stride = bs.dst_stride;
  // channel k's input delayed by its pre-shift: sample t reads x[t - pre]
  const int64_t sh = pre[k];
  const Tin *x = in + bs.src_off + static_cast<int64_t>(k) * nt;
  Tacc *o = out + bs.dst_off + static_cast<int64_t>(leaf_off[k]) * out_stride;
  const int n = leaf_rows[k];
#pragma unroll
  for (int i = 0; i < kPerThread; ++i) {
    const int64_t t = static_cast<int64_t>(bs.tile) * kTile + i * kThreads + threadIdx.x;
    if (t >= nt) break;
    Tacc acc = 0;
    for (int d = 0; d < n; ++d) {
      if (t - sh - d >= 0) acc += widen<Tacc>(x[t - sh - d]);
      o[d * out_stride + t] = acc;
    }
  }
}

// The input copied to 2^levels channel rows with zeros past row nf, so that
// every channel position of the tree has an input row. Grid: (channel
// position, time tile, beam).
template <typename Tin, bool RAGGED>
__global__ __launch_bounds__(kThreads) void pad_input_kernel(const Tin *__restrict__ in, Tin *__restrict__ out,
                                                             int32_t nf, int64_t nt_u, int64_t in_bstride,
                                                             int64_t out_bstride, RaggedMap rg) {
  const int k = blockIdx.x;
  const BeamSpan bs = beam_span<RAGGED>(rg, static_cast<int>(nt_u), nt_u, in_bstride, nt_u, out_bstride);
  const int64_t nt = bs.nt;
  const Tin *x = in + bs.src_off + static_cast<int64_t>(k) * nt;
  Tin *o = out + bs.dst_off + static_cast<int64_t>(k) * nt;
#pragma unroll
  for (int i = 0; i < kPerThread; ++i) {
    const int64_t t = static_cast<int64_t>(bs.tile) * kTile + i * kThreads + threadIdx.x;
    if (t >= nt) break;
    o[t] = k < nf ? x[t] : Tin(0);
  }
}

// The same copy for a uniform batch whose beam blocks are 16-byte aligned: a
// beam's padded block is its input block followed by zeros, copied in
// 16-byte units. Grid: (chunks, beam).
__global__ __launch_bounds__(kThreads) void pad_flat_kernel(const uint4 *__restrict__ in, uint4 *__restrict__ out,
                                                            int64_t in_vecs, int64_t out_vecs) {
  const int64_t b = blockIdx.y;
  const uint4 *x = in + b * in_vecs;
  uint4 *o = out + b * out_vecs;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; i < out_vecs;
       i += static_cast<int64_t>(gridDim.x) * kThreads)
    o[i] = i < in_vecs ? x[i] : make_uint4(0u, 0u, 0u, 0u);
}

// One iteration: out[r][t] = prev[lo][t] + (t >= s ? prev[hi][t - s] : 0).
// Grid: (plane row, time tile, beam).
template <typename Tacc, bool RAGGED>
__global__ __launch_bounds__(kThreads) void merge_kernel(
    const Tacc *__restrict__ prev, Tacc *__restrict__ next, const int4 *__restrict__ rows,
    int64_t nt_u, int64_t prev_stride_u, int64_t prev_bstride, int64_t next_stride_u,
    int64_t next_bstride, RaggedMap rg) {
  const int r = blockIdx.x;
  const BeamSpan bs = beam_span<RAGGED>(rg, static_cast<int>(nt_u), prev_stride_u, prev_bstride, next_stride_u, next_bstride);
  const int64_t nt = bs.nt;
  const int4 e = rows[r];
  const Tacc *lo = prev + bs.src_off + static_cast<int64_t>(e.x) * bs.src_stride;
  const Tacc *hi = prev + bs.src_off + static_cast<int64_t>(e.y) * bs.src_stride;
  Tacc *o = next + bs.dst_off + static_cast<int64_t>(r) * bs.dst_stride;
  const int64_t s = e.z;
#pragma unroll
  for (int i = 0; i < kPerThread; ++i) {
    const int64_t t = static_cast<int64_t>(bs.tile) * kTile + i * kThreads + threadIdx.x;
    if (t >= nt) break;
    Tacc v = lo[t];
    if (t >= s) v += hi[t - s];
    o[t] = v;
  }
}

// Transpose of one iteration: child row r of plane l-1 gathers the `count`
// consecutive parent rows that read it, in ascending dt, shifted back by the
// parent's s if it is their upper half. Grid: (child row, time tile, beam).
template <typename Tacc, bool RAGGED>
__global__ __launch_bounds__(kThreads) void merge_adjoint_kernel(
    const Tacc *__restrict__ parent, Tacc *__restrict__ child, const int4 *__restrict__ adj,
    const int4 *__restrict__ fwd, int64_t nt_u, int64_t parent_stride_u, int64_t parent_bstride,
    int64_t child_stride_u, int64_t child_bstride, RaggedMap rg) {
  const int r = blockIdx.x;
  const BeamSpan bs = beam_span<RAGGED>(rg, static_cast<int>(nt_u), parent_stride_u, parent_bstride, child_stride_u, child_bstride);
  const int64_t nt = bs.nt, parent_stride = bs.src_stride;
  const int4 a = adj[r];
  const Tacc *g = parent + bs.src_off;
  Tacc *o = child + bs.dst_off + static_cast<int64_t>(r) * bs.dst_stride;
#pragma unroll
  for (int i = 0; i < kPerThread; ++i) {
    const int64_t t = static_cast<int64_t>(bs.tile) * kTile + i * kThreads + threadIdx.x;
    if (t >= nt) break;
    Tacc acc = 0;
    for (int p = a.x; p < a.x + a.y; ++p) {
      const int64_t s = a.z ? fwd[p].z : 0;
      if (t + s < nt) acc += g[static_cast<int64_t>(p) * parent_stride + t + s];
    }
    o[t] = acc;
  }
}

// Transpose of the initialisation: grad_I[k][t] = sum_d sum_{i<=d} P_bar[d][t + i].
// Grid: (channel, time tile, beam).
template <typename Tacc, bool RAGGED>
__global__ __launch_bounds__(kThreads) void init_adjoint_kernel(
    const Tacc *__restrict__ plane, Tacc *__restrict__ out, const int32_t *__restrict__ leaf_off,
    const int32_t *__restrict__ leaf_rows, const int32_t *__restrict__ pre, int64_t nt_u, int64_t plane_stride_u,
    int64_t plane_bstride, int64_t out_bstride, RaggedMap rg) {
  const int k = blockIdx.x;
  const BeamSpan bs = beam_span<RAGGED>(rg, static_cast<int>(nt_u), plane_stride_u, plane_bstride, nt_u, out_bstride);
  const int64_t nt = bs.nt, plane_stride = bs.src_stride;
  const int64_t sh = pre[k];  // transpose of the pre-shift: reads t + pre
  const Tacc *g = plane + bs.src_off + static_cast<int64_t>(leaf_off[k]) * plane_stride;
  Tacc *o = out + bs.dst_off + static_cast<int64_t>(k) * nt;
  const int n = leaf_rows[k];
#pragma unroll
  for (int i = 0; i < kPerThread; ++i) {
    const int64_t t = static_cast<int64_t>(bs.tile) * kTile + i * kThreads + threadIdx.x;
    if (t >= nt) break;
    Tacc acc = 0;
    for (int d = 0; d < n; ++d)
      for (int j = 0; j <= d; ++j)
        if (t + sh + j < nt) acc += g[d * plane_stride + t + sh + j];
    o[t] = acc;
  }
}

// ---------------------------------------------------------------------------
// Fused pass: iterations l0+1 .. l1 of one block (a row range of one sub-band
// of plane l1) over one time tile, every intermediate plane held in LDS.
//
// The host flattens the block's dependency tree into per-row records (Rec):
// level 0 rows are staged from global memory into LDS buffer A, level i is
// merged from the buffer of level i-1 into the other buffer, and the top
// level goes straight to global memory. Each output element is the same
// single addition lower[d_lo][t] + upper[d_hi][t - s] (or the copy rule) as
// in the per-iteration kernels, so every schedule gives identical bits.
//
// Work split: rows are dealt round-robin to the waves. A lane handles columns
// lane + 64*j, so each LDS access of a wave touches 64 consecutive words (no
// bank conflicts) and each global access is a coalesced 256-byte run; whole
// 256-column chunks run without bounds or copy-rule checks.
constexpr int kFusedThreads = 512;
constexpr int kWaves = kFusedThreads / 64;

struct FusedArgs {
  const void *src;      // input [beam][Nf][Nt] (first pass) or plane l0
  void *dst;            // plane l1 or the user output
  const Rec *recs;      // this pass's records
  const int32_t *heads; // this pass's block headers (kRecHeader each)
  int64_t src_stride, src_bstride, dst_stride, dst_bstride;
  int32_t nt, k, nblocks, tile, lds_a, lds_b;
  int32_t tiles_per_wg; // consecutive time tiles one workgroup runs
};

// Option-1 partial sum of chain length n at column c: x[c] + x[c-1] + ... + x[c-n].
template <typename Tacc>
__device__ __forceinline__ Tacc chain(const Tacc *x, int c, int n) {
  Tacc v = x[c];
  for (int d = 1; d <= n; ++d) v += x[c - d];
  return v;
}

// Leaf rows a wave keeps in flight in registers: two rows of up to 512
// columns (8 per lane). Rows beyond the first two of a wave, and columns past
// 512, are staged synchronously.
template <typename Tacc>
struct StageRegs {
  Tacc v[2][8];
  int wd[2], dst[2];
};


__device__ __forceinline__ Rec load_rec(ConstInts recs, int q) {
  const ConstInts r = recs + 8 * q;
  return Rec{r[0], r[1], r[2], r[3], r[4], r[5], r[6], r[7]};
}

template <typename Tin, typename Tacc, bool FROM_INPUT, bool RAGGED>
__global__ __launch_bounds__(kFusedThreads) void fused_pass_kernel(FusedArgs a, RaggedMap rg) {
  typedef typename std::conditional<FROM_INPUT, Tin, Tacc>::type Tsrc;
  extern __shared__ __align__(16) unsigned char smem[];
  Tacc *buf_a = reinterpret_cast<Tacc *>(smem);
  Tacc *buf_b = buf_a + a.lds_a + kLdsSlack;

  const int blk = xcd_local_order(blockIdx.x, a.nblocks);
  const BeamSpan bs = beam_span<RAGGED>(rg, a.nt, a.src_stride, a.src_bstride, a.dst_stride, a.dst_bstride);
  const int nt = bs.nt;
  const int tile_first = bs.tile * a.tiles_per_wg;
  const int ntiles = (nt + a.tile - 1) / a.tile;
  const int tile_end = tile_first + a.tiles_per_wg < ntiles ? tile_first + a.tiles_per_wg : ntiles;
  const int wave = uniform(threadIdx.x / 64);
  const int lane = threadIdx.x % 64;
  const ConstInts head = (ConstInts)(a.heads) + blk * kRecHeader;
  const ConstInts rec = (ConstInts)(a.recs) + 8 * head[0];
  const int nstage = head[1];
  const Tsrc *in_base = static_cast<const Tsrc *>(a.src) + bs.src_off;
  const int64_t in_stride = FROM_INPUT ? static_cast<int64_t>(nt) : bs.src_stride;
  Tacc *out_base = static_cast<Tacc *>(a.dst) + bs.dst_off;

  // Leaf rows q0 and q0 + kWaves of the tile at T0 (first 512 columns) into
  // registers, zero outside [0, nt); every load is issued before any use.
  auto issue = [&](int q0, int T0, StageRegs<Tacc> &r) {
#pragma unroll
    for (int m = 0; m < 2; ++m) {
      const int q = q0 + m * kWaves;
      r.wd[m] = 0;
      r.dst[m] = 0;
      if (q < nstage) {
        const Rec e = load_rec(rec, q);
        const int t0 = T0 - e.d;
        const Tsrc *row = in_base + static_cast<int64_t>(e.a) * in_stride;
        r.wd[m] = e.e;
        r.dst[m] = e.c;
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          const int c = 64 * j + lane;
          const int t = t0 + c;
          r.v[m][j] = (c < e.e && t >= 0 && t < nt) ? widen<Tacc>(row[t]) : Tacc(0);
        }
      }
    }
  };
  auto store = [&](const StageRegs<Tacc> &r) {
#pragma unroll
    for (int m = 0; m < 2; ++m) {
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        const int c = 64 * j + lane;
        if (c < r.wd[m]) buf_a[r.dst[m] + c] = r.v[m][j];
      }
    }
  };
  // Writes the prefetched rows to LDS, then stages the wave's other rows
  // (two at a time) and the columns past 512 of any row.
  auto commit = [&](int T0, const StageRegs<Tacc> &r) {
    store(r);
    for (int q0 = wave + 2 * kWaves; q0 < nstage; q0 += 2 * kWaves) {
      StageRegs<Tacc> t;
      issue(q0, T0, t);
      store(t);
    }
    for (int q = wave; q < nstage; q += kWaves) {
      const Rec e = load_rec(rec, q);
      if (e.e <= 512) continue;
      const int t0 = T0 - e.d;
      const Tsrc *row = in_base + static_cast<int64_t>(e.a) * in_stride;
      for (int c = 512 + lane; c < e.e; c += 64) {
        const int t = t0 + c;
        buf_a[e.c + c] = (t >= 0 && t < nt) ? widen<Tacc>(row[t]) : Tacc(0);
      }
    }
  };

  // One merged row: o[c] = lower[c] (+ chains) + (c >= c_hi ? upper[c] : 0)
  // for c < w, lanes on columns lane + 64j. LDS operands may be read up to 63
  // columns past a row's end (the buffers carry that much slack); those
  // columns are never written. `limit` < w only at the end of the record.
  auto merge_row = [&](const Rec &e, const Tacc *S, auto o, int T0, int w, bool chained) {
    const int c_hi = e.d - T0;  // first column with t - s >= 0
    const Tacc *pl = S + e.a + lane;
    const Tacc *ph = S + e.b + lane;
    if (chained) {
      const int gl = e.g, gh = e.h;
      for (int c0 = 0; c0 < w; c0 += 64) {
        Tacc v = chain(pl, c0, gl);
        if (c0 + lane >= c_hi) v += chain(ph, c0, gh);
        if (c0 + lane < w) o[c0] = v;
      }
      return;
    }
    if (c_hi > 0) {
      for (int c0 = 0; c0 < w; c0 += 64) {
        Tacc v = pl[c0];
        if (c0 + lane >= c_hi) v += ph[c0];
        if (c0 + lane < w) o[c0] = v;
      }
      return;
    }
    const int full = w & ~63;
    int c0 = 0;
    for (; c0 + 256 <= full; c0 += 256) {
      const Tacc v0 = pl[c0] + ph[c0];
      const Tacc v1 = pl[c0 + 64] + ph[c0 + 64];
      const Tacc v2 = pl[c0 + 128] + ph[c0 + 128];
      const Tacc v3 = pl[c0 + 192] + ph[c0 + 192];
      o[c0] = v0;
      o[c0 + 64] = v1;
      o[c0 + 128] = v2;
      o[c0 + 192] = v3;
    }
    for (; c0 < full; c0 += 64) o[c0] = pl[c0] + ph[c0];
    if (c0 < w) {
      const Tacc v = pl[c0] + ph[c0];
      if (c0 + lane < w) o[c0] = v;
    }
  };

  StageRegs<Tacc> regs;
  if (tile_first < tile_end) issue(wave, tile_first * a.tile, regs);
  for (int tl = tile_first; tl < tile_end; ++tl) {
    const int T0 = tl * a.tile;
    commit(T0, regs);
    __syncthreads();
    // The next tile's leaves are in flight while this tile's levels run.
    if (tl + 1 < tile_end) issue(wave, T0 + a.tile, regs);

    for (int i = 1; i <= a.k; ++i) {
      const Tacc *S = (i & 1) ? buf_a : buf_b;
      Tacc *D = (i & 1) ? buf_b : buf_a;
      const bool chained = FROM_INPUT && i == 1;
      const int qe = head[1 + i];
      if (i < a.k) {
        for (int q = head[i] + wave; q < qe; q += kWaves) {
          const Rec e = load_rec(rec, q);
          merge_row(e, S, D + e.c + lane, T0, e.e, chained);
        }
      } else {
        const int w = nt - T0 < a.tile ? nt - T0 : a.tile;
        for (int q = head[i] + wave; q < qe; q += kWaves) {
          const Rec e = load_rec(rec, q);
          merge_row(e, S, out_base + e.c * bs.dst_stride + T0 + lane, T0, w, chained);
        }
      }
      __syncthreads();
    }
  }
}

struct View {
  void *ptr;
  int64_t stride, bstride;
};

// ---------------------------------------------------------------------------
// Staged gather over k fused iterations. A block is a row range of one
// sub-band of plane l1; a workgroup keeps the block's tables in LDS and
// streams over a run of time tiles. Per tile it stages, once each, the rows
// of plane l0 (or the input channels) its outputs read, zero outside
// [0, nt); in the first pass it then builds each channel's Option-1 partial
// sums from the staged input in LDS, in the chain order x[t] + x[t-1] + ...
// Each output element is the sum of its 2^k terms (row of plane l0,
// accumulated shift) read from LDS, added as the recursion adds them:
// sibling pairs first, lower half before upper half. A term before the
// record start reads a staged zero, so the copy rule needs no branch and
// every result equals the per-iteration kernels' bit for bit.
//
// Latency: the next tile's staging loads are issued into registers before
// the current tile's outputs are computed, so they are in flight meanwhile.
// Staging is one flat copy of 4-sample quads (thread x moves quads x,
// x + 512, ...); the compute loop gives each wave whole output rows and each
// lane the columns lane + 64*j, so every LDS read of a wave is 64 consecutive
// words (no bank conflicts).
constexpr int kStagedThreads = 512;
constexpr int kStagedWaves = kStagedThreads / 64;
constexpr int kStageQuads = kMaxStagedQuads / kStagedThreads;  // quads per thread in registers

struct StagedArgs {
  const void *src;      // input [beam][Nf][Nt] (first pass) or plane l0
  void *dst;            // plane l1 or the user output
  const Rec *stage;     // this pass's staging records
  const Rec *psums;     // this pass's partial-sum records (first pass)
  const int2 *terms;    // this pass's terms {LDS offset at column 0, unused}
  const int32_t *heads; // this pass's block headers
  int64_t src_stride, src_bstride, dst_stride, dst_bstride;
  int32_t nt, nblocks, tile, ntiles, tiles_per_wg, lds_rec, lds_prec, lds_term;
};

template <typename Tacc, int N>
struct TreeSum {
  static __device__ __forceinline__ void eval(const int2 *tm, const Tacc *lds, int col, Tacc out[4]) {
    Tacc l[4], r[4];
    TreeSum<Tacc, N / 2>::eval(tm, lds, col, l);
    TreeSum<Tacc, N / 2>::eval(tm + N / 2, lds, col, r);
#pragma unroll
    for (int j = 0; j < 4; ++j) out[j] = l[j] + r[j];
  }
};
template <typename Tacc>
struct TreeSum<Tacc, 1> {
  static __device__ __forceinline__ void eval(const int2 *tm, const Tacc *lds, int col, Tacc out[4]) {
    const Tacc *p = lds + tm[0].x + col;
#pragma unroll
    for (int j = 0; j < 4; ++j) out[j] = p[64 * j];
  }
};

template <typename Tsrc, typename Tacc>
struct Stager {
  Tacc v[kStageQuads][4];
  int dst[kStageQuads];

  // Loads this thread's quads of the tile starting at T0 into registers.
  __device__ __forceinline__ void load(const Tsrc *base, const int4 *lrec, int total, int qpr,
                                       uint32_t magic, int T0, int nt, int64_t row_stride) {
#pragma unroll
    for (int u = 0; u < kStageQuads; ++u) {
      const int q = threadIdx.x + u * kStagedThreads;
      dst[u] = -1;
      if (q < total) {
        const int row = static_cast<int>(__umulhi(static_cast<uint32_t>(q), magic));
        const int col = 4 * (q - row * qpr);
        const int4 e = lrec[row];  // {source row, LDS offset, win, padded width}
        if (col < e.w) {
          dst[u] = e.y + col;
          const int t = T0 - e.z + col;
          const Tsrc *src = base + static_cast<int64_t>(e.x) * row_stride;
          if (t >= 0 && t + 4 <= nt) {
            if constexpr (std::is_same<Tsrc, Tacc>::value) {
              const typename Vec4<Tacc>::type w = *reinterpret_cast<const typename Vec4<Tacc>::type *>(src + t);
#pragma unroll
              for (int i = 0; i < 4; ++i) v[u][i] = w[i];
            } else {
#pragma unroll
              for (int i = 0; i < 4; ++i) v[u][i] = widen<Tacc>(src[t + i]);
            }
          } else {
#pragma unroll
            for (int i = 0; i < 4; ++i)
              v[u][i] = (t + i >= 0 && t + i < nt) ? widen<Tacc>(src[t + i]) : Tacc(0);
          }
        }
      }
    }
  }

  // Writes the quads to LDS (16-byte aligned: offsets and columns are multiples of 4).
  __device__ __forceinline__ void store(Tacc *lds) const {
    typedef Tacc V4 __attribute__((ext_vector_type(4)));
#pragma unroll
    for (int u = 0; u < kStageQuads; ++u) {
      if (dst[u] >= 0) {
        V4 w;
#pragma unroll
        for (int i = 0; i < 4; ++i) w[i] = v[u][i];
        *reinterpret_cast<V4 *>(lds + dst[u]) = w;
      }
    }
  }
};

template <typename Tin, typename Tacc, bool FROM_INPUT, int K>
__global__ __launch_bounds__(kStagedThreads) void staged_pass_kernel(StagedArgs a) {
  constexpr int N = 1 << K;
  typedef typename std::conditional<FROM_INPUT, Tin, Tacc>::type Tsrc;
  extern __shared__ __align__(16) unsigned char smem[];
  Tacc *lds = reinterpret_cast<Tacc *>(smem);
  int4 *lrec = reinterpret_cast<int4 *>(reinterpret_cast<int32_t *>(smem) + a.lds_rec);
  int4 *lprec = reinterpret_cast<int4 *>(reinterpret_cast<int32_t *>(smem) + a.lds_prec);
  int2 *lterm = reinterpret_cast<int2 *>(reinterpret_cast<int32_t *>(smem) + a.lds_term);

  const int nchunks = (a.ntiles + a.tiles_per_wg - 1) / a.tiles_per_wg;
  const int w = xcd_local_order(blockIdx.x, a.nblocks * nchunks);
  const int blk = w % a.nblocks;
  const int tile_begin = (w / a.nblocks) * a.tiles_per_wg;
  const int tile_end = tile_begin + a.tiles_per_wg < a.ntiles ? tile_begin + a.tiles_per_wg : a.ntiles;
  const int64_t beam = blockIdx.z;
  const int32_t *head = a.heads + blk * kStagedHeader;
  const int nstage = head[1], nout = head[3], qpr = head[5], npsum = head[8];
  const uint32_t magic = static_cast<uint32_t>(head[6]);
  const int wave = uniform(threadIdx.x / 64);
  const int lane = threadIdx.x % 64;

  // Block tables into LDS.
  {
    const Rec *gs = a.stage + head[0];
    for (int x = threadIdx.x; x < nstage; x += kStagedThreads) {
      const Rec e = gs[x];
      lrec[x] = make_int4(e.a, e.c, e.d, e.e);
    }
    if (FROM_INPUT) {
      const Rec *gp = a.psums + head[7];
      for (int x = threadIdx.x; x < npsum; x += kStagedThreads) {
        const Rec e = gp[x];
        lprec[2 * x] = make_int4(e.a, e.b, e.c, e.d);
        lprec[2 * x + 1] = make_int4(e.e, e.f, 0, 0);
      }
    }
    const int2 *gt = a.terms + head[2];
    for (int x = threadIdx.x; x < nout * N; x += kStagedThreads) lterm[x] = gt[x];
  }
  __syncthreads();

  const Tsrc *base = static_cast<const Tsrc *>(a.src) + beam * a.src_bstride;
  const int64_t row_stride = FROM_INPUT ? static_cast<int64_t>(a.nt) : a.src_stride;
  const int total = nstage * qpr;
  Stager<Tsrc, Tacc> st;
  st.load(base, lrec, total, qpr, magic, tile_begin * a.tile, a.nt, row_stride);

  for (int tile = tile_begin; tile < tile_end; ++tile) {
    const int T0 = tile * a.tile;
    st.store(lds);
    __syncthreads();
    if (FROM_INPUT) {
      // Option-1 partial sums of each channel, rows 0 .. d_last.
      for (int j = wave; j < npsum; j += kStagedWaves) {
        const int4 e = lprec[2 * j];       // {LDS row 0, LDS input row, d_last, row stride}
        const int4 f = lprec[2 * j + 1];   // {width, input columns ahead}
        const Tacc *x = lds + e.y + f.y;
        for (int c = lane; c < f.x; c += 64) {
          Tacc acc = x[c];
          lds[e.x + c] = acc;
          for (int d = 1; d <= e.z; ++d) {
            acc += x[c - d];
            lds[e.x + d * e.w + c] = acc;
          }
        }
      }
      __syncthreads();
    }
    if (tile + 1 < tile_end)
      st.load(base, lrec, total, qpr, magic, T0 + a.tile, a.nt, row_stride);
    const int cmax = a.nt - T0 < a.tile ? a.nt - T0 : a.tile;
    for (int r = wave; r < nout; r += kStagedWaves) {
      int2 tm[N];
#pragma unroll
      for (int j = 0; j < N; ++j) tm[j] = lterm[r * N + j];
      Tacc *o = static_cast<Tacc *>(a.dst) + beam * a.dst_bstride +
                (head[4] + r) * a.dst_stride + T0;
      for (int c0 = 0; c0 < a.tile; c0 += 256) {
        Tacc acc[4];
        TreeSum<Tacc, N>::eval(tm, lds, c0 + lane, acc);
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const int c = c0 + 64 * j + lane;
          if (c < cmax) o[c] = acc[j];
        }
      }
    }
    __syncthreads();
  }
}

size_t fused_lds_bytes(const Pass &ps) {
  if (ps.kind == PassKind::Staged)  // staged rows, partial sums, records, terms (4-byte units)
    return static_cast<size_t>(ps.lds_a + ps.lds_p + ps.lds_b + ps.max_recs) * 4;
  return static_cast<size_t>(ps.lds_a + ps.lds_b + 2 * kLdsSlack) * 4;  // two level buffers
}

View view(const Plan &p, Buf b, const void *in, void *out, void *ws, int batch, bool adjoint,
          const RaggedBatch *rb) {
  const int64_t nt = p.nt;
  const int64_t plane_b = p.ws_rows * (rb ? rb->sum_ntp : p.ntp);
  const int64_t nb = rb ? 1 : batch;
  const int64_t in_rows = adjoint ? p.tab.nd : p.tab.nf;
  const int64_t out_rows = adjoint ? p.tab.nf : p.tab.nd;
  switch (b) {
    case Buf::In: return {const_cast<void *>(in), nt, in_rows * nt};
    case Buf::Out: return {out, nt, out_rows * nt};
    case Buf::Ws0: return {ws, p.ntp, plane_b};
    case Buf::Ws1:
      return {static_cast<unsigned char *>(ws) + static_cast<size_t>(plane_b) * nb * 4, p.ntp, plane_b};
    case Buf::InPad:
      return {static_cast<unsigned char *>(ws) + round_up(2 * plane_b * nb * 4, 256), nt, p.tab.slots * nt};
  }
  return {nullptr, 0, 0};
}

int64_t buf_rows(const Plan &p, Buf b, bool adjoint) {
  switch (b) {
    case Buf::In: return adjoint ? p.tab.nd : p.tab.nf;
    case Buf::Out: return adjoint ? p.tab.nf : p.tab.nd;
    case Buf::InPad: return p.tab.slots;
    default: return p.ws_rows;
  }
}

constexpr int64_t kMaxGridY = 65535;

// Runs of 4 samples per lane in the forward gathers: at most 2 (their 2^k
// terms per run live in registers); the adjoint gather takes the plan's value.
// Runs of 4 samples per lane of a forward gather pass: the plan's (1 or 2);
// 1 for four-iteration passes, whose 16 terms of two runs each would not fit
// the register budget of a 1024-thread workgroup.
inline int forward_vecs(const Plan &p, const Pass &ps) {
  if (ps.l1 - ps.l0 >= 4) return 1;
  return p.gather_vecs < 2 ? p.gather_vecs : 2;
}

// Issues the launches of one step over time tiles of width `tile`. A uniform
// batch is one launch: ceil(nt / tile) tiles in grid y, beams in grid z. A
// ragged batch walks the flattened tile map of that width, at most 65535
// tiles per launch. `launch(ragged, grid_y, grid_z, map)` issues one launch
// and returns its status.
template <typename F>
hipError_t for_each_launch(const Plan &p, const RaggedBatch *rb, const Step &st, bool adjoint,
                           int tile, int batch, F &&launch) {
  if (rb == nullptr) {
    RaggedMap order{};
    // Consecutive steps run their beams and time tiles in opposite orders, so
    // a step starts on the part of its input plane that its predecessor wrote
    // last, which the GPU's last-level cache (256 MiB) may still hold: the
    // Nf=4096 step and the batch-16 differentiable step each gained 1.5%.
    const std::vector<Step> &steps = adjoint ? p.adj_steps : p.fwd_steps;
    order.reverse = static_cast<int32_t>((&st - steps.data()) & 1);
    const hipError_t e = launch(std::false_type{}, static_cast<unsigned>((p.nt + tile - 1) / tile),
                                static_cast<unsigned>(batch), order);
    return e != hipSuccess ? e : hipGetLastError();
  }
  const RaggedBatch::Map *m = nullptr;
  for (const RaggedBatch::Map &x : rb->maps)
    if (x.tile == tile) m = &x;
  if (m == nullptr) return hipErrorInvalidValue;
  RaggedMap rg{};
  rg.beam = rb->beam;
  rg.src_rows = static_cast<int32_t>(buf_rows(p, st.src, adjoint));
  rg.dst_rows = static_cast<int32_t>(buf_rows(p, st.dst, adjoint));
  rg.src_padded = st.src == Buf::Ws0 || st.src == Buf::Ws1;
  rg.dst_padded = st.dst == Buf::Ws0 || st.dst == Buf::Ws1;
  for (int64_t off = 0; off < m->count; off += kMaxGridY) {
    rg.tiles = m->tiles + off;
    hipError_t e = launch(std::true_type{}, static_cast<unsigned>(std::min(kMaxGridY, m->count - off)), 1u, rg);
    if (e == hipSuccess) e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename Tin, typename Tacc>
hipError_t run_forward_step(const Plan &p, const Step &st, const void *in, void *out, int batch,
                            void *ws, hipStream_t stream, const RaggedBatch *rb, const SearchTile *search) {
  const Tables &T = p.tab;
  const int64_t nt = p.nt;
  const View src = view(p, st.src, in, out, ws, batch, false, rb);
  const View dst = view(p, st.dst, in, out, ws, batch, false, rb);
  switch (st.kind) {
    case Step::PadIn: {
      const int64_t in_bytes = T.nf * nt * static_cast<int64_t>(sizeof(Tin));
      const int64_t out_bytes = T.slots * nt * static_cast<int64_t>(sizeof(Tin));
      if (rb == nullptr && in_bytes % 16 == 0 && (reinterpret_cast<uintptr_t>(src.ptr) & 15) == 0 &&
          (reinterpret_cast<uintptr_t>(dst.ptr) & 15) == 0) {
        const int64_t vecs = out_bytes / 16;
        const unsigned gx = static_cast<unsigned>(std::min<int64_t>((vecs + kThreads - 1) / kThreads, 4096));
        hipLaunchKernelGGL(pad_flat_kernel, dim3(gx, static_cast<unsigned>(batch)), dim3(kThreads), 0, stream,
                           static_cast<const uint4 *>(src.ptr), static_cast<uint4 *>(dst.ptr), in_bytes / 16, vecs);
        return hipGetLastError();
      }
    }
      return for_each_launch(p, rb, st, false, kTile, batch, [&](auto r, unsigned gy, unsigned gz, const RaggedMap &rg) {
        hipLaunchKernelGGL((pad_input_kernel<Tin, decltype(r)::value>), dim3(T.slots, gy, gz), dim3(kThreads), 0,
                           stream, static_cast<const Tin *>(src.ptr), static_cast<Tin *>(dst.ptr), T.nf, nt,
                           src.bstride, dst.bstride, rg);
        return hipSuccess;
      });
    case Step::Init:
      return for_each_launch(p, rb, st, false, kTile, batch, [&](auto r, unsigned gy, unsigned gz, const RaggedMap &rg) {
        hipLaunchKernelGGL((init_kernel<Tin, Tacc, decltype(r)::value>), dim3(T.slots, gy, gz), dim3(kThreads), 0, stream,
                           static_cast<const Tin *>(src.ptr), static_cast<Tacc *>(dst.ptr),
                           p.dev.leaf_off, p.dev.leaf_rows, p.dev.pre, nt, src.bstride, dst.stride, dst.bstride, rg);
        return hipSuccess;
      });
    case Step::Merge:
      return for_each_launch(p, rb, st, false, kTile, batch, [&](auto r, unsigned gy, unsigned gz, const RaggedMap &rg) {
        hipLaunchKernelGGL((merge_kernel<Tacc, decltype(r)::value>),
                           dim3(static_cast<unsigned>(T.total[st.index]), gy, gz), dim3(kThreads), 0, stream,
                           static_cast<const Tacc *>(src.ptr), static_cast<Tacc *>(dst.ptr),
                           p.dev.merge[st.index], nt, src.stride, src.bstride, dst.stride, dst.bstride, rg);
        return hipSuccess;
      });
    case Step::Fused: {
      const Pass &ps = p.fwd.passes[st.index];
      if (ps.kind == PassKind::Staged) {
        if (rb != nullptr) return hipErrorInvalidValue;
        StagedArgs a{};
        a.src = src.ptr;
        a.dst = dst.ptr;
        a.stage = p.dev_stage + ps.rec_offset;
        a.psums = p.dev_psums + ps.psum_offset;
        a.terms = p.dev_sterms + ps.term_offset;
        a.heads = p.dev_sheads + ps.head_offset;
        a.src_stride = src.stride;
        a.src_bstride = src.bstride;
        a.dst_stride = dst.stride;
        a.dst_bstride = dst.bstride;
        a.nt = static_cast<int32_t>(nt);
        a.nblocks = ps.nblocks;
        a.tile = ps.tile;
        a.ntiles = static_cast<int32_t>((nt + ps.tile - 1) / ps.tile);
        a.tiles_per_wg = std::max(1, std::min(a.ntiles, p.tiles_per_wg));
        a.lds_rec = ps.lds_a + ps.lds_p;
        a.lds_prec = a.lds_rec + ps.stage_ints;
        a.lds_term = ps.lds_a + ps.lds_p + ps.lds_b;
        const size_t lds = fused_lds_bytes(ps);
        const int nchunks = (a.ntiles + a.tiles_per_wg - 1) / a.tiles_per_wg;
        dim3 grid(static_cast<unsigned>(ps.nblocks * nchunks), 1, batch);
        const int k = ps.l1 - ps.l0;
#define FDMT_STAGED(FI, KK) hipLaunchKernelGGL((staged_pass_kernel<Tin, Tacc, FI, KK>), grid, dim3(kStagedThreads), lds, stream, a)
        if (ps.from_input) {
          switch (k) {
            case 1: FDMT_STAGED(true, 1); break;
            case 2: FDMT_STAGED(true, 2); break;
            case 3: FDMT_STAGED(true, 3); break;
            case 4: FDMT_STAGED(true, 4); break;
            default: return hipErrorInvalidValue;
          }
        } else {
          switch (k) {
            case 1: FDMT_STAGED(false, 1); break;
            case 2: FDMT_STAGED(false, 2); break;
            case 3: FDMT_STAGED(false, 3); break;
            case 4: FDMT_STAGED(false, 4); break;
            default: return hipErrorInvalidValue;
          }
        }
#undef FDMT_STAGED
        return hipGetLastError();
      }
      if (ps.gather && ps.from_input) {
        const int k = ps.l1 - ps.l0;
        if (k < 1 || k > 4) return hipErrorInvalidValue;
        const int rpw = forward_rows(p, ps);
        const int cv = forward_vecs(p, ps);
        const int tile = 256 * cv * (forward_threads(p, ps) / 64 / rpw);
        const unsigned gx = static_cast<unsigned>((ps.nblocks + rpw - 1) / rpw);
        const int32_t nt32 = static_cast<int32_t>(nt);
        const int4 *tm = p.dev_iterms + ps.term_offset;
        const Tin *sp = static_cast<const Tin *>(src.ptr);
        const bool narrow_out = p.narrow[st.index];
        const bool int_sums = p.int_sums[st.index];
        return for_each_launch(p, rb, st, false, tile, batch, [&](auto r, unsigned gy, unsigned gz, const RaggedMap &rg) {
          GatherLaunch g{dim3(gx, gy, gz), stream, rg, decltype(r)::value, k, cv, rpw};
          g.threads = forward_threads(p, ps);
          g.max_chain = ps.max_chain;
          if constexpr (std::is_same<Tin, uint8_t>::value) {
            if (narrow_out)  // exact integer sums below 2^16
              return launch_narrow_input_gather<uint16_t>(g, sp, static_cast<uint16_t *>(dst.ptr), tm, nt32,
                                                          src.bstride, dst.stride, dst.bstride, ps.nblocks);
            if (int_sums)
              return launch_narrow_input_gather<Tacc>(g, sp, static_cast<Tacc *>(dst.ptr), tm, nt32, src.bstride,
                                                      dst.stride, dst.bstride, ps.nblocks);
          }
          return launch_input_gather<Tin, Tacc, Tacc>(g, sp, static_cast<Tacc *>(dst.ptr), tm, nt32, src.bstride,
                                                      dst.stride, dst.bstride, ps.nblocks);
        });
      }
      if (ps.gather) {
        const int k = ps.l1 - ps.l0;
        if (k < 1 || k > 4) return hipErrorInvalidValue;
        // rows per workgroup (1, 2, 4, 8 or 16) and workgroup size; a pass
        // that runs the search may take its own
        const int rpw = search && search->rows ? search->rows : forward_rows(p, ps);
        const int threads = search && search->threads ? search->threads : forward_threads(p, ps);
        const int cv = forward_vecs(p, ps);  // runs of 4 samples per lane: 1 or 2
        const int tile = 256 * cv * (threads / 64 / rpw);
        const unsigned gx = static_cast<unsigned>((ps.nblocks + rpw - 1) / rpw);
        const int32_t nt32 = static_cast<int32_t>(nt);
        const int2 *tm = p.dev_terms + ps.term_offset;
        const bool narrow_in = st.index > 0 && p.narrow[st.index - 1];
        const bool narrow_out = p.narrow[st.index];
        return for_each_launch(p, rb, st, false, tile, batch, [&](auto r, unsigned gy, unsigned gz, const RaggedMap &rg) {
          GatherLaunch g{dim3(gx, gy, gz), stream, rg, decltype(r)::value, k, cv, rpw};
          g.threads = threads;
          g.streaming = st.dst == Buf::Out;
          if (search) g.search = *search;
          if (narrow_in) {  // uint16 plane in: exact integer sums
            const uint16_t *sp = static_cast<const uint16_t *>(src.ptr);
            // the integer-sum kernel (a lane's 8 samples are one 16-byte
            // load per term); a pass that runs the search takes the
            // 4-sample-run kernel, which has it
            if (narrow_out)
              return launch_narrow_gather<uint16_t>(g, sp, static_cast<uint16_t *>(dst.ptr), tm, nt32, src.stride,
                                                    src.bstride, dst.stride, dst.bstride, ps.nblocks);
            if (!search)
              return launch_narrow_gather<Tacc>(g, sp, static_cast<Tacc *>(dst.ptr), tm, nt32, src.stride,
                                                src.bstride, dst.stride, dst.bstride, ps.nblocks);
            return launch_gather<uint16_t, int32_t, Tacc>(g, sp, static_cast<Tacc *>(dst.ptr), tm, nt32, src.stride,
                                                          src.bstride, dst.stride, dst.bstride, ps.nblocks);
          }
          if (narrow_out) return hipErrorInvalidValue;  // narrow planes are made from narrow planes
          return launch_gather<Tacc, Tacc, Tacc>(g, static_cast<const Tacc *>(src.ptr), static_cast<Tacc *>(dst.ptr),
                                                 tm, nt32, src.stride, src.bstride, dst.stride, dst.bstride,
                                                 ps.nblocks);
        });
      }
      FusedArgs a{};
      a.src = src.ptr;
      a.dst = dst.ptr;
      a.recs = p.dev_recs + ps.rec_offset;
      a.heads = p.dev_heads + ps.head_offset;
      a.nt = static_cast<int32_t>(nt);
      a.src_stride = src.stride;
      a.src_bstride = src.bstride;
      a.dst_stride = dst.stride;
      a.dst_bstride = dst.bstride;
      a.k = ps.l1 - ps.l0;
      a.nblocks = ps.nblocks;
      a.tile = ps.tile;
      a.lds_a = ps.lds_a;
      a.lds_b = ps.lds_b;
      a.tiles_per_wg = p.rec_tiles;
      const size_t lds = fused_lds_bytes(ps);
      return for_each_launch(p, rb, st, false, ps.tile * p.rec_tiles, batch, [&](auto r, unsigned gy, unsigned gz, const RaggedMap &rg) {
        constexpr bool R = decltype(r)::value;
        const dim3 grid(static_cast<unsigned>(a.nblocks), gy, gz);
        if (ps.from_input)
          hipLaunchKernelGGL((fused_pass_kernel<Tin, Tacc, true, R>), grid, dim3(kFusedThreads), lds, stream, a, rg);
        else
          hipLaunchKernelGGL((fused_pass_kernel<Tin, Tacc, false, R>), grid, dim3(kFusedThreads), lds, stream, a, rg);
        return hipSuccess;
      });
    }
    default: return hipErrorInvalidValue;
  }
}

template <typename Tacc>
hipError_t run_adjoint_step(const Plan &p, const Step &st, const void *in, void *out, int batch,
                            void *ws, hipStream_t stream, const RaggedBatch *rb) {
  const Tables &T = p.tab;
  const int64_t nt = p.nt;
  const View src = view(p, st.src, in, out, ws, batch, true, rb);
  const View dst = view(p, st.dst, in, out, ws, batch, true, rb);
  switch (st.kind) {
    case Step::MergeAdj: {
      const int l = st.index;
      return for_each_launch(p, rb, st, true, kTile, batch, [&](auto r, unsigned gy, unsigned gz, const RaggedMap &rg) {
        hipLaunchKernelGGL((merge_adjoint_kernel<Tacc, decltype(r)::value>),
                           dim3(static_cast<unsigned>(T.total[l - 1]), gy, gz), dim3(kThreads), 0, stream,
                           static_cast<const Tacc *>(src.ptr), static_cast<Tacc *>(dst.ptr),
                           p.dev.adj[l], p.dev.merge[l], nt, src.stride, src.bstride, dst.stride,
                           dst.bstride, rg);
        return hipSuccess;
      });
    }
    case Step::AdjGather: {
      const AdjPass &ps = p.adj.passes[st.index];
      if (ps.depth < 1 || ps.depth > 5) return hipErrorInvalidValue;
      const int rpw = adjoint_rows(p, st.index);
      const int cv = p.gather_vecs;
      const int threads = adjoint_threads(p, st.index);
      const int tile = adjoint_wave_span(cv, ps.lagged) * (threads / 64 / rpw);
      const unsigned gx = static_cast<unsigned>((ps.nrows + rpw - 1) / rpw);
      const int4 *lv = p.dev_adj_leaves + ps.leaf_offset;
      const int32_t *sr = p.dev_adj_starts + ps.start_offset;
      const int32_t *od = p.dev_adj_order + ps.order_offset;
      const Tacc *sp = static_cast<const Tacc *>(src.ptr);
      Tacc *dp = static_cast<Tacc *>(dst.ptr);
      const int32_t nt32 = static_cast<int32_t>(nt);
      return for_each_launch(p, rb, st, true, tile, batch, [&](auto r, unsigned gy, unsigned gz, const RaggedMap &rg) {
        GatherLaunch g{dim3(gx, gy, gz), stream, rg, decltype(r)::value, ps.depth, cv, rpw, ps.lagged,
                       st.index < 32 ? static_cast<int>((p.adjoint_tile_major >> st.index) & 1u) : 0,
                       threads};
        // the tile-major order numbers the workgroups in 32 bits
        if (static_cast<uint64_t>(gx) * gy >= (1ull << 31)) g.tiles_fastest = 0;
        g.streaming = ps.to_input;
        return launch_adjoint_gather<Tacc>(g, sp, dp, lv, sr, od, nt32, ps.max_shift, src.stride, src.bstride,
                                           dst.stride, dst.bstride, ps.nrows);
      });
    }
    case Step::InitAdj:
      return for_each_launch(p, rb, st, true, kTile, batch, [&](auto r, unsigned gy, unsigned gz, const RaggedMap &rg) {
        hipLaunchKernelGGL((init_adjoint_kernel<Tacc, decltype(r)::value>), dim3(T.nf, gy, gz), dim3(kThreads), 0,
                           stream, static_cast<const Tacc *>(src.ptr), static_cast<Tacc *>(dst.ptr),
                           p.dev.leaf_off, p.dev.leaf_rows, p.dev.pre, nt, src.stride, src.bstride, dst.bstride, rg);
        return hipSuccess;
      });
    default: return hipErrorInvalidValue;
  }
}

} // namespace

void plan_steps(Plan &p) {
  const Tables &T = p.tab;
  const int L = T.levels;
  p.fwd_steps.clear();
  p.adj_steps.clear();
  p.ws_rows = 0;
  auto ws = [](int i) { return (i & 1) ? Buf::Ws1 : Buf::Ws0; };
  // Nf not a power of two: the forward reads a copy of the input with a zero
  // row for every channel position past Nf
  const Buf fin = p.pad_input ? Buf::InPad : Buf::In;
  if (p.pad_input) p.fwd_steps.push_back({Step::PadIn, 0, Buf::In, Buf::InPad});
  if (L == 0) {
    p.fwd_steps.push_back({Step::Init, 0, fin, Buf::Out});
  } else if (p.fwd.passes.empty()) {
    p.fwd_steps.push_back({Step::Init, 0, fin, Buf::Ws0});
    for (int l = 1; l <= L; ++l)
      p.fwd_steps.push_back({Step::Merge, l, ws(l - 1), l == L ? Buf::Out : ws(l)});
    for (int l = 0; l < L; ++l) p.ws_rows = std::max<int64_t>(p.ws_rows, T.total[l]);
  } else {
    const int n = static_cast<int>(p.fwd.passes.size());
    // With a separate initialisation, plane 0 occupies workspace 0 and pass i
    // reads ws(i) and writes ws(i + 1).
    const int sh = p.fwd.init_separate ? 1 : 0;
    if (sh) {
      p.fwd_steps.push_back({Step::Init, 0, fin, Buf::Ws0});
      p.ws_rows = std::max<int64_t>(p.ws_rows, T.total[0]);
    }
    for (int i = 0; i < n; ++i) {
      const Pass &ps = p.fwd.passes[i];
      const Buf src = (i == 0 && !sh) ? fin : ws(i - 1 + sh);
      p.fwd_steps.push_back({Step::Fused, i, src, i == n - 1 ? Buf::Out : ws(i + sh)});
      if (i < n - 1) p.ws_rows = std::max<int64_t>(p.ws_rows, T.total[ps.l1]);
    }
  }
  // Adjoint: fused gathers (or, unfused, one gather per iteration from the
  // output back to plane 0, then the transpose of the initialisation).
  if (L == 0) {
    p.adj_steps.push_back({Step::InitAdj, 0, Buf::In, Buf::Out});
  } else if (!p.adj.passes.empty()) {
    const int n = static_cast<int>(p.adj.passes.size());
    const bool sep = p.adj.init_separate;
    for (int i = 0; i < n; ++i) {
      const AdjPass &ps = p.adj.passes[i];
      const bool last = i == n - 1 && !sep;
      p.adj_steps.push_back({Step::AdjGather, i, i == 0 ? Buf::In : ws(i - 1), last ? Buf::Out : ws(i)});
      if (!last) p.ws_rows = std::max<int64_t>(p.ws_rows, T.total[ps.l_lo]);
    }
    if (sep) p.adj_steps.push_back({Step::InitAdj, 0, ws(n - 1), Buf::Out});
  } else {
    for (int l = L; l >= 1; --l)
      p.adj_steps.push_back({Step::MergeAdj, l, l == L ? Buf::In : ws(l), ws(l - 1)});
    p.adj_steps.push_back({Step::InitAdj, 0, ws(0), Buf::Out});
    for (int l = 0; l < L; ++l) p.ws_rows = std::max<int64_t>(p.ws_rows, T.total[l]);
  }
}

static int64_t in_elem_bytes(const Plan &p) {
  return p.in_dtype == FDMT_U8 ? 1 : (p.in_dtype == FDMT_F16 ? 2 : 4);
}

size_t workspace_bytes(const Plan &p, int batch) {
  size_t b = static_cast<size_t>(2) * batch * p.ws_rows * p.ntp * 4;
  if (p.pad_input) b = round_up(b, 256) + static_cast<size_t>(batch) * p.tab.slots * p.nt * in_elem_bytes(p);
  return b;
}

size_t ragged_workspace_bytes(const Plan &p, const RaggedBatch &rb) {
  size_t b = static_cast<size_t>(2) * p.ws_rows * rb.sum_ntp * 4;
  if (p.pad_input) b = round_up(b, 256) + static_cast<size_t>(p.tab.slots) * rb.sum_nt * in_elem_bytes(p);
  return b;
}

template <typename Tin, typename Tacc, bool FI>
hipError_t set_staged_lds_k(int lds) {
  const void *fns[] = {reinterpret_cast<const void *>(&staged_pass_kernel<Tin, Tacc, FI, 1>),
                       reinterpret_cast<const void *>(&staged_pass_kernel<Tin, Tacc, FI, 2>),
                       reinterpret_cast<const void *>(&staged_pass_kernel<Tin, Tacc, FI, 3>),
                       reinterpret_cast<const void *>(&staged_pass_kernel<Tin, Tacc, FI, 4>)};
  for (const void *f : fns) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, lds);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t set_staged_lds(int lds) {
  hipError_t e;
  if ((e = set_staged_lds_k<float, float, true>(lds)) != hipSuccess) return e;
  if ((e = set_staged_lds_k<_Float16, float, true>(lds)) != hipSuccess) return e;
  if ((e = set_staged_lds_k<uint8_t, float, true>(lds)) != hipSuccess) return e;
  if ((e = set_staged_lds_k<uint8_t, int32_t, true>(lds)) != hipSuccess) return e;
  if ((e = set_staged_lds_k<int32_t, int32_t, true>(lds)) != hipSuccess) return e;
  if ((e = set_staged_lds_k<float, float, false>(lds)) != hipSuccess) return e;
  if ((e = set_staged_lds_k<_Float16, float, false>(lds)) != hipSuccess) return e;
  if ((e = set_staged_lds_k<uint8_t, float, false>(lds)) != hipSuccess) return e;
  if ((e = set_staged_lds_k<uint8_t, int32_t, false>(lds)) != hipSuccess) return e;
  return set_staged_lds_k<int32_t, int32_t, false>(lds);
}

hipError_t prepare_kernels(const Plan &p) {
  size_t lds = 0;
  for (const Pass &ps : p.fwd.passes)
    if (!ps.gather) lds = std::max(lds, fused_lds_bytes(ps));
  if (lds <= 64 * 1024) return hipSuccess;
  const void *fns[] = {
#define FDMT_FUSED_ALL(R)                                                                   \
  reinterpret_cast<const void *>(&fused_pass_kernel<float, float, true, R>),                \
      reinterpret_cast<const void *>(&fused_pass_kernel<_Float16, float, true, R>),         \
      reinterpret_cast<const void *>(&fused_pass_kernel<uint8_t, float, true, R>),          \
      reinterpret_cast<const void *>(&fused_pass_kernel<uint8_t, int32_t, true, R>),        \
      reinterpret_cast<const void *>(&fused_pass_kernel<int32_t, int32_t, true, R>),        \
      reinterpret_cast<const void *>(&fused_pass_kernel<float, float, false, R>),           \
      reinterpret_cast<const void *>(&fused_pass_kernel<_Float16, float, false, R>),        \
      reinterpret_cast<const void *>(&fused_pass_kernel<uint8_t, float, false, R>),         \
      reinterpret_cast<const void *>(&fused_pass_kernel<uint8_t, int32_t, false, R>),       \
      reinterpret_cast<const void *>(&fused_pass_kernel<int32_t, int32_t, false, R>)
      FDMT_FUSED_ALL(false), FDMT_FUSED_ALL(true)};
#undef FDMT_FUSED_ALL
  for (const void *f : fns) {
    hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
    if (e != hipSuccess) return e;
  }
  return set_staged_lds(static_cast<int>(lds));
}

hipError_t run_step(const Plan &p, bool adjoint, int i, const void *in, void *out, int batch,
                    void *ws, hipStream_t stream, const RaggedBatch *rb, const SearchTile *search) {
  if (adjoint) {
    const Step &st = p.adj_steps[i];
    if (p.acc_dtype == FDMT_F32) return run_adjoint_step<float>(p, st, in, out, batch, ws, stream, rb);
    return run_adjoint_step<int32_t>(p, st, in, out, batch, ws, stream, rb);
  }
  const Step &st = p.fwd_steps[i];
  if (p.acc_dtype == FDMT_F32) {
    switch (p.in_dtype) {
      case FDMT_F32: return run_forward_step<float, float>(p, st, in, out, batch, ws, stream, rb, search);
      case FDMT_F16: return run_forward_step<_Float16, float>(p, st, in, out, batch, ws, stream, rb, search);
      case FDMT_U8: return run_forward_step<uint8_t, float>(p, st, in, out, batch, ws, stream, rb, search);
      default: return hipErrorInvalidValue;
    }
  }
  switch (p.in_dtype) {
    case FDMT_U8: return run_forward_step<uint8_t, int32_t>(p, st, in, out, batch, ws, stream, rb, search);
    case FDMT_I32: return run_forward_step<int32_t, int32_t>(p, st, in, out, batch, ws, stream, rb, search);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_init_f32(const Plan &p, const void *in, float *plane0, int64_t stride, hipStream_t stream) {
  const dim3 grid(static_cast<unsigned>(p.tab.slots), static_cast<unsigned>((p.nt + kTile - 1) / kTile), 1);
  const int64_t in_bstride = p.tab.nf * p.nt, out_bstride = p.tab.total[0] * stride;
  switch (p.in_dtype) {
    case FDMT_F32:
      hipLaunchKernelGGL((init_kernel<float, float, false>), grid, dim3(kThreads), 0, stream,
                         static_cast<const float *>(in), plane0, p.dev.leaf_off, p.dev.leaf_rows, p.dev.pre, p.nt,
                         in_bstride, stride, out_bstride, RaggedMap{});
      break;
    case FDMT_F16:
      hipLaunchKernelGGL((init_kernel<_Float16, float, false>), grid, dim3(kThreads), 0, stream,
                         static_cast<const _Float16 *>(in), plane0, p.dev.leaf_off, p.dev.leaf_rows, p.dev.pre, p.nt,
                         in_bstride, stride, out_bstride, RaggedMap{});
      break;
    case FDMT_U8:
      hipLaunchKernelGGL((init_kernel<uint8_t, float, false>), grid, dim3(kThreads), 0, stream,
                         static_cast<const uint8_t *>(in), plane0, p.dev.leaf_off, p.dev.leaf_rows, p.dev.pre, p.nt,
                         in_bstride, stride, out_bstride, RaggedMap{});
      break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_forward(const Plan &p, const void *in, void *out, int batch, void *ws,
                          hipStream_t stream, const RaggedBatch *rb) {
  for (size_t i = 0; i < p.fwd_steps.size(); ++i) {
    hipError_t e = run_step(p, false, static_cast<int>(i), in, out, batch, ws, stream, rb);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

// Geometry of the last forward pass when it runs the search: tiles of
// kBoxTile samples, p.search_rows (> 0) rows per workgroup.
static void search_geometry(const Plan &p, int &rows, int &threads) {
  const Pass &ps = p.fwd.passes[p.fwd_steps.back().index];
  const int col_waves = kBoxTile / (256 * forward_vecs(p, ps));
  rows = p.search_rows;
  threads = 64 * col_waves * rows;
}

bool search_fusable(const Plan &p, int max_log2) {
  if (p.search_rows == 0) return false;
  if (p.acc_dtype != FDMT_F32 || p.fwd_steps.empty() || max_log2 < 0 || max_log2 > kBoxMaxLog2) return false;
  const int last = static_cast<int>(p.fwd_steps.size()) - 1;
  const Step &st = p.fwd_steps[last];
  if (st.kind != Step::Fused) return false;
  const Pass &ps = p.fwd.passes[st.index];
  if (!ps.gather || ps.from_input) return false;
  int rows, threads;
  search_geometry(p, rows, threads);
  if (threads > kGatherThreads) return false;
  const size_t lds = static_cast<size_t>(rows) * ((1 << max_log2) - 1 + kBoxTile) * 4 + 8 +
                     static_cast<size_t>(threads / 64) * 24;
  return lds <= 64 * 1024;
}

hipError_t launch_forward_search(const Plan &p, const void *in, float *out, int batch, void *ws, BoxPartial *part,
                                 int max_log2, hipStream_t stream) {
  const int last = static_cast<int>(p.fwd_steps.size()) - 1;
  for (int i = 0; i < last; ++i) {
    hipError_t e = run_step(p, false, i, in, out, batch, ws, stream);
    if (e != hipSuccess) return e;
  }
  SearchTile st;
  st.part = part;
  st.max_log2 = max_log2;
  st.ntiles = static_cast<int32_t>((p.nt + kBoxTile - 1) / kBoxTile);
  search_geometry(p, st.rows, st.threads);
  hipError_t e = run_step(p, false, last, in, out, batch, ws, stream, nullptr, &st);
  if (e != hipSuccess) return e;
  return launch_boxcar_edges(out, batch, p.tab.nd, p.nt, max_log2, part, stream);
}

hipError_t launch_adjoint(const Plan &p, const void *gout, void *gin, int batch, void *ws,
                          hipStream_t stream, const RaggedBatch *rb) {
  for (size_t i = 0; i < p.adj_steps.size(); ++i) {
    hipError_t e = run_step(p, true, static_cast<int>(i), gout, gin, batch, ws, stream, rb);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

int adjoint_rows(const Plan &p, int pass) {
  const int rows = p.adjoint_rows ? p.adjoint_rows : p.gather_rows;
  return p.adj.passes[pass].to_input && p.adjoint_last_rows ? p.adjoint_last_rows : rows;
}

int forward_rows(const Plan &p, const Pass &ps) {
  return ps.from_input && p.first_rows ? p.first_rows : p.gather_rows;
}

int forward_threads(const Plan &p, const Pass &ps) {
  return ps.from_input && p.first_threads ? p.first_threads : p.gather_threads;
}

int adjoint_threads(const Plan &p, int pass) {
  return p.adj.passes[pass].to_input && p.adjoint_last_threads ? p.adjoint_last_threads : p.adjoint_threads;
}

int step_tile(const Plan &p, bool adjoint, int i) {
  const Step &st = adjoint ? p.adj_steps[i] : p.fwd_steps[i];
  switch (st.kind) {
    case Step::PadIn:
    case Step::Init:
    case Step::Merge:
    case Step::MergeAdj:
    case Step::InitAdj: return kTile;
    case Step::AdjGather:
      return adjoint_wave_span(p.gather_vecs, p.adj.passes[st.index].lagged) *
             (adjoint_threads(p, st.index) / 64 / adjoint_rows(p, st.index));
    case Step::Fused: {
      const Pass &ps = p.fwd.passes[st.index];
      if (ps.kind == PassKind::Staged) return 0;
      return ps.gather ? 256 * forward_vecs(p, ps) * (forward_threads(p, ps) / 64 / forward_rows(p, ps))
                       : ps.tile * p.rec_tiles;
    }
  }
  return 0;
}

} // namespace fdmt
