// Register-gather kernels of the forward transform: later iterations from a
// plane, and the first iterations straight from the input.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "fdmt_launch.h"

namespace fdmt {

namespace {

// ---------------------------------------------------------------------------
// Register gather over k fused iterations: walking the tables down from an
// output row of plane l1 gives 2^k terms (row of plane l0, accumulated shift
// sigma); the output is their sum, evaluated as the recursion evaluates it:
// sibling pairs first, then pairs of pairs, lower half before upper half.
// A term whose time t - sigma is negative is zero (the record starts at 0),
// and an upper half made only of such terms adds +0, so each element equals
// the per-iteration result exactly (the copy rule).
//
// Work split: a workgroup covers 1024 consecutive samples of one output row,
// 4 per lane; every term is one unaligned 16-byte load per lane, all issued
// before any add. Rows run fastest in the workgroup order so neighbouring
// rows - which share most of their terms - meet in one XCD's L2.
template <typename T>
__device__ __forceinline__ T xor_lane(T x, int mask) {
  return __shfl_xor(x, mask, 64);
}

// Peak order: larger value first, then earlier time.
__device__ __forceinline__ bool better_peak(float v, int t, float bv, int bt) {
  return v > bv || (v == bv && t < bt);
}

// Boxcar search over a workgroup's output tile, fused into the last forward
// pass (Sec. 4.2, pulse profile: one transform serves every width). Each row
// of the workgroup puts its tile of W = 256 * CV * col_waves samples into
// LDS after 2^m - 1 zeros, builds width 2w from width w as
// b_2w[i] = b_w[i] + b_w[i - w] (the doubling tree of the standalone search,
// so every value is the same sum of the same terms) and, per width, reduces
// the sum, sum of squares and first peak of b_w over the windows that lie
// inside the tile into its partial. A window that reaches back past the
// tile start is left to the edge kernel, except in the first tile, where
// the zeros are the record's zero history.
typedef float F4 __attribute__((ext_vector_type(4)));

template <int CV>
__device__ __forceinline__ void search_tile(const F4 (&out)[CV],
                                            const SearchTile &st, int wave, int lane, int col_waves,
                                            int rows_per_wg, int r, bool row_ok, int tile, int nt, int nrows,
                                            int beam) {
  extern __shared__ float sbuf[];
  struct Red {
    double s, q;
    float peak;
    int t;
  };
  constexpr int kPer = 4 * CV;  // tile samples per thread: W / (64 * col_waves)
  const int m = st.max_log2;
  const int halo = (1 << m) - 1;
  const int width = 256 * CV * col_waves;
  const int len = halo + width;
  const int rl = wave / col_waves;              // row within the workgroup
  const int rt = (wave % col_waves) * 64 + lane;  // thread within the row
  const int nthr = 64 * col_waves;
  float *rb = sbuf + rl * len;
  Red *red = reinterpret_cast<Red *>(sbuf + ((rows_per_wg * len + 1) & ~1));
  const int64_t start = static_cast<int64_t>(tile) * width;
  const int nvalid = nt - start < width ? static_cast<int>(nt - start) : width;
  for (int i = rt; i < halo; i += nthr) rb[i] = 0.0f;
  const int u0 = (wave % col_waves) * 256 * CV + 4 * lane;
#pragma unroll
  for (int c = 0; c < CV; ++c)
#pragma unroll
    for (int q = 0; q < 4; ++q) rb[halo + u0 + 256 * c + q] = out[c][q];
  __syncthreads();
  for (int j = 0; j <= m; ++j) {
    if (j > 0) {
      const int hw = 1 << (j - 1);
      float nv[kPer];
#pragma unroll
      for (int k = 0; k < kPer; ++k) {
        const int i = halo + rt + k * nthr;
        nv[k] = rb[i] + rb[i - hw];
      }
      __syncthreads();
#pragma unroll
      for (int k = 0; k < kPer; ++k) rb[halo + rt + k * nthr] = nv[k];
      __syncthreads();
    }
    const int lo = tile == 0 ? 0 : (1 << j) - 1;
    double s = 0.0, q = 0.0;
    float best = -__builtin_inff();
    int bt = INT32_MAX;
#pragma unroll
    for (int k = 0; k < kPer; ++k) {
      const int u = rt + k * nthr;  // increasing in k: equal values keep the first
      if (u >= lo && u < nvalid) {
        const float x = rb[halo + u];
        s += static_cast<double>(x);
        q += static_cast<double>(x) * static_cast<double>(x);
        if (x > best || (x == best && bt == INT32_MAX)) {
          best = x;
          bt = u;
        }
      }
    }
#pragma unroll
    for (int mk = 32; mk >= 1; mk >>= 1) {
      s += xor_lane(s, mk);
      q += xor_lane(q, mk);
      const float ov = xor_lane(best, mk);
      const int ot = xor_lane(bt, mk);
      if (better_peak(ov, ot, best, bt)) {
        best = ov;
        bt = ot;
      }
    }
    if (lane == 0) red[rl * col_waves + wave % col_waves] = Red{s, q, best, bt};
    __syncthreads();
    if (rt == 0 && row_ok) {
      Red a = red[rl * col_waves];
      for (int c = 1; c < col_waves; ++c) {
        const Red x = red[rl * col_waves + c];
        a.s += x.s;
        a.q += x.q;
        if (better_peak(x.peak, x.t, a.peak, a.t)) {
          a.peak = x.peak;
          a.t = x.t;
        }
      }
      const int b = beam;
      BoxPartial &p = st.part[((static_cast<int64_t>(b) * (m + 1) + j) * nrows + r) * st.ntiles + tile];
      p.sum = a.s;
      p.sumsq = a.q;
      p.peak = a.peak;
      p.t = a.t == INT32_MAX ? INT32_MAX : static_cast<int32_t>(start) + a.t;
    }
  }
}

// SEARCH (the last pass of a forward with the boxcar search, uniform
// batches, FP32 output): after storing its outputs, the workgroup runs the
// boxcar search over its tile of each of its rows in LDS (see search_tile).
// NT: the output is not read again by this call (the last pass), so its
// full-run stores are non-temporal; the search pass always writes the output.
template <typename Tsrc, typename Tacc, typename Tdst, int K, int CV, bool RAGGED, bool SEARCH = false,
          bool NT = SEARCH>
__global__ __launch_bounds__(kGatherThreads) void gather_pass_kernel(
    const Tsrc *__restrict__ src, Tdst *__restrict__ dst, const int2 *__restrict__ terms,
    int32_t nt_u, int64_t src_stride_u, int64_t src_bstride, int64_t dst_stride_u,
    int64_t dst_bstride, int32_t nrows, int32_t rows_per_wg, RaggedMap rg, SearchTile search) {
  typedef typename Vec4<Tacc>::type V;
  typedef typename Vec4<Tsrc>::type S4;
  typedef typename Vec4<Tdst>::type D4;
  constexpr int N = 1 << K;
  // A workgroup holds rows_per_wg consecutive output rows (the rows share
  // most terms, so repeats hit this CU's L1) over one tile of
  // 256 * CV * (blockDim.x / 64 / rows_per_wg) samples; a lane handles CV
  // runs of 4 samples, 256 apart.
  const int wave = uniform(threadIdx.x / 64), lane = threadIdx.x % 64;
  const WaveLayout wl = wave_layout(wave, rows_per_wg, nrows);
  const int col_waves = wl.col_waves;  // waves per row
  const int2 item = gather_item<RAGGED>(wl.groups, false);
  const int g = item.x;
  const int r = g * rows_per_wg + wl.row;
  // with the search every thread stays for its barriers: rows past the last
  // and samples past the record compute zeros and store nothing
  if (!SEARCH && r >= nrows) return;
  const bool row_ok = r < nrows;
  BeamSpan bs = beam_span<RAGGED>(rg, nt_u, src_stride_u, src_bstride, dst_stride_u, dst_bstride);
  if (!RAGGED) bs.tile = rg.reverse ? static_cast<int>(gridDim.y) - 1 - item.y : item.y;
  const int nt = bs.nt;
  const int64_t src_stride = bs.src_stride;
  const int tw = (bs.tile * col_waves + wl.col) * 256 * CV;  // first sample of the wave
  const int t = tw + lane * 4;
  if (!SEARCH && t >= nt) return;
  const Tsrc *base = src + bs.src_off;
  const int2 *tm = terms + static_cast<int64_t>(row_ok ? r : nrows - 1) * N;
  int2 e[N];
  int smax = 0;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    e[j] = tm[j];
    smax = e[j].y > smax ? e[j].y : smax;
  }
  V v[N][CV];
  if (std::is_same<Tsrc, uint16_t>::value && tw >= smax) {
    // uint16 planes (workspace rows, word-aligned, padded): a term's samples
    // start 2 bytes off a word exactly when its shift is odd, the same for
    // every lane, so each lane loads the three aligned words around its run
    // and shifts them into place. The words end at most 4 bytes past the run,
    // inside the padded row or the workspace that follows it.
    uint32_t w[N][CV][3];
    int mis[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const char *p = reinterpret_cast<const char *>(base + row_offset(e[j].x, src_stride) + (t - e[j].y));
      mis[j] = uniform(static_cast<int>(reinterpret_cast<uintptr_t>(p) & 3));
#pragma unroll
      for (int c = 0; c < CV; ++c) {
        if (t + 256 * c < nt) {
          const uint32_t *q = reinterpret_cast<const uint32_t *>(p + 512 * c - mis[j]);
          w[j][c][0] = q[0];
          w[j][c][1] = q[1];
          w[j][c][2] = q[2];
        } else {
          w[j][c][0] = w[j][c][1] = w[j][c][2] = 0;
        }
      }
    }
#pragma unroll
    for (int j = 0; j < N; ++j)
#pragma unroll
      for (int c = 0; c < CV; ++c) {
        const uint32_t lo = __builtin_amdgcn_alignbyte(w[j][c][1], w[j][c][0], mis[j]);
        const uint32_t hi = __builtin_amdgcn_alignbyte(w[j][c][2], w[j][c][1], mis[j]);
        v[j][c][0] = static_cast<Tacc>(lo & 0xffffu);
        v[j][c][1] = static_cast<Tacc>(lo >> 16);
        v[j][c][2] = static_cast<Tacc>(hi & 0xffffu);
        v[j][c][3] = static_cast<Tacc>(hi >> 16);
      }
  } else if (tw >= smax && tw + 256 * CV <= nt) {
    // every term and run inside the record for the whole wave: no lane
    // conditions, so no exec-mask branches around the loads
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const Tsrc *p = base + row_offset(e[j].x, src_stride) + (t - e[j].y);
#pragma unroll
      for (int c = 0; c < CV; ++c)
        v[j][c] = __builtin_convertvector(*reinterpret_cast<const S4 *>(p + 256 * c), V);
    }
  } else if (tw >= smax) {  // every term inside the record for the whole wave
#pragma unroll
    for (int j = 0; j < N; ++j)
#pragma unroll
      for (int c = 0; c < CV; ++c)
        v[j][c] = t + 256 * c < nt
                      ? __builtin_convertvector(
                            *reinterpret_cast<const S4 *>(base + row_offset(e[j].x, src_stride) + (t + 256 * c - e[j].y)), V)
                      : V(0);
  } else {
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const Tsrc *row = base + row_offset(e[j].x, src_stride);
#pragma unroll
      for (int c = 0; c < CV; ++c) {
        const int ts = t + 256 * c - e[j].y;
#pragma unroll
        for (int i = 0; i < 4; ++i)
          v[j][c][i] = ts + i >= 0 && t + 256 * c < nt ? static_cast<Tacc>(row[ts + i]) : Tacc(0);
      }
    }
  }
#pragma unroll
  for (int span = 1; span < N; span *= 2)
#pragma unroll
    for (int j = 0; j < N; j += 2 * span)
#pragma unroll
      for (int c = 0; c < CV; ++c) v[j][c] = v[j][c] + v[j + span][c];
  if (row_ok) {
#pragma unroll
    for (int c = 0; c < CV; ++c) {
      const int tc = t + 256 * c;
      Tdst *o = dst + bs.dst_off + r * bs.dst_stride + tc;
      if (tc + 4 <= nt) {
        if constexpr (NT)
          __builtin_nontemporal_store(__builtin_convertvector(v[0][c], D4), reinterpret_cast<D4 *>(o));
        else
          *reinterpret_cast<D4 *>(o) = __builtin_convertvector(v[0][c], D4);
      } else {
        for (int i = 0; i < 4 && tc + i < nt; ++i) o[i] = static_cast<Tdst>(v[0][c][i]);
      }
    }
  }
  if constexpr (SEARCH) {
    F4 outf[CV];  // the values just stored (FP32 output)
#pragma unroll
    for (int c = 0; c < CV; ++c) outf[c] = __builtin_convertvector(v[0][c], F4);
    search_tile<CV>(outf, search, wave, lane, col_waves, rows_per_wg, r, row_ok, bs.tile, nt, nrows, bs.beam);
  }
}

// ---------------------------------------------------------------------------
// Register gather straight from the input: the first k iterations and the
// Option-1 initialisation in one pass. An output row of plane k is the tree
// sum of its 2^k terms (InTerm), each term channel ch's partial sum
// I[t - shift] + I[t - shift - 1] + ... + I[t - shift - chain], added in that
// order, and the terms added as the recursion adds them. Every element
// therefore equals the level-by-level result bit for bit. Work split as in
// gather_pass_kernel; a lane loads 4 consecutive input samples per access.
template <typename T>
struct In4;
template <>
struct In4<float> {
  typedef float type __attribute__((ext_vector_type(4), aligned(4)));
};
template <>
struct In4<int32_t> {
  typedef int type __attribute__((ext_vector_type(4), aligned(4)));
};
template <>
struct In4<_Float16> {
  typedef _Float16 type __attribute__((ext_vector_type(4), aligned(2)));
};
template <>
struct In4<uint8_t> {
  typedef uint8_t type __attribute__((ext_vector_type(4), aligned(1)));
};

template <typename Tin, typename Tacc, typename Tdst, int K, int CV, bool RAGGED>
__global__ __launch_bounds__(kGatherThreads) void input_gather_kernel(
    const Tin *__restrict__ src, Tdst *__restrict__ dst, const int4 *__restrict__ terms,
    int32_t nt_u, int64_t src_bstride, int64_t dst_stride_u, int64_t dst_bstride, int32_t nrows,
    int32_t rows_per_wg, RaggedMap rg) {
  typedef typename Vec4<Tacc>::type V;
  typedef typename Vec4<Tdst>::type D4;
  typedef typename In4<Tin>::type I4;
  constexpr int N = 1 << K;
  const int wave = uniform(threadIdx.x / 64), lane = threadIdx.x % 64;
  const WaveLayout wl = wave_layout(wave, rows_per_wg, nrows);
  const int col_waves = wl.col_waves;
  const int2 item = gather_item<RAGGED>(wl.groups, false);
  const int g = item.x;
  const int r = g * rows_per_wg + wl.row;
  if (r >= nrows) return;
  BeamSpan bs = beam_span<RAGGED>(rg, nt_u, nt_u, src_bstride, dst_stride_u, dst_bstride);
  if (!RAGGED) bs.tile = rg.reverse ? static_cast<int>(gridDim.y) - 1 - item.y : item.y;
  const int nt = bs.nt;
  const int tw = (bs.tile * col_waves + wl.col) * 256 * CV;  // first sample of the wave
  const int t = tw + lane * 4;
  if (t >= nt) return;
  const Tin *base = src + bs.src_off;
  const int4 *tm = terms + static_cast<int64_t>(r) * N;
  int4 e[N];
  int reach = 0;    // furthest sample back any term reads
  int longest = 0;  // longest chain of any term
#pragma unroll
  for (int j = 0; j < N; ++j) {
    e[j] = tm[j];
    const int back = e[j].y + e[j].z;
    reach = back > reach ? back : reach;
    longest = e[j].z > longest ? e[j].z : longest;
  }
  V v[N][CV];
  if (std::is_same<Tin, uint8_t>::value && (reinterpret_cast<uintptr_t>(src) & 3) == 0 && tw >= reach &&
      tw + 256 * CV + 12 <= nt && longest <= 4) {
    // Bytes: the misalignment of a term's samples is the same for every lane
    // (t is a multiple of 4), so each lane loads the three aligned words from
    // just before its window and shifts them into place. They start at most 3
    // bytes before the window, never before the (word-aligned) buffer, and end
    // at most 11 bytes after its first sample, inside the row as 12 samples
    // follow the wave's last one. All loads are issued before any is used.
    uint32_t w[N][CV][3];
    int mis[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const uint8_t *p = reinterpret_cast<const uint8_t *>(base) + row_offset(e[j].x, nt) +
                         (t - e[j].y - e[j].z);
      mis[j] = uniform(static_cast<int>(reinterpret_cast<uintptr_t>(p) & 3));
#pragma unroll
      for (int c = 0; c < CV; ++c) {
        const uint32_t *q = reinterpret_cast<const uint32_t *>(p + 256 * c - mis[j]);
        w[j][c][0] = q[0];
        w[j][c][1] = q[1];
        w[j][c][2] = q[2];
      }
    }
#pragma unroll
    for (int j = 0; j < N; ++j) {
#pragma unroll
      for (int c = 0; c < CV; ++c) {
        // chain element i (sample t - shift - i) starts mis + chain - i bytes in
        auto take = [&](int o) {
          const uint32_t lo = o < 4 ? w[j][c][0] : w[j][c][1], hi = o < 4 ? w[j][c][1] : w[j][c][2];
          const uint32_t x = __builtin_amdgcn_alignbyte(hi, lo, o & 3);
          V r4;
          r4[0] = static_cast<Tacc>(x & 0xffu);
          r4[1] = static_cast<Tacc>((x >> 8) & 0xffu);
          r4[2] = static_cast<Tacc>((x >> 16) & 0xffu);
          r4[3] = static_cast<Tacc>(x >> 24);
          return r4;
        };
        const int d = e[j].z;
        V acc = take(mis[j] + d);
        for (int i = 1; i <= d; ++i) acc = acc + take(mis[j] + d - i);
        v[j][c] = acc;
      }
    }
  } else if (std::is_same<Tin, _Float16>::value && (reinterpret_cast<uintptr_t>(src) & 3) == 0 &&
             tw >= reach && tw + 256 * CV + 8 <= nt && longest <= 2) {
    // Halves: as for bytes, a term's misalignment (0 or 2 bytes) is the same
    // for every lane. Each lane loads the four aligned words that start at or
    // just before its earliest chain sample t - shift - chain (never before the
    // word-aligned buffer, as tw >= reach); they end at most 14 bytes after
    // it, inside the row as 8 samples follow the wave's last one.
    uint32_t w[N][CV][4];
    int mis[N];
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const char *p = reinterpret_cast<const char *>(base + row_offset(e[j].x, nt) +
                                                     (t - e[j].y - e[j].z));
      mis[j] = uniform(static_cast<int>(reinterpret_cast<uintptr_t>(p) & 3));
#pragma unroll
      for (int c = 0; c < CV; ++c) {
        typedef uint32_t W4 __attribute__((ext_vector_type(4), aligned(4)));
        const W4 q = *reinterpret_cast<const W4 *>(p + 512 * c - mis[j]);
        w[j][c][0] = q[0];
        w[j][c][1] = q[1];
        w[j][c][2] = q[2];
        w[j][c][3] = q[3];
      }
    }
#pragma unroll
    for (int j = 0; j < N; ++j) {
#pragma unroll
      for (int c = 0; c < CV; ++c) {
        // chain element i (sample t - shift - i) starts mis + 2 (chain - i) bytes in
        auto take = [&](int o) {
          const int k = o >> 2;
          const uint32_t lo = __builtin_amdgcn_alignbyte(k ? w[j][c][2] : w[j][c][1], k ? w[j][c][1] : w[j][c][0], o & 3);
          const uint32_t hi = __builtin_amdgcn_alignbyte(k ? w[j][c][3] : w[j][c][2], k ? w[j][c][2] : w[j][c][1], o & 3);
          V r4;
          r4[0] = static_cast<Tacc>(__builtin_bit_cast(_Float16, static_cast<uint16_t>(lo & 0xffffu)));
          r4[1] = static_cast<Tacc>(__builtin_bit_cast(_Float16, static_cast<uint16_t>(lo >> 16)));
          r4[2] = static_cast<Tacc>(__builtin_bit_cast(_Float16, static_cast<uint16_t>(hi & 0xffffu)));
          r4[3] = static_cast<Tacc>(__builtin_bit_cast(_Float16, static_cast<uint16_t>(hi >> 16)));
          return r4;
        };
        const int d = e[j].z;
        V acc = take(mis[j] + 2 * d);
        for (int i = 1; i <= d; ++i) acc = acc + take(mis[j] + 2 * (d - i));
        v[j][c] = acc;
      }
    }
  } else if (tw >= reach && tw + 256 * CV <= nt) {  // every access of the wave inside [0, nt)
#pragma unroll
    for (int j = 0; j < N; ++j) {
#pragma unroll
      for (int c = 0; c < CV; ++c) {
        const Tin *p = base + row_offset(e[j].x, nt) + (t + 256 * c - e[j].y);
        V acc = __builtin_convertvector(*reinterpret_cast<const I4 *>(p), V);
        for (int d = 1; d <= e[j].z; ++d) acc = acc + __builtin_convertvector(*reinterpret_cast<const I4 *>(p - d), V);
        v[j][c] = acc;
      }
    }
  } else {
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const Tin *p = base + row_offset(e[j].x, nt);
#pragma unroll
      for (int c = 0; c < CV; ++c) {
        const int ts = t + 256 * c - e[j].y;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          Tacc acc = (ts + i >= 0 && ts + i < nt) ? widen<Tacc>(p[ts + i]) : Tacc(0);
          for (int d = 1; d <= e[j].z; ++d)
            acc += (ts + i - d >= 0 && ts + i - d < nt) ? widen<Tacc>(p[ts + i - d]) : Tacc(0);
          v[j][c][i] = acc;
        }
      }
    }
  }
#pragma unroll
  for (int span = 1; span < N; span *= 2)
#pragma unroll
    for (int j = 0; j < N; j += 2 * span)
#pragma unroll
      for (int c = 0; c < CV; ++c) v[j][c] = v[j][c] + v[j + span][c];
#pragma unroll
  for (int c = 0; c < CV; ++c) {
    const int tc = t + 256 * c;
    Tdst *o = dst + bs.dst_off + r * bs.dst_stride + tc;
    if (tc + 4 <= nt) {
      *reinterpret_cast<D4 *>(o) = __builtin_convertvector(v[0][c], D4);
    } else {
      for (int i = 0; i < 4 && tc + i < nt; ++i) o[i] = static_cast<Tdst>(v[0][c][i]);
    }
  }
}

} // namespace

template <typename Tsrc, typename Tacc, typename Tdst>
hipError_t launch_gather(const GatherLaunch &g, const Tsrc *src, Tdst *dst, const int2 *terms, int32_t nt,
                         int64_t src_stride, int64_t src_bstride, int64_t dst_stride, int64_t dst_bstride,
                         int32_t nrows) {
  if (!gather_shape_ok(g)) return hipErrorInvalidValue;
  if (g.search.part) {
    // the last forward pass with the boxcar search: FP32 output, uniform batches
    if constexpr (std::is_same<Tdst, float>::value) {
      if (g.ragged) return hipErrorInvalidValue;
      const int col_waves = g.threads / 64 / g.rows_per_wg;
      const int len = (1 << g.search.max_log2) - 1 + 256 * g.vecs * col_waves;
      const size_t lds = ((g.rows_per_wg * len + 1) & ~1) * sizeof(float) +
                         static_cast<size_t>(g.rows_per_wg) * col_waves * 24;
#define FDMT_SEARCH(KK, CC)                                                                                   \
  hipLaunchKernelGGL((gather_pass_kernel<Tsrc, Tacc, Tdst, KK, CC, false, true>), g.grid, dim3(g.threads), lds, \
                     g.stream, src, dst, terms, nt, src_stride, src_bstride, dst_stride, dst_bstride, nrows,       \
                     g.rows_per_wg, g.rg, g.search)
#define FDMT_SEARCH_K(CC)                  \
  switch (g.depth) {                       \
    case 1: FDMT_SEARCH(1, CC); break;     \
    case 2: FDMT_SEARCH(2, CC); break;     \
    case 3: FDMT_SEARCH(3, CC); break;     \
    case 4: if (CC != 1) return hipErrorInvalidValue; FDMT_SEARCH(4, 1); break; \
    default: return hipErrorInvalidValue;  \
  }
      if (g.vecs == 2) { FDMT_SEARCH_K(2) } else { FDMT_SEARCH_K(1) }
#undef FDMT_SEARCH_K
#undef FDMT_SEARCH
      return hipGetLastError();
    } else {
      return hipErrorInvalidValue;
    }
  }
#define FDMT_GATHER_NT(KK, CC, RR, NN)                                                                      \
  hipLaunchKernelGGL((gather_pass_kernel<Tsrc, Tacc, Tdst, KK, CC, RR, false, NN>), g.grid, dim3(g.threads), 0, \
                     g.stream, src, dst, terms, nt, src_stride, src_bstride, dst_stride, dst_bstride, nrows,     \
                     g.rows_per_wg, g.rg, g.search)
#define FDMT_GATHER(KK, CC, RR)          \
  if (g.streaming) {                     \
    FDMT_GATHER_NT(KK, CC, RR, true);    \
  } else {                               \
    FDMT_GATHER_NT(KK, CC, RR, false);   \
  }
#define FDMT_GATHER_K(CC, RR)             \
  switch (g.depth) {                      \
    case 1: FDMT_GATHER(1, CC, RR); break; \
    case 2: FDMT_GATHER(2, CC, RR); break; \
    case 3: FDMT_GATHER(3, CC, RR); break; \
    case 4: if (CC != 1) return hipErrorInvalidValue; FDMT_GATHER(4, 1, RR); break; \
    default: return hipErrorInvalidValue; \
  }
  if (g.ragged) {
    if (g.vecs == 2) { FDMT_GATHER_K(2, true) } else { FDMT_GATHER_K(1, true) }
  } else {
    if (g.vecs == 2) { FDMT_GATHER_K(2, false) } else { FDMT_GATHER_K(1, false) }
  }
#undef FDMT_GATHER_K
#undef FDMT_GATHER
#undef FDMT_GATHER_NT
  return hipGetLastError();
}

template <typename Tin, typename Tacc, typename Tdst>
hipError_t launch_input_gather(const GatherLaunch &g, const Tin *src, Tdst *dst, const int4 *terms, int32_t nt,
                               int64_t src_bstride, int64_t dst_stride, int64_t dst_bstride, int32_t nrows) {
  if (!gather_shape_ok(g)) return hipErrorInvalidValue;
#define FDMT_IGATHER(KK, CC, RR)                                                                          \
  hipLaunchKernelGGL((input_gather_kernel<Tin, Tacc, Tdst, KK, CC, RR>), g.grid, dim3(g.threads), 0, \
                     g.stream, src, dst, terms, nt, src_bstride, dst_stride, dst_bstride, nrows,          \
                     g.rows_per_wg, g.rg)
#define FDMT_IGATHER_K(CC, RR)             \
  switch (g.depth) {                       \
    case 1: FDMT_IGATHER(1, CC, RR); break; \
    case 2: FDMT_IGATHER(2, CC, RR); break; \
    case 3: FDMT_IGATHER(3, CC, RR); break; \
    case 4: if (CC != 1) return hipErrorInvalidValue; FDMT_IGATHER(4, 1, RR); break; \
    default: return hipErrorInvalidValue;  \
  }
  if (g.ragged) {
    if (g.vecs == 2) { FDMT_IGATHER_K(2, true) } else { FDMT_IGATHER_K(1, true) }
  } else {
    if (g.vecs == 2) { FDMT_IGATHER_K(2, false) } else { FDMT_IGATHER_K(1, false) }
  }
#undef FDMT_IGATHER_K
#undef FDMT_IGATHER
  return hipGetLastError();
}

#define FDMT_G_INST(TS, TA, TD)                                                                             \
  template hipError_t launch_gather<TS, TA, TD>(const GatherLaunch &, const TS *, TD *, const int2 *, int32_t, \
                                                int64_t, int64_t, int64_t, int64_t, int32_t);
FDMT_G_INST(float, float, float)
FDMT_G_INST(int32_t, int32_t, int32_t)
FDMT_G_INST(uint16_t, int32_t, float)
FDMT_G_INST(uint16_t, int32_t, int32_t)
#undef FDMT_G_INST
#define FDMT_IG_INST(TI, TA, TD)                                                                           \
  template hipError_t launch_input_gather<TI, TA, TD>(const GatherLaunch &, const TI *, TD *, const int4 *, \
                                                      int32_t, int64_t, int64_t, int64_t, int32_t);
FDMT_IG_INST(float, float, float)
FDMT_IG_INST(_Float16, float, float)
FDMT_IG_INST(uint8_t, float, float)
FDMT_IG_INST(uint8_t, int32_t, int32_t)
FDMT_IG_INST(int32_t, int32_t, int32_t)
#undef FDMT_IG_INST

} // namespace fdmt
