// Register gathers over uint8 input or uint16 planes, with exact integer sums.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <type_traits>

#include "fdmt_launch.h"

namespace fdmt {

namespace {

// ---------------------------------------------------------------------------
// The same sums as gather_pass_kernel and input_gather_kernel (2^k terms per
// output, each a plane-l0 row at a shift, or an Option-1 chain of input
// samples), over data whose every partial sum is an integer below 2^24: then
// the sums are exact in any order and equal the tree-order FP32 or int32
// results bit for bit. They are added into int32 lanes as they arrive.
//
// Layout: a wave covers 256 * CV consecutive samples like the other gathers,
// but a lane owns S = 4 * CV consecutive samples, so a term is one wide load
// per lane: W aligned words that cover the lane's bytes whatever their
// misalignment, which is the same for every lane of a term (t is a multiple
// of 4). Bytes take 16 bytes for 8 samples (12 when no chain of the pass is
// longer than 1). uint16 take 20 bytes for 8 samples, of which a lane loads
// only its own 16 and takes the last word from the next lane: one 16-byte
// load per term, which cut the uint16 passes of the Nf=4096 step by 15-17%
// (taking the 8 bytes past the lane the same way for byte input made that
// pass 25% slower: its loads are not the limit).
template <bool FROM_INPUT, int CV>
struct NarrowShape {
  static constexpr int S = 4 * CV;  // samples per lane
  // words per term: bytes: misalignment (<= 3) + chain (<= 4) + S;
  // uint16: misalignment (0 or 2) + 2 S
  static constexpr int W = FROM_INPUT ? (3 + 4 + S + 3) / 4 : (2 + 2 * S + 3) / 4;
};

template <int W, int M>
__device__ __forceinline__ void load_words(uint32_t (&w)[M], const char *q) {
  static_assert(W <= M, "word buffer too small");
  if constexpr (W == 2) {
    typedef uint32_t W2 __attribute__((ext_vector_type(2), aligned(4)));
    const W2 x = *reinterpret_cast<const W2 *>(q);
    w[0] = x[0];
    w[1] = x[1];
  } else if constexpr (W == 3) {
    typedef uint32_t W3 __attribute__((ext_vector_type(3), aligned(4)));
    const W3 x = *reinterpret_cast<const W3 *>(q);
    w[0] = x[0];
    w[1] = x[1];
    w[2] = x[2];
  } else {
    typedef uint32_t W4 __attribute__((ext_vector_type(4), aligned(4)));
    const W4 x = *reinterpret_cast<const W4 *>(q);
    w[0] = x[0];
    w[1] = x[1];
    w[2] = x[2];
    w[3] = x[3];
    if constexpr (W == 5) w[4] = *reinterpret_cast<const uint32_t *>(q + 16);
  }
}

// Adds one term of the uint8 first pass into a lane's packed sums: samples
// 4 q4 and 4 q4 + 2 into pk[2 q4] (one per 16-bit half), 4 q4 + 1 and
// 4 q4 + 3 into pk[2 q4 + 1]. The term's words w start at byte b before the
// chain's earliest sample, and the chain has c + 1 elements, so element i of
// sample 4 q4 + e is byte 4 q4 + b + c - i + e: the even pair takes the byte
// pairs (u, u + 2) for u = b .. b + c of word pair (q4, q4 + 1), the odd pair
// those for u = b + 1 .. b + c + 1. That is c + 2 byte-pair extractions (one
// v_perm each) per group, the middle c shared. A pair stays inside its two
// words while b + c <= 4; otherwise the words are first realigned to byte b.
// SHORT (no chain of the pass longer than 1, so b + c <= 4 always) runs
// without branches: the middle extraction's selector is swapped for one that
// gives zeros when c = 0.
template <bool SHORT, int CV, int W>
__device__ __forceinline__ void add_byte_chain(uint32_t (&pk)[2 * CV], uint32_t (&w)[W], int b, int c) {
  static_assert(W == CV + 2, "a byte term spans CV + 2 words");
  // v_perm selector: byte u of {hi:lo} to the low half, byte u + 2 to the high
  // half, zero bytes (selector 0x0c) above each
  const auto sel = [](int u) { return 0x0c020c00u + static_cast<uint32_t>(u) * 0x10001u; };
  if constexpr (SHORT) {
    // sel(u + k) = sel(u) + k * 0x10001
    const uint32_t s_lo = sel(b);
    const uint32_t s_mid = c ? s_lo + 0x10001u : 0x0c0c0c0cu;
    const uint32_t s_hi = s_lo + static_cast<uint32_t>(c + 1) * 0x10001u;
#pragma unroll
    for (int q4 = 0; q4 < CV; ++q4) {
      const uint32_t lo = w[q4], hi = w[q4 + 1];
      const uint32_t mid = __builtin_amdgcn_perm(hi, lo, s_mid);
      pk[2 * q4] += mid + __builtin_amdgcn_perm(hi, lo, s_lo);
      pk[2 * q4 + 1] += mid + __builtin_amdgcn_perm(hi, lo, s_hi);
    }
  } else {
    if (b + c > 4) {
#pragma unroll
      for (int m = 0; m <= CV; ++m) w[m] = __builtin_amdgcn_alignbyte(w[m + 1], w[m], b);
      b = 0;
    }
#pragma unroll
    for (int q4 = 0; q4 < CV; ++q4) {
      const uint32_t lo = w[q4], hi = w[q4 + 1];
      uint32_t mid = 0;
      for (int u = b + 1; u <= b + c; ++u) mid += __builtin_amdgcn_perm(hi, lo, sel(u));
      pk[2 * q4] += mid + __builtin_amdgcn_perm(hi, lo, sel(b));
      pk[2 * q4 + 1] += mid + __builtin_amdgcn_perm(hi, lo, sel(b + c + 1));
    }
  }
}

template <typename T>
__device__ __forceinline__ T from_int(int32_t x) {
  return static_cast<T>(x);
}

// Stores a lane's S samples (t .. t+S-1 of one row), clipped at nt.
template <typename Tdst, int S>
__device__ __forceinline__ void store_lane(Tdst *o, const int32_t (&acc)[S], int t, int nt) {
  if (t + S <= nt) {
    if constexpr (sizeof(Tdst) == 2) {
      // 2 S bytes at an offset that is a multiple of 2 S: whole 16-, 8-byte words
      typedef uint16_t H __attribute__((ext_vector_type(S), aligned(4)));
      H h;
#pragma unroll
      for (int q = 0; q < S; ++q) h[q] = static_cast<uint16_t>(acc[q]);
      *reinterpret_cast<H *>(o) = h;
    } else {
      typedef typename Vec4<Tdst>::type D4;
#pragma unroll
      for (int g = 0; g < S / 4; ++g) {
        D4 d;
#pragma unroll
        for (int q = 0; q < 4; ++q) d[q] = from_int<Tdst>(acc[4 * g + q]);
        *reinterpret_cast<D4 *>(o + 4 * g) = d;
      }
    }
  } else {
#pragma unroll
    for (int q = 0; q < S; ++q)
      if (t + q < nt) o[q] = from_int<Tdst>(acc[q]);
  }
}

// SHORT: uint8 input into uint16 planes whose Option-1 chains are all at most
// 1 long (the host knows this per pass); a template parameter rather than a
// branch, as one kernel holding both byte-chain forms took 67 VGPRs against
// 40-43 for either alone.
template <bool FROM_INPUT, typename Tdst, int K, int CV, bool RAGGED, bool SHORT>
__global__ __launch_bounds__(kGatherThreads) void narrow_gather_kernel(
    const void *__restrict__ src_v, Tdst *__restrict__ dst, const void *__restrict__ terms_v, int32_t nt_u,
    int64_t src_stride_u, int64_t src_bstride, int64_t dst_stride_u, int64_t dst_bstride, int32_t nrows,
    int32_t rows_per_wg, RaggedMap rg) {
  typedef typename std::conditional<FROM_INPUT, uint8_t, uint16_t>::type Tsrc;
  static_assert(!SHORT || (FROM_INPUT && sizeof(Tdst) == 2), "short chains: uint8 input into uint16 planes");
  constexpr int N = 1 << K;
  constexpr int S = NarrowShape<FROM_INPUT, CV>::S;
  constexpr int W = NarrowShape<FROM_INPUT, CV>::W;
  const int wave = uniform(threadIdx.x / 64), lane = threadIdx.x % 64;
  const WaveLayout wl = wave_layout(wave, rows_per_wg, nrows);
  const int col_waves = wl.col_waves;
  const int2 item = gather_item<RAGGED>(wl.groups, false);
  const int g = item.x;
  const int r = g * rows_per_wg + wl.row;
  if (r >= nrows) return;
  // the input's rows are Nt samples apart; a plane's by its (padded) stride
  BeamSpan bs = beam_span<RAGGED>(rg, nt_u, FROM_INPUT ? nt_u : src_stride_u, src_bstride, dst_stride_u,
                                        dst_bstride);
  if (!RAGGED) bs.tile = rg.reverse ? static_cast<int>(gridDim.y) - 1 - item.y : item.y;
  const int nt = bs.nt;
  const int64_t src_stride = FROM_INPUT ? nt : bs.src_stride;
  const int tw = (bs.tile * col_waves + wl.col) * 256 * CV;  // first sample of the wave
  const int t = tw + lane * S;
  // Lanes past the record's end return early, except where the outputs pass
  // through LDS: there every lane stores 4 samples of another lane's range.
  constexpr bool kTranspose = sizeof(Tdst) == 4 && CV == 2;
  if (!kTranspose && t >= nt) return;
  const Tsrc *base = static_cast<const Tsrc *>(src_v) + bs.src_off;
  // terms: (row or channel, shift, chain)
  int row[N], shift[N], chain[N];
  int reach = 0, longest = 0;
#pragma unroll
  for (int j = 0; j < N; ++j) {
    if constexpr (FROM_INPUT) {
      const int4 e = static_cast<const int4 *>(terms_v)[static_cast<int64_t>(r) * N + j];
      row[j] = e.x;
      shift[j] = e.y;
      chain[j] = e.z;
    } else {
      const int2 e = static_cast<const int2 *>(terms_v)[static_cast<int64_t>(r) * N + j];
      row[j] = e.x;
      shift[j] = e.y;
      chain[j] = 0;
    }
    reach = shift[j] + chain[j] > reach ? shift[j] + chain[j] : reach;
    longest = chain[j] > longest ? chain[j] : longest;
  }
  int32_t acc[S];
#pragma unroll
  for (int q = 0; q < S; ++q) acc[q] = 0;
  // Whole-word path: no sample of the wave before 0 (tw >= reach), its words
  // inside the row (input: 8 samples of room after the wave's last; a plane
  // row may be over-read by up to 4 bytes, into its padding or the workspace
  // that follows, which is sized for 4-byte planes), a word-aligned buffer (a
  // beam's rows may start off a word: the words before them are the buffer's)
  // and chains of at most 4.
  const bool words = (reinterpret_cast<uintptr_t>(src_v) & 3) == 0 && tw >= reach &&
                     (FROM_INPUT ? tw + 256 * CV + 8 <= nt && longest <= 4 : tw + 256 * CV <= nt);
  if (words) {
    uint32_t w[N][W];
    int mis[N];
    if constexpr (FROM_INPUT) {
#pragma unroll
      for (int j = 0; j < N; ++j) {
        // the wave's first sample of the term, a wave-uniform address: its
        // misalignment is every lane's (lanes are S bytes apart) and comes
        // from scalar arithmetic, not a read back from a lane
        const Tsrc *pw = base + row_offset(row[j], src_stride) + (tw - shift[j] - chain[j]);
        mis[j] = static_cast<int>(reinterpret_cast<uintptr_t>(pw) & 3);
        const char *p = reinterpret_cast<const char *>(pw + lane * S);
        // a chain of at most 1 ends by byte 3 + 1 + S - 1 of the words: CV + 1 of them
        load_words<SHORT ? CV + 1 : W>(w[j], p - mis[j]);
      }
    } else {
      // uint16: the wave's lanes cover one contiguous run of words, S / 2 per
      // lane, so a lane loads only its own words; an odd-shifted term (2
      // bytes off) needs one word more, the next lane's first, taken across
      // lanes. The last lane's is the word just past the wave's run, at an
      // address the same for every lane: one scalar load, where a vector
      // load for that lane alone would take an address-unit slot per term.
      constexpr int H = S / 2;
      static_assert(W == H + 1, "uint16 terms span S / 2 + 1 words");
      uint32_t past[N];
#pragma unroll
      for (int j = 0; j < N; ++j) {
        const Tsrc *rp = base + row_offset(row[j], src_stride);
        const Tsrc *pw = rp + (tw - shift[j]);  // wave-uniform; lanes are 2 S bytes apart
        mis[j] = static_cast<int>(reinterpret_cast<uintptr_t>(pw) & 3);
        const char *p = reinterpret_cast<const char *>(pw + lane * S);
        load_words<H>(w[j], p - mis[j]);
        w[j][H] = 0;
        past[j] = 0;
        if (mis[j]) past[j] = scalar_word(reinterpret_cast<const char *>(rp + (tw + 64 * S - shift[j])) - mis[j]);
      }
      const int next_lane = ((lane + 1) & 63) << 2;  // ds_bpermute byte address of lane + 1
#pragma unroll
      for (int j = 0; j < N; ++j) {
        if (mis[j]) {
          const uint32_t next = static_cast<uint32_t>(__builtin_amdgcn_ds_bpermute(next_lane, static_cast<int>(w[j][0])));
          w[j][H] = lane == 63 ? past[j] : next;
        }
      }
    }
    if constexpr (sizeof(Tdst) == 2) {
      // uint16 output: the plan stores a plane as uint16 only when every
      // element is below 2^16, and every term is non-negative, so every
      // partial sum of a sample is below 2^16 too. Two samples then share a
      // 32-bit word (one in each half) and one add serves both, with no
      // carry between the halves: pk[m] holds the lane's samples 2m (low
      // half) and 2m + 1 (high half), which is their uint16 layout.
      uint32_t pk[S / 2];
#pragma unroll
      for (int m = 0; m < S / 2; ++m) pk[m] = 0;
      if constexpr (FROM_INPUT) {
#pragma unroll
        for (int j = 0; j < N; ++j) add_byte_chain<SHORT, CV>(pk, w[j], mis[j], chain[j]);
      } else {
#pragma unroll
        for (int j = 0; j < N; ++j)
#pragma unroll
          for (int m = 0; m < S / 2; ++m) pk[m] += __builtin_amdgcn_alignbyte(w[j][m + 1], w[j][m], mis[j]);
      }
      if constexpr (FROM_INPUT) {
        // (even, odd) word pairs to sample order: bytes 0-1 of the even word
        // and 0-1 of the odd word, then bytes 2-3 of each
#pragma unroll
        for (int q4 = 0; q4 < CV; ++q4) {
          const uint32_t ev = pk[2 * q4], od = pk[2 * q4 + 1];
          pk[2 * q4] = __builtin_amdgcn_perm(od, ev, 0x05040100u);
          pk[2 * q4 + 1] = __builtin_amdgcn_perm(od, ev, 0x07060302u);
        }
      }
      Tdst *o = dst + bs.dst_off + r * bs.dst_stride + t;
      if (t + S <= nt) {
        // 2 S bytes at an offset that is a multiple of 2 S
        typedef uint32_t P __attribute__((ext_vector_type(S / 2), aligned(4)));
        P v;
#pragma unroll
        for (int m = 0; m < S / 2; ++m) v[m] = pk[m];
        *reinterpret_cast<P *>(o) = v;
      } else {
#pragma unroll
        for (int q = 0; q < S; ++q)
          if (t + q < nt) o[q] = static_cast<Tdst>(q & 1 ? pk[q / 2] >> 16 : pk[q / 2] & 0xffffu);
      }
      return;
    } else {
#pragma unroll
      for (int j = 0; j < N; ++j) {
        if constexpr (FROM_INPUT) {
          // chain element i (sample t - shift - i) starts mis + chain - i bytes in
          for (int i = 0; i <= chain[j]; ++i) {
            const int o = mis[j] + chain[j] - i;
            const int k = o >> 2;
#pragma unroll
            for (int q4 = 0; q4 < CV; ++q4) {
              const uint32_t lo = k ? w[j][q4 + 1] : w[j][q4];
              const uint32_t hi = k ? w[j][q4 + 2] : w[j][q4 + 1];
              const uint32_t x = __builtin_amdgcn_alignbyte(hi, lo, o & 3);
#pragma unroll
              for (int q = 0; q < 4; ++q) acc[4 * q4 + q] += (x >> (8 * q)) & 0xffu;
            }
          }
        } else {
#pragma unroll
          for (int m = 0; m < S / 2; ++m) {
            const uint32_t x = __builtin_amdgcn_alignbyte(w[j][m + 1], w[j][m], mis[j]);
            acc[2 * m] += x & 0xffffu;
            acc[2 * m + 1] += x >> 16;
          }
        }
      }
    }
  } else {
    // row edges: every sample checked against [0, nt)
#pragma unroll
    for (int j = 0; j < N; ++j) {
      const Tsrc *rp = base + row_offset(row[j], src_stride);
      for (int i = 0; i <= chain[j]; ++i) {
#pragma unroll
        for (int q = 0; q < S; ++q) {
          const int ts = t + q - shift[j] - i;
          if (ts >= 0 && ts < nt) acc[q] += rp[ts];
        }
      }
    }
  }
  Tdst *orow = dst + bs.dst_off + r * bs.dst_stride;
  if constexpr (kTranspose) {
    // 4-byte outputs: a lane's 8 consecutive samples would be two 16-byte
    // stores that each cover every other 16 bytes of the wave's span. Pass
    // them through LDS so each store instruction writes 256 consecutive
    // samples (4 per lane, whole lines). One wave's LDS accesses are ordered,
    // so no barrier is needed.
    typedef Tdst T4 __attribute__((ext_vector_type(4)));
    __shared__ T4 xbuf[kGatherThreads / 64][128];
    T4 *xb = xbuf[wave];
    T4 lo, hi;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      lo[q] = from_int<Tdst>(acc[q]);
      hi[q] = from_int<Tdst>(acc[4 + q]);
    }
    xb[2 * lane] = lo;
    xb[2 * lane + 1] = hi;
#pragma unroll
    for (int run = 0; run < 2; ++run) {
      const T4 d = xb[64 * run + lane];
      const int tc = tw + 256 * run + 4 * lane;
      if (tc + 4 <= nt) {
        *reinterpret_cast<typename Vec4<Tdst>::type *>(orow + tc) = d;
      } else {
        for (int q = 0; q < 4 && tc + q < nt; ++q) orow[tc + q] = d[q];
      }
    }
  } else {
    store_lane<Tdst, S>(orow + t, acc, t, nt);
  }
}

template <bool FROM_INPUT, typename Tdst, bool SHORT = false>
hipError_t launch_narrow(const GatherLaunch &g, const void *src, Tdst *dst, const void *terms, int32_t nt,
                         int64_t src_stride, int64_t src_bstride, int64_t dst_stride, int64_t dst_bstride,
                         int32_t nrows) {
  if (!gather_shape_ok(g)) return hipErrorInvalidValue;
#define FDMT_NARROW(KK, CC, RR)                                                                                 \
  hipLaunchKernelGGL((narrow_gather_kernel<FROM_INPUT, Tdst, KK, CC, RR, SHORT>), g.grid, dim3(g.threads), 0, \
                     g.stream, src, dst, terms, nt, src_stride, src_bstride, dst_stride, dst_bstride, nrows,   \
                     g.rows_per_wg, g.rg)
#define FDMT_NARROW_K(CC, RR)              \
  switch (g.depth) {                       \
    case 1: FDMT_NARROW(1, CC, RR); break; \
    case 2: FDMT_NARROW(2, CC, RR); break; \
    case 3: FDMT_NARROW(3, CC, RR); break; \
    case 4: if (CC != 1) return hipErrorInvalidValue; FDMT_NARROW(4, 1, RR); break; \
    default: return hipErrorInvalidValue;  \
  }
  if (g.ragged) {
    if (g.vecs == 2) { FDMT_NARROW_K(2, true) } else { FDMT_NARROW_K(1, true) }
  } else {
    if (g.vecs == 2) { FDMT_NARROW_K(2, false) } else { FDMT_NARROW_K(1, false) }
  }
#undef FDMT_NARROW_K
#undef FDMT_NARROW
  return hipGetLastError();
}

} // namespace

template <typename Tdst>
hipError_t launch_narrow_input_gather(const GatherLaunch &g, const uint8_t *src, Tdst *dst, const int4 *terms,
                                      int32_t nt, int64_t src_bstride, int64_t dst_stride, int64_t dst_bstride,
                                      int32_t nrows) {
  if (g.vecs != 1 && g.vecs != 2) return hipErrorInvalidValue;
  if constexpr (sizeof(Tdst) == 2) {
    if (g.max_chain >= 0 && g.max_chain <= 1)
      return launch_narrow<true, Tdst, true>(g, src, dst, terms, nt, nt, src_bstride, dst_stride, dst_bstride, nrows);
  }
  return launch_narrow<true, Tdst>(g, src, dst, terms, nt, nt, src_bstride, dst_stride, dst_bstride, nrows);
}

template <typename Tdst>
hipError_t launch_narrow_gather(const GatherLaunch &g, const uint16_t *src, Tdst *dst, const int2 *terms,
                                int32_t nt, int64_t src_stride, int64_t src_bstride, int64_t dst_stride,
                                int64_t dst_bstride, int32_t nrows) {
  if (g.vecs != 1 && g.vecs != 2) return hipErrorInvalidValue;
  return launch_narrow<false, Tdst>(g, src, dst, terms, nt, src_stride, src_bstride, dst_stride, dst_bstride,
                                    nrows);
}

#define FDMT_NARROW_INST(T)                                                                                   \
  template hipError_t launch_narrow_input_gather<T>(const GatherLaunch &, const uint8_t *, T *, const int4 *, \
                                                    int32_t, int64_t, int64_t, int64_t, int32_t);
FDMT_NARROW_INST(uint16_t)
FDMT_NARROW_INST(int32_t)
FDMT_NARROW_INST(float)
#undef FDMT_NARROW_INST
#define FDMT_NARROW_INST(T)                                                                                   \
  template hipError_t launch_narrow_gather<T>(const GatherLaunch &, const uint16_t *, T *, const int2 *, int32_t, \
                                              int64_t, int64_t, int64_t, int64_t, int32_t);
FDMT_NARROW_INST(uint16_t)
FDMT_NARROW_INST(int32_t)
FDMT_NARROW_INST(float)
#undef FDMT_NARROW_INST

} // namespace fdmt
