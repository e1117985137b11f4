// Boxcar search over FDMT output planes: for every row (trial delay) and
// width w = 2^j, the causal running sum b_w[t] = y[t] + ... + y[t - w + 1]
// (zero before the record), its largest value with the first time it occurs,
// and the mean and standard deviation of b_w over the record. A pulse
// profile shared by all frequencies commutes with the transform (Sec. 4.2,
// pulse profile), so one transform serves every width.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <mutex>

#include "fdmt_boxcar.h"

// Device scratch of the allocation-free boxcar search: the per-(row, tile,
// width) partials, for callers that cannot allocate (see
// boxcar_static_scratch). Each GPU the library runs on holds its own copy
// until the process ends. Host code must not pass this name to a kernel: on
// the host it stands for a host-side shadow, not the device address, which
// boxcar_static_scratch looks up per device.
static __device__ __align__(256) unsigned char scratch[fdmt::kBoxScratchBytes];

namespace fdmt {

namespace {

constexpr int kBoxThreads = 64;  // one wave: its LDS steps need no workgroup barrier to wait on other waves
constexpr int kBoxPerThread = kBoxTile / kBoxThreads;

// Peak order: larger value first, then earlier time.
__device__ __forceinline__ bool better(float v, int t, float bv, int bt) { return v > bv || (v == bv && t < bt); }

template <typename T>
__device__ __forceinline__ T xor_lane(T x, int mask) {
  return __shfl_xor(x, mask, 64);
}

// One workgroup (one wave): one row, one tile of kBoxTile samples plus the
// w_max - 1 samples before it. Width 2w is built in LDS from width w as
// b_2w[t] = b_w[t] + b_w[t - w], which sums each window in a fixed tree; each
// level's tile samples then add to the partial statistics of that width.
__global__ __launch_bounds__(kBoxThreads) void boxcar_tile_kernel(const float *__restrict__ plane,
                                                                  BoxPartial *__restrict__ part, int64_t nt,
                                                                  int32_t nd, int32_t ntiles, int32_t max_log2) {
  extern __shared__ float buf[];  // kBoxTile + 2^max_log2 - 1 samples
  const int tile = blockIdx.x, row = blockIdx.y, b = blockIdx.z;
  const int tid = threadIdx.x;
  const int halo = (1 << max_log2) - 1;
  const int64_t t0 = static_cast<int64_t>(tile) * kBoxTile;  // first sample of the tile
  const int64_t left = nt - t0;
  const int nvalid = left < kBoxTile ? static_cast<int>(left) : kBoxTile;
  const float *y = plane + (static_cast<int64_t>(b) * nd + row) * nt;
  // local index i holds time t0 - halo + i; every load is issued before the
  // first store to LDS
  {
    constexpr int kLoads = (kBoxTile + (1 << kBoxMaxLog2) - 1 + kBoxThreads - 1) / kBoxThreads;
    float v[kLoads];
#pragma unroll
    for (int k = 0; k < kLoads; ++k) {
      const int i = tid + k * kBoxThreads;
      const int64_t t = t0 - halo + i;
      v[k] = i < halo + nvalid && t >= 0 ? y[t] : 0.0f;
    }
#pragma unroll
    for (int k = 0; k < kLoads; ++k) {
      const int i = tid + k * kBoxThreads;
      if (i < halo + nvalid) buf[i] = v[k];
    }
  }
  __syncthreads();
  for (int j = 0; j <= max_log2; ++j) {
    if (j > 0) {
      // width 2^j from width w = 2^(j-1); valid from local index 2^j - 1 on,
      // which covers every index a later width or the statistics read
      // In place, from the top index down, kGroup * 64 indices at a time: a
      // group reads all its old values before writing, and every index it
      // reads lies at or below its own top, which later groups never write.
      constexpr int kGroup = 8;
      const int w = 1 << (j - 1);
      const int first = (1 << j) - 1;
      for (int top = halo + nvalid - 1; top >= first; top -= kGroup * kBoxThreads) {
        float nv[kGroup];
        const int base = top - tid;
        if (top - kGroup * kBoxThreads + 1 >= first) {  // the whole group lies at or above `first`
#pragma unroll
          for (int g = 0; g < kGroup; ++g) nv[g] = buf[base - g * kBoxThreads] + buf[base - g * kBoxThreads - w];
#pragma unroll
          for (int g = 0; g < kGroup; ++g) buf[base - g * kBoxThreads] = nv[g];
        } else {
#pragma unroll
          for (int g = 0; g < kGroup; ++g) {
            const int i = base - g * kBoxThreads;
            if (i >= first) nv[g] = buf[i] + buf[i - w];
          }
#pragma unroll
          for (int g = 0; g < kGroup; ++g) {
            const int i = base - g * kBoxThreads;
            if (i >= first) buf[i] = nv[g];
          }
        }
      }
      __syncthreads();
    }
    // A thread visits its samples in increasing time, so a strictly larger
    // value is the only way to move its peak: equal values keep the first.
    double s = 0.0, q = 0.0;
    float best = -__builtin_inff();
    int best_t = INT32_MAX;
    if (nvalid == kBoxTile) {
      // The thread's first sample opens its peak unless it is a NaN; after
      // that only a strictly larger value moves it.
      const float v0 = buf[halo + tid];
      s += static_cast<double>(v0);
      q += static_cast<double>(v0) * static_cast<double>(v0);
      if (v0 == v0) {
        best = v0;
        best_t = tid;
      }
      if (best_t != INT32_MAX) {
#pragma unroll
        for (int k = 1; k < kBoxPerThread; ++k) {
          const int i = tid + k * kBoxThreads;
          const float v = buf[halo + i];
          s += static_cast<double>(v);
          q += static_cast<double>(v) * static_cast<double>(v);
          if (v > best) {
            best = v;
            best_t = i;
          }
        }
      } else {
        for (int k = 1; k < kBoxPerThread; ++k) {
          const int i = tid + k * kBoxThreads;
          const float v = buf[halo + i];
          s += static_cast<double>(v);
          q += static_cast<double>(v) * static_cast<double>(v);
          if (v > best || (v == best && best_t == INT32_MAX)) {
            best = v;
            best_t = i;
          }
        }
      }
    } else {
#pragma unroll
      for (int k = 0; k < kBoxPerThread; ++k) {
        const int i = tid + k * kBoxThreads;
        if (i < nvalid) {
          const float v = buf[halo + i];
          s += static_cast<double>(v);
          q += static_cast<double>(v) * static_cast<double>(v);
          if (v > best || (v == best && best_t == INT32_MAX)) {
            best = v;
            best_t = i;
          }
        }
      }
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
      s += xor_lane(s, m);
      q += xor_lane(q, m);
      const float ov = xor_lane(best, m);
      const int ot = xor_lane(best_t, m);
      if (better(ov, ot, best, best_t)) {
        best = ov;
        best_t = ot;
      }
    }
    if (tid == 0) {
      BoxPartial &p = part[((static_cast<int64_t>(b) * (max_log2 + 1) + j) * nd + row) * ntiles + tile];
      p.sum = s;
      p.sumsq = q;
      p.peak = best;
      p.t = static_cast<int32_t>(t0) + best_t;
    }
  }
}

// Windows that straddle the start of tile k >= 1 (their first samples lie in
// tile k - 1), for a search whose tile partials cover only the windows
// inside each tile (the search fused into the last forward pass). One wave
// per (tile start, row, beam) loads the 2^max_log2 - 1 samples before the
// start and as many from it, builds the widths with the same doubling tree,
// and for width w folds b_w at t = start .. start + w - 2 into the tile's
// partial: its sums, and its peak when not smaller than the tile's (these
// times come first).
__global__ __launch_bounds__(kBoxThreads) void boxcar_edge_kernel(const float *__restrict__ plane,
                                                                  BoxPartial *__restrict__ part, int64_t nt,
                                                                  int32_t nd, int32_t ntiles, int32_t max_log2) {
  extern __shared__ float ebuf[];  // 2 * (2^max_log2 - 1) samples
  const int tile = blockIdx.x + 1, row = blockIdx.y, b = blockIdx.z;
  const int tid = threadIdx.x;
  const int halo = (1 << max_log2) - 1;
  const int64_t start = static_cast<int64_t>(tile) * kBoxTile;
  const int64_t left = nt - start;
  const int after = left < halo ? static_cast<int>(left) : halo;  // samples of the tile the edge windows end at
  const int n = halo + after;
  const float *y = plane + (static_cast<int64_t>(b) * nd + row) * nt;
  // local index i holds time start - halo + i (start - halo >= 0 since tile >= 1)
  for (int i = tid; i < n; i += kBoxThreads) ebuf[i] = y[start - halo + i];
  __syncthreads();
  for (int j = 0; j <= max_log2; ++j) {
    const int w = 1 << j;
    if (j > 0) {
      // width w from width w/2, in place from the top down: a group of 64
      // reads all its old values before writing, and reads only below its top
      const int hw = w >> 1;
      for (int top = n - 1; top >= hw; top -= kBoxThreads) {
        const int i = top - tid;
        float nv = 0.0f;
        if (i >= hw) nv = ebuf[i] + ebuf[i - hw];
        if (i >= hw) ebuf[i] = nv;
      }
      __syncthreads();
    }
    // times start .. start + min(w - 1, after) - 1: local index halo + u
    const int cnt = w - 1 < after ? w - 1 : after;
    double s = 0.0, q = 0.0;
    float best = -__builtin_inff();
    int best_t = INT32_MAX;
    for (int u = tid; u < cnt; u += kBoxThreads) {
      const float v = ebuf[halo + u];
      s += static_cast<double>(v);
      q += static_cast<double>(v) * static_cast<double>(v);
      if (v > best || (v == best && u < best_t)) {
        best = v;
        best_t = u;
      }
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
      s += xor_lane(s, m);
      q += xor_lane(q, m);
      const float ov = xor_lane(best, m);
      const int ot = xor_lane(best_t, m);
      if (better(ov, ot, best, best_t)) {
        best = ov;
        best_t = ot;
      }
    }
    if (tid == 0 && cnt > 0) {
      BoxPartial &p = part[((static_cast<int64_t>(b) * (max_log2 + 1) + j) * nd + row) * ntiles + tile];
      p.sum += s;
      p.sumsq += q;
      // an edge time precedes every time of the tile's own partial
      if (best_t != INT32_MAX && (best >= p.peak || p.t == INT32_MAX)) {
        p.peak = best;
        p.t = static_cast<int32_t>(start) + best_t;
      }
    }
    __syncthreads();
  }
}

// One thread per (beam, width, row): the tiles' partials in time order.
// mean_sd (optional) receives the float64 mean and standard deviation.
__global__ __launch_bounds__(256) void boxcar_combine_kernel(const BoxPartial *__restrict__ part,
                                                             fdmt_boxcar_t *__restrict__ out, int64_t nt,
                                                             int32_t ntiles, int64_t count,
                                                             double2 *__restrict__ mean_sd) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= count) return;
  const BoxPartial *p = part + k * ntiles;
  double s = 0.0, q = 0.0;
  float best = -__builtin_inff();
  int best_t = INT32_MAX;
  for (int i = 0; i < ntiles; ++i) {
    s += p[i].sum;
    q += p[i].sumsq;
    if (better(p[i].peak, p[i].t, best, best_t)) {
      best = p[i].peak;
      best_t = p[i].t;
    }
  }
  const double mean = s / static_cast<double>(nt);
  const double var = q / static_cast<double>(nt) - mean * mean;
  const double sd = var > 0.0 ? sqrt(var) : 0.0;
  fdmt_boxcar_t r;
  r.peak = best;
  r.t = best_t;
  r.mean = static_cast<float>(mean);
  r.stdev = static_cast<float>(sd);
  r.snr = sd > 0.0 ? static_cast<float>((static_cast<double>(best) - mean) / sd) : 0.0f;
  out[k] = r;
  if (mean_sd) mean_sd[k] = make_double2(mean, sd);
}

// One thread per (beam, width, row, tile): the tile's peak is a candidate
// when its S/N against the row's float64 statistics reaches the threshold.
__global__ __launch_bounds__(256) void boxcar_candidate_kernel(const BoxPartial *__restrict__ part,
                                                               const double2 *__restrict__ mean_sd, int32_t nd,
                                                               int32_t ntiles, int32_t max_log2, int64_t count,
                                                               float threshold, fdmt_candidate_t *__restrict__ cand,
                                                               int32_t cap, int32_t *__restrict__ found) {
  const int64_t k = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (k >= count) return;
  const BoxPartial p = part[k];
  if (p.t == INT32_MAX) return;  // a tile without a peak (every value NaN)
  const int64_t r = k / ntiles;  // (beam, width, row)
  const double2 ms = mean_sd[r];
  const double snr = ms.y > 0.0 ? (static_cast<double>(p.peak) - ms.x) / ms.y : 0.0;
  if (!(snr >= static_cast<double>(threshold))) return;
  const int32_t row = static_cast<int32_t>(r % nd);
  const int32_t j = static_cast<int32_t>((r / nd) % (max_log2 + 1));
  const int32_t b = static_cast<int32_t>(r / nd / (max_log2 + 1));
  const int32_t slot = atomicAdd(found, 1);
  if (slot < cap) {
    fdmt_candidate_t c;
    c.beam = b;
    c.dt = row;
    c.t = p.t;
    c.width_log2 = j;
    c.peak = p.peak;
    c.snr = static_cast<float>(snr);
    cand[slot] = c;
  }
}

__global__ void zero_count_kernel(int32_t *found) {
  if (threadIdx.x == 0) *found = 0;
}

} // namespace

size_t boxcar_workspace_bytes(int32_t batch, int32_t nd, int64_t nt, int32_t max_log2) {
  const int64_t ntiles = (nt + kBoxTile - 1) / kBoxTile;
  return static_cast<size_t>(batch) * (max_log2 + 1) * nd * ntiles * sizeof(BoxPartial);
}

hipError_t boxcar_static_scratch(int device, void **ptr) {
  // device addresses of `scratch`, looked up once per device with that device current
  static std::mutex lock;
  static void *addr[kMaxDevices] = {};
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> guard(lock);
  if (!addr[device]) {
    int current = -1;
    hipError_t e = hipGetDevice(&current);
    if (e != hipSuccess) return e;
    if (current != device) return hipErrorInvalidDevice;
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    addr[device] = p;
  }
  *ptr = addr[device];
  return hipSuccess;
}

hipError_t launch_boxcar_tiles(const float *plane, int32_t batch, int32_t nd, int64_t nt, int32_t max_log2,
                               BoxPartial *part, hipStream_t stream) {
  const int64_t ntiles = (nt + kBoxTile - 1) / kBoxTile;
  const size_t lds = (kBoxTile + (1 << max_log2) - 1) * sizeof(float);
  hipLaunchKernelGGL(boxcar_tile_kernel, dim3(static_cast<unsigned>(ntiles), nd, batch), dim3(kBoxThreads), lds,
                     stream, plane, part, nt, nd, static_cast<int32_t>(ntiles), max_log2);
  return hipGetLastError();
}

hipError_t launch_boxcar_edges(const float *plane, int32_t batch, int32_t nd, int64_t nt, int32_t max_log2,
                               BoxPartial *part, hipStream_t stream) {
  const int64_t ntiles = (nt + kBoxTile - 1) / kBoxTile;
  if (ntiles < 2 || max_log2 == 0) return hipSuccess;  // no window straddles a tile start
  const size_t lds = 2 * ((1 << max_log2) - 1) * sizeof(float);
  hipLaunchKernelGGL(boxcar_edge_kernel, dim3(static_cast<unsigned>(ntiles - 1), nd, batch), dim3(kBoxThreads),
                     lds, stream, plane, part, nt, nd, static_cast<int32_t>(ntiles), max_log2);
  return hipGetLastError();
}

hipError_t launch_boxcar_combine(const BoxPartial *part, int32_t batch, int32_t nd, int64_t nt, int32_t max_log2,
                                 fdmt_boxcar_t *out, double2 *mean_sd, hipStream_t stream) {
  const int64_t ntiles = (nt + kBoxTile - 1) / kBoxTile;
  const int64_t count = static_cast<int64_t>(batch) * (max_log2 + 1) * nd;
  hipLaunchKernelGGL(boxcar_combine_kernel, dim3(static_cast<unsigned>((count + 255) / 256)), dim3(256), 0, stream,
                     part, out, nt, static_cast<int32_t>(ntiles), count, mean_sd);
  return hipGetLastError();
}

hipError_t launch_boxcar_candidates(const BoxPartial *part, const double2 *mean_sd, int32_t batch, int32_t nd,
                                    int64_t nt, int32_t max_log2, float threshold, fdmt_candidate_t *cand,
                                    int32_t cap, int32_t *found, hipStream_t stream) {
  const int64_t ntiles = (nt + kBoxTile - 1) / kBoxTile;
  const int64_t count = static_cast<int64_t>(batch) * (max_log2 + 1) * nd * ntiles;
  hipLaunchKernelGGL(zero_count_kernel, dim3(1), dim3(64), 0, stream, found);
  hipLaunchKernelGGL(boxcar_candidate_kernel, dim3(static_cast<unsigned>((count + 255) / 256)), dim3(256), 0,
                     stream, part, mean_sd, nd, static_cast<int32_t>(ntiles), max_log2, count, threshold, cand, cap,
                     found);
  return hipGetLastError();
}

hipError_t launch_boxcar(const float *plane, int32_t batch, int32_t nd, int64_t nt, int32_t max_log2,
                         fdmt_boxcar_t *out, void *ws, hipStream_t stream) {
  BoxPartial *part = static_cast<BoxPartial *>(ws);
  hipError_t e = launch_boxcar_tiles(plane, batch, nd, nt, max_log2, part, stream);
  if (e != hipSuccess) return e;
  return launch_boxcar_combine(part, batch, nd, nt, max_log2, out, nullptr, stream);
}

} // namespace fdmt
