// FDMT kernels for gfx950 (CDNA4): Option-1 initialisation, the iteration
// merges of Algorithm 1 and their transposes.
//
// Data layout: a plane holds every sub-band of one iteration, rows of a
// sub-band consecutive, sub-bands in frequency order, time contiguous, row
// stride `ntp` (padded to 64 samples) inside the workspace, `nt` in user
// buffers. The work is a gather-add along time: no contraction, so no MFMA;
// every kernel streams rows with coalesced loads (lane i reads sample base+i).
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fdmt_plan.h"

namespace fdmt {

namespace {

constexpr int kThreads = 256;
constexpr int kPerThread = 4;
constexpr int kTile = kThreads * kPerThread;  // samples per workgroup

template <typename Tacc, typename Tin>
__device__ __forceinline__ Tacc widen(Tin x) {
  return static_cast<Tacc>(x);
}
template <>
__device__ __forceinline__ float widen<float, _Float16>(_Float16 x) {
  return static_cast<float>(x);
}

// ---------------------------------------------------------------------------
// Option-1 initialisation (Sec. 3): row d of channel k holds
// sum_{i=0}^{d} I[k][t - i], zero before t = 0. Grid: (channel, time tile, beam).
template <typename Tin, typename Tacc>
__global__ __launch_bounds__(kThreads) void init_kernel(
    const Tin *__restrict__ in, Tacc *__restrict__ out, const int32_t *__restrict__ leaf_off,
    const int32_t *__restrict__ leaf_rows, int64_t nt, int64_t in_bstride, int64_t out_stride,
    int64_t out_bstride) {
  const int k = blockIdx.x;
  const int64_t b = blockIdx.z;
  const Tin *x = in + b * in_bstride + static_cast<int64_t>(k) * nt;
  Tacc *o = out + b * out_bstride + static_cast<int64_t>(leaf_off[k]) * out_stride;
  const int n = leaf_rows[k];
#pragma unroll
  for (int i = 0; i < kPerThread; ++i) {
    const int64_t t = static_cast<int64_t>(blockIdx.y) * kTile + i * kThreads + threadIdx.x;
    if (t >= nt) break;
    Tacc acc = 0;
    for (int d = 0; d < n; ++d) {
      if (t - d >= 0) acc += widen<Tacc>(x[t - d]);
      o[d * out_stride + t] = acc;
    }
  }
}

// One iteration: out[r][t] = prev[lo][t] + (t >= s ? prev[hi][t - s] : 0).
// Grid: (plane row, time tile, beam).
template <typename Tacc>
__global__ __launch_bounds__(kThreads) void merge_kernel(
    const Tacc *__restrict__ prev, Tacc *__restrict__ next, const int4 *__restrict__ rows,
    int64_t nt, int64_t prev_stride, int64_t prev_bstride, int64_t next_stride,
    int64_t next_bstride) {
  const int r = blockIdx.x;
  const int64_t b = blockIdx.z;
  const int4 e = rows[r];
  const Tacc *lo = prev + b * prev_bstride + static_cast<int64_t>(e.x) * prev_stride;
  const Tacc *hi = prev + b * prev_bstride + static_cast<int64_t>(e.y) * prev_stride;
  Tacc *o = next + b * next_bstride + static_cast<int64_t>(r) * next_stride;
  const int64_t s = e.z;
#pragma unroll
  for (int i = 0; i < kPerThread; ++i) {
    const int64_t t = static_cast<int64_t>(blockIdx.y) * kTile + i * kThreads + threadIdx.x;
    if (t >= nt) break;
    Tacc v = lo[t];
    if (t >= s) v += hi[t - s];
    o[t] = v;
  }
}

// Transpose of one iteration: child row r of plane l-1 gathers the `count`
// consecutive parent rows that read it, in ascending dt, shifted back by the
// parent's s if it is their upper half. Grid: (child row, time tile, beam).
template <typename Tacc>
__global__ __launch_bounds__(kThreads) void merge_adjoint_kernel(
    const Tacc *__restrict__ parent, Tacc *__restrict__ child, const int4 *__restrict__ adj,
    const int4 *__restrict__ fwd, int64_t nt, int64_t parent_stride, int64_t parent_bstride,
    int64_t child_stride, int64_t child_bstride) {
  const int r = blockIdx.x;
  const int64_t b = blockIdx.z;
  const int4 a = adj[r];
  const Tacc *g = parent + b * parent_bstride;
  Tacc *o = child + b * child_bstride + static_cast<int64_t>(r) * child_stride;
#pragma unroll
  for (int i = 0; i < kPerThread; ++i) {
    const int64_t t = static_cast<int64_t>(blockIdx.y) * kTile + i * kThreads + threadIdx.x;
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
template <typename Tacc>
__global__ __launch_bounds__(kThreads) void init_adjoint_kernel(
    const Tacc *__restrict__ plane, Tacc *__restrict__ out, const int32_t *__restrict__ leaf_off,
    const int32_t *__restrict__ leaf_rows, int64_t nt, int64_t plane_stride,
    int64_t plane_bstride, int64_t out_bstride) {
  const int k = blockIdx.x;
  const int64_t b = blockIdx.z;
  const Tacc *g = plane + b * plane_bstride + static_cast<int64_t>(leaf_off[k]) * plane_stride;
  Tacc *o = out + b * out_bstride + static_cast<int64_t>(k) * nt;
  const int n = leaf_rows[k];
#pragma unroll
  for (int i = 0; i < kPerThread; ++i) {
    const int64_t t = static_cast<int64_t>(blockIdx.y) * kTile + i * kThreads + threadIdx.x;
    if (t >= nt) break;
    Tacc acc = 0;
    for (int d = 0; d < n; ++d)
      for (int j = 0; j <= d; ++j)
        if (t + j < nt) acc += g[d * plane_stride + t + j];
    o[t] = acc;
  }
}

template <typename Tin, typename Tacc>
hipError_t forward_unfused(const Plan &p, const Tin *in, Tacc *out, int batch, void *ws,
                           hipStream_t stream) {
  const Tables &T = p.tab;
  const int L = T.levels;
  const int64_t nt = p.nt;
  const unsigned tiles = static_cast<unsigned>((nt + kTile - 1) / kTile);
  const int64_t plane_b = p.rmax * p.ntp;
  Tacc *buf[2] = {static_cast<Tacc *>(ws), static_cast<Tacc *>(ws) + plane_b * batch};

  // Initialisation writes plane 0, or the output directly when Nf = 1.
  {
    Tacc *dst = L == 0 ? out : buf[0];
    const int64_t stride = L == 0 ? nt : p.ntp;
    const int64_t bstride = L == 0 ? static_cast<int64_t>(T.nd) * nt : plane_b;
    dim3 grid(T.nf, tiles, batch);
    hipLaunchKernelGGL((init_kernel<Tin, Tacc>), grid, dim3(kThreads), 0, stream, in, dst,
                       p.dev.leaf_off, p.dev.leaf_rows, nt, static_cast<int64_t>(T.nf) * nt,
                       stride, bstride);
  }
  for (int l = 1; l <= L; ++l) {
    const Tacc *src = buf[(l - 1) & 1];
    const bool last = l == L;
    Tacc *dst = last ? out : buf[l & 1];
    const int64_t stride = last ? nt : p.ntp;
    const int64_t bstride = last ? static_cast<int64_t>(T.nd) * nt : plane_b;
    dim3 grid(static_cast<unsigned>(T.total[l]), tiles, batch);
    hipLaunchKernelGGL((merge_kernel<Tacc>), grid, dim3(kThreads), 0, stream, src, dst,
                       p.dev.merge[l], nt, p.ntp, plane_b, stride, bstride);
  }
  return hipGetLastError();
}

template <typename Tacc>
hipError_t adjoint_unfused(const Plan &p, const Tacc *gout, Tacc *gin, int batch, void *ws,
                           hipStream_t stream) {
  const Tables &T = p.tab;
  const int L = T.levels;
  const int64_t nt = p.nt;
  const unsigned tiles = static_cast<unsigned>((nt + kTile - 1) / kTile);
  const int64_t plane_b = p.rmax * p.ntp;
  Tacc *buf[2] = {static_cast<Tacc *>(ws), static_cast<Tacc *>(ws) + plane_b * batch};

  const Tacc *src = gout;
  int64_t src_stride = nt, src_bstride = static_cast<int64_t>(T.nd) * nt;
  for (int l = L; l >= 1; --l) {
    Tacc *dst = buf[l & 1];
    dim3 grid(static_cast<unsigned>(T.total[l - 1]), tiles, batch);
    hipLaunchKernelGGL((merge_adjoint_kernel<Tacc>), grid, dim3(kThreads), 0, stream, src, dst,
                       p.dev.adj[l], p.dev.merge[l], nt, src_stride, src_bstride, p.ntp, plane_b);
    src = dst;
    src_stride = p.ntp;
    src_bstride = plane_b;
  }
  dim3 grid(T.nf, tiles, batch);
  hipLaunchKernelGGL((init_adjoint_kernel<Tacc>), grid, dim3(kThreads), 0, stream, src, gin,
                     p.dev.leaf_off, p.dev.leaf_rows, nt, src_stride, src_bstride,
                     static_cast<int64_t>(T.nf) * nt);
  return hipGetLastError();
}

} // namespace

size_t workspace_bytes(const Plan &p, int batch) {
  if (p.tab.levels == 0) return 0;
  return static_cast<size_t>(2) * batch * p.rmax * p.ntp * 4;
}

hipError_t launch_forward(const Plan &p, const void *in, void *out, int batch, void *ws,
                          hipStream_t stream) {
  if (p.acc_dtype == FDMT_F32) {
    float *o = static_cast<float *>(out);
    switch (p.in_dtype) {
      case FDMT_F32: return forward_unfused(p, static_cast<const float *>(in), o, batch, ws, stream);
      case FDMT_F16: return forward_unfused(p, static_cast<const _Float16 *>(in), o, batch, ws, stream);
      case FDMT_U8: return forward_unfused(p, static_cast<const uint8_t *>(in), o, batch, ws, stream);
      default: return hipErrorInvalidValue;
    }
  }
  int32_t *o = static_cast<int32_t *>(out);
  switch (p.in_dtype) {
    case FDMT_U8: return forward_unfused(p, static_cast<const uint8_t *>(in), o, batch, ws, stream);
    case FDMT_I32: return forward_unfused(p, static_cast<const int32_t *>(in), o, batch, ws, stream);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_adjoint(const Plan &p, const void *gout, void *gin, int batch, void *ws,
                          hipStream_t stream) {
  if (p.acc_dtype == FDMT_F32)
    return adjoint_unfused(p, static_cast<const float *>(gout), static_cast<float *>(gin), batch,
                           ws, stream);
  return adjoint_unfused(p, static_cast<const int32_t *>(gout), static_cast<int32_t *>(gin), batch,
                         ws, stream);
}

} // namespace fdmt
