// Streaming device copy: the bandwidth a kernel that reads and writes every
// byte once can reach on this GPU, the practical ceiling the transform's
// HBM-bound kernels are measured against beside the HBM peak.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "fdmt_copy.h"

namespace fdmt {

namespace {

typedef unsigned int U4 __attribute__((ext_vector_type(4)));

constexpr int kCopyThreads = 256;
constexpr int kCopyUnits = 4;  // 16-byte units per thread, all loaded before any store

// Thread i of block b moves units b*1024 + i + 256*k, k = 0..3: every load and
// store instruction of a wave covers 1 KiB of consecutive bytes.
__global__ __launch_bounds__(kCopyThreads) void stream_copy_kernel(const U4 *__restrict__ src,
                                                                   U4 *__restrict__ dst, int64_t n16) {
  const int64_t base = static_cast<int64_t>(blockIdx.x) * (kCopyThreads * kCopyUnits) + threadIdx.x;
  U4 v[kCopyUnits];
#pragma unroll
  for (int k = 0; k < kCopyUnits; ++k) {
    const int64_t i = base + k * kCopyThreads;
    if (i < n16) v[k] = src[i];
  }
#pragma unroll
  for (int k = 0; k < kCopyUnits; ++k) {
    const int64_t i = base + k * kCopyThreads;
    if (i < n16) dst[i] = v[k];
  }
}

// A stream with a given read/write mix: unit i of dst (i < nw) takes src unit
// i, or i - nr past the source's end, when nw >= nr; when nr > nw it takes
// src unit i xor unit i + nw (the latter only while inside the source). So
// every source unit is read once, every destination unit written once, with
// nr <= 2 nw and nw <= 2 nr. Same thread shape as the copy.
__global__ __launch_bounds__(kCopyThreads) void stream_mix_kernel(const U4 *__restrict__ src, U4 *__restrict__ dst,
                                                                  int64_t nw, int64_t nr) {
  const int64_t base = static_cast<int64_t>(blockIdx.x) * (kCopyThreads * kCopyUnits) + threadIdx.x;
  U4 v[kCopyUnits];
#pragma unroll
  for (int k = 0; k < kCopyUnits; ++k) {
    const int64_t i = base + k * kCopyThreads;
    if (i < nw) {
      if (nw >= nr) {
        v[k] = src[i < nr ? i : i - nr];
      } else {
        v[k] = src[i];
        if (i + nw < nr) v[k] ^= src[i + nw];
      }
    }
  }
#pragma unroll
  for (int k = 0; k < kCopyUnits; ++k) {
    const int64_t i = base + k * kCopyThreads;
    if (i < nw) dst[i] = v[k];
  }
}

// The last bytes % 16 bytes.
__global__ void copy_tail_kernel(const unsigned char *__restrict__ src, unsigned char *__restrict__ dst, int n) {
  if (static_cast<int>(threadIdx.x) < n) dst[threadIdx.x] = src[threadIdx.x];
}

}  // namespace

hipError_t launch_stream_copy(void *dst, const void *src, size_t bytes, hipStream_t stream) {
  const int64_t n16 = static_cast<int64_t>(bytes / 16);
  const int tail = static_cast<int>(bytes % 16);
  if (n16 > 0) {
    const int64_t blocks = (n16 + kCopyThreads * kCopyUnits - 1) / (kCopyThreads * kCopyUnits);
    hipLaunchKernelGGL(stream_copy_kernel, dim3(static_cast<unsigned>(blocks)), dim3(kCopyThreads), 0, stream,
                       static_cast<const U4 *>(src), static_cast<U4 *>(dst), n16);
  }
  if (tail > 0)
    hipLaunchKernelGGL(copy_tail_kernel, dim3(1), dim3(16), 0, stream,
                       static_cast<const unsigned char *>(src) + n16 * 16,
                       static_cast<unsigned char *>(dst) + n16 * 16, tail);
  return hipGetLastError();
}

hipError_t launch_stream_mix(void *dst, size_t write_bytes, const void *src, size_t read_bytes,
                             hipStream_t stream) {
  const int64_t nw = static_cast<int64_t>(write_bytes / 16), nr = static_cast<int64_t>(read_bytes / 16);
  if (nw == 0) return hipSuccess;
  const int64_t blocks = (nw + kCopyThreads * kCopyUnits - 1) / (kCopyThreads * kCopyUnits);
  hipLaunchKernelGGL(stream_mix_kernel, dim3(static_cast<unsigned>(blocks)), dim3(kCopyThreads), 0, stream,
                     static_cast<const U4 *>(src), static_cast<U4 *>(dst), nw, nr);
  return hipGetLastError();
}

}  // namespace fdmt
