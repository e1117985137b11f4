// Streaming device copy (measurement of the copy ceiling).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace fdmt {

// Enqueues a copy of `bytes` bytes; src and dst 16-byte aligned, not overlapping.
hipError_t launch_stream_copy(void *dst, const void *src, size_t bytes, hipStream_t stream);

// Enqueues a stream that reads read_bytes of src once and writes write_bytes
// of dst once (multiples of 16, 16-byte aligned, not overlapping, each at
// most twice the other).
hipError_t launch_stream_mix(void *dst, size_t write_bytes, const void *src, size_t read_bytes,
                             hipStream_t stream);

}  // namespace fdmt
