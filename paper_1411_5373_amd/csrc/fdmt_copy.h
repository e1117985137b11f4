// Streaming device copy (measurement of the copy ceiling).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>

namespace fdmt {

// Enqueues a copy of `bytes` bytes; src and dst 16-byte aligned, not overlapping.
hipError_t launch_stream_copy(void *dst, const void *src, size_t bytes, hipStream_t stream);

}  // namespace fdmt
