// Boxcar search over FDMT output planes (device side, fdmt_boxcar.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "../../include/fdmt.h"

namespace fdmt {

constexpr int kBoxTile = 2048;   // samples of one row per workgroup
constexpr int kBoxMaxLog2 = 10;  // widths up to 2^10 samples

// Statistics of one width over one tile of one row.
struct BoxPartial {
  double sum, sumsq;  // of b_w over the tile's samples
  float peak;         // largest b_w
  int32_t t;          // first time of it
};

size_t boxcar_workspace_bytes(int32_t batch, int32_t nd, int64_t nt, int32_t max_log2);

// Size of the library's static boxcar scratch (fdmt_boxcar_search_noalloc):
// 32 MiB, the partials of e.g. 2048 rows x 65536 samples x 11 widths.
constexpr size_t kBoxScratchBytes = size_t(32) << 20;
constexpr int kMaxDevices = 64;

// Device address of the static boxcar scratch on `device`, which must be the
// calling thread's current device (looked up on the first call per device).
hipError_t boxcar_static_scratch(int device, void **ptr);

// plane: device [batch][nd][nt] FP32; out: device [batch][max_log2 + 1][nd];
// ws: boxcar_workspace_bytes() of device memory.
hipError_t launch_boxcar(const float *plane, int32_t batch, int32_t nd, int64_t nt, int32_t max_log2,
                         fdmt_boxcar_t *out, void *ws, hipStream_t stream);

} // namespace fdmt
