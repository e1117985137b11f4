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

// The steps of the search. Partials part[((b * (max_log2 + 1) + j) * nd + row) * ntiles + tile]
// cover tile `tile` = samples [tile * kBoxTile, (tile + 1) * kBoxTile) of
// row `row`; the tile kernel fills them from the plane, or the last forward
// pass fills the windows inside each tile and launch_boxcar_edges adds the
// windows straddling each tile start. combine reduces them per row (and
// stores the float64 mean and stdev in mean_sd when not null); candidates
// keeps each tile's peak whose S/N reaches the threshold.
hipError_t launch_boxcar_tiles(const float *plane, int32_t batch, int32_t nd, int64_t nt, int32_t max_log2,
                               BoxPartial *part, hipStream_t stream);
hipError_t launch_boxcar_edges(const float *plane, int32_t batch, int32_t nd, int64_t nt, int32_t max_log2,
                               BoxPartial *part, hipStream_t stream);
hipError_t launch_boxcar_combine(const BoxPartial *part, int32_t batch, int32_t nd, int64_t nt, int32_t max_log2,
                                 fdmt_boxcar_t *out, double2 *mean_sd, hipStream_t stream);
hipError_t launch_boxcar_candidates(const BoxPartial *part, const double2 *mean_sd, int32_t batch, int32_t nd,
                                    int64_t nt, int32_t max_log2, float threshold, fdmt_candidate_t *cand,
                                    int32_t cap, int32_t *found, hipStream_t stream);

} // namespace fdmt
