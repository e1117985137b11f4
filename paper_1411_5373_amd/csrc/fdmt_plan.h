// Plan object shared by the C ABI and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/fdmt.h"
#include "fdmt_tables.h"

namespace fdmt {

constexpr int64_t kRowAlign = 64;  // plane rows start on 256-byte boundaries

inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

struct DeviceTables {
  const int4 *merge[32] = {};     // per iteration l >= 1: MergeRow per row of plane l
  const int4 *adj[32] = {};       // per iteration l >= 1: AdjRow per row of plane l - 1
  const int32_t *leaf_off = nullptr;
  const int32_t *leaf_rows = nullptr;
};

struct Plan {
  Tables tab;
  int64_t nt = 0;        // samples per beam
  int64_t ntp = 0;       // padded row stride of workspace planes
  int in_dtype = FDMT_F32, acc_dtype = FDMT_F32;
  uint32_t flags = 0;
  int device = -1;
  int64_t rmax = 0;      // tallest plane (rows)
  void *dbuf = nullptr;  // device copy of every table
  DeviceTables dev;
};

// Kernel sequences (fdmt_kernels.hip). Both assume validated arguments.
hipError_t launch_forward(const Plan &p, const void *in, void *out, int batch, void *ws,
                          hipStream_t stream);
hipError_t launch_adjoint(const Plan &p, const void *grad_out, void *grad_in, int batch, void *ws,
                          hipStream_t stream);
size_t workspace_bytes(const Plan &p, int batch);

} // namespace fdmt
