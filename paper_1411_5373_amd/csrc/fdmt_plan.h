// Plan object shared by the C ABI and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/fdmt.h"
#include "fdmt_launch.h"
#include "fdmt_schedule.h"
#include "fdmt_tables.h"

namespace fdmt {

constexpr int64_t kRowAlign = 64;  // plane rows start on 256-byte boundaries

inline int64_t round_up(int64_t x, int64_t m) { return (x + m - 1) / m * m; }

struct DeviceTables {
  const int4 *merge[32] = {};     // per iteration l >= 1: MergeRow per row of plane l
  const int4 *adj[32] = {};       // per iteration l >= 1: AdjRow per row of plane l - 1
  const int32_t *leaf_off = nullptr;
  const int32_t *leaf_rows = nullptr;
  const int32_t *pre = nullptr;   // per channel: d_min pre-shift
};

struct FftPlan;  // FFT-FDMT state (fdmt_fft.hip)

// Where a step reads or writes: the caller's input/output or one of the two
// workspace planes.
// InPad: the input copied to 2^levels channel rows, the rows past Nf zero
// (Nf not a power of two); it follows the two planes in the workspace.
enum class Buf { In, Out, Ws0, Ws1, InPad };

// One kernel launch of a transform.
struct Step {
  enum Kind { Init, Merge, Fused, MergeAdj, InitAdj, AdjGather, PadIn } kind;
  int index;  // Merge/MergeAdj: iteration l; Fused: pass index in the schedule
  Buf src, dst;
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
  Schedule fwd;                // fused forward schedule (empty when unfused)
  AdjSchedule adj;             // fused adjoint schedule (empty when unfused)
  const int4 *dev_adj_leaves = nullptr;
  const int32_t *dev_adj_starts = nullptr;
  const int32_t *dev_adj_order = nullptr;
  const Rec *dev_recs = nullptr;
  const int32_t *dev_heads = nullptr;
  const int2 *dev_terms = nullptr;
  const int4 *dev_iterms = nullptr;
  const Rec *dev_stage = nullptr;
  const Rec *dev_psums = nullptr;
  int tiles_per_wg = 1;        // time tiles one staged workgroup streams over
  int rec_tiles = 8;           // time tiles one level-by-level (LDS) workgroup runs
  int gather_rows = 8;         // output rows per register-gather workgroup
  int gather_vecs = 1;         // runs of 4 samples per lane in register gathers (1, 2 or 4)
  int gather_threads = 1024;   // workgroup size of the forward register gathers (64 .. 1024)
  int adjoint_threads = 1024;  // workgroup size of the adjoint register gathers (64 .. 1024)
  int adjoint_last_threads = 0;  // ... of the last adjoint pass (0: adjoint_threads)
  int search_rows = 0;         // rows per workgroup of the last forward pass when it runs the
                               // search (0: the search runs after the transform)
  int adjoint_last_rows = 0;   // channels per workgroup of the last adjoint pass (0: adjoint rows)
  int first_rows = 0;          // rows per workgroup of a first pass gathering from the input (0: gather_rows)
  int first_threads = 0;       // ... its workgroup size (0: gather_threads)
  int adjoint_rows = 0;        // rows per workgroup of the adjoint gathers into planes (0: gather_rows)
  uint32_t adjoint_tile_major = 0;  // bit i: adjoint pass i runs each row group's tiles back to back
  const int2 *dev_sterms = nullptr;
  const int32_t *dev_sheads = nullptr;
  std::vector<uint8_t> narrow; // per forward pass: its output plane holds uint16 sums
  std::vector<uint8_t> int_sums; // per forward pass: uint8 input or uint16 planes in, sums integers below 2^24
  std::vector<Step> fwd_steps, adj_steps;
  int64_t ws_rows = 0;         // rows of each workspace plane
  bool pad_input = false;      // Nf not a power of two: the forward reads a zero-padded copy
  FftPlan *fft = nullptr;      // FFT-FDMT state (FDMT_PLAN_FFT plans only)
};

// Beams of different lengths packed back to back: beam b's [rows][Nt_b]
// block starts at rows * (samples of beams 0..b-1) in caller buffers and at
// rows * (padded samples of beams 0..b-1) in workspace planes. Device tables
// are owned by the ragged plan of the C ABI.
struct RaggedBatch {
  int nbeams = 0;
  int64_t sum_nt = 0, sum_ntp = 0;  // samples; padded samples
  const int4 *beam = nullptr;       // per beam {nt, padded nt, first sample, first padded sample}
  struct Map {
    int tile;            // time-tile width
    int64_t count;       // tiles over all beams
    const int2 *tiles;   // per tile {beam, tile index within the beam}
  };
  std::vector<Map> maps;            // one per tile width the plan's steps use
};

// Builds fwd_steps/adj_steps and ws_rows from the tables and the schedule.
void plan_steps(Plan &p);

// Kernel sequences (fdmt_kernels.hip). All assume validated arguments; `rb`
// (null: `batch` beams of p.nt samples) switches every launch to a ragged batch.
hipError_t run_step(const Plan &p, bool adjoint, int step, const void *in, void *out, int batch,
                    void *ws, hipStream_t stream, const RaggedBatch *rb = nullptr,
                    const SearchTile *search = nullptr);
hipError_t launch_forward(const Plan &p, const void *in, void *out, int batch, void *ws,
                          hipStream_t stream, const RaggedBatch *rb = nullptr);
hipError_t launch_adjoint(const Plan &p, const void *grad_out, void *grad_in, int batch, void *ws,
                          hipStream_t stream, const RaggedBatch *rb = nullptr);
// Forward whose last pass also runs the boxcar search over its output tiles
// (uniform batches; only when search_fusable): the tile partials of windows
// inside each tile, then the edge kernel's windows across tile starts.
bool search_fusable(const Plan &p, int max_log2);
hipError_t launch_forward_search(const Plan &p, const void *in, float *out, int batch, void *ws, BoxPartial *part,
                                 int max_log2, hipStream_t stream);
// Time-tile width of a step's launches; 0 when the step has no ragged form.
int step_tile(const Plan &p, bool adjoint, int step);
// Output rows per workgroup of adjoint register-gather pass `pass`.
int adjoint_rows(const Plan &p, int pass);
// Output rows and workgroup size of forward register-gather pass `ps`.
int forward_rows(const Plan &p, const Pass &ps);
int forward_threads(const Plan &p, const Pass &ps);
// Workgroup size of adjoint register-gather pass `pass`.
int adjoint_threads(const Plan &p, int pass);
size_t workspace_bytes(const Plan &p, int batch);
size_t ragged_workspace_bytes(const Plan &p, const RaggedBatch &rb);
// Option-1 rows of every channel position of one beam into FP32 rows of
// `stride` elements (samples t < nt; the rest of each row is untouched).
hipError_t launch_init_f32(const Plan &p, const void *in, float *plane0, int64_t stride, hipStream_t stream);
// Sets the dynamic-LDS limit of the fused kernels the plan uses.
hipError_t prepare_kernels(const Plan &p);

} // namespace fdmt
