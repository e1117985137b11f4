/*
 * fdmt.h - C ABI of the MI355X (gfx950) Fast Dispersion Measure Transform.
 *
 * The transform is the one of Zackay & Ofek, arXiv:1411.5373, Sec. 4 and
 * Algorithm 1: the input is an intensity matrix I[f][t] (channel 0 = lowest
 * frequency f_min, time contiguous, Sec. 4.2 "Memory access"), the output is
 * A[dt][t0] = the sum of I along the dispersion curve of Eq. (DtD) that
 * reaches f_min at sample t0 and spans dt samples across the band
 * (Eq. parametrization), for dt = 0 .. Nd-1 and t0 = 0 .. Nt-1.
 *
 * Discretisation (the paper leaves it to the implementation, Sec. 4.2
 * "Rounding and binning"):
 *   - channel k covers [f_min + k*df, f_min + (k+1)*df), df = (f_max-f_min)/Nf;
 *   - the addition rule merges sub-bands [f0,f1) and [f1,f2) with f1 their
 *     border frequency, t0 - t1 = round_half_up(dt * C_{f2,f0}) (Eq. Cf2f0,
 *     evaluated in IEEE float64 as (1/(f1*f1) - 1/(f0*f0)) / (1/(f2*f2) - 1/(f0*f0)),
 *     no fused multiply-add), the upper half shifted by that same amount;
 *   - Option-1 initialisation: A_f(t, d) = sum_{i=0}^{d} I[f][t-i];
 *   - samples before t = 0 are zero (the alternative addition rule for t1 < 0),
 *     so outputs with t0 < dt are sums over the part of the path inside the record;
 *   - the rows each sub-band needs are derived top-down from Nd;
 *   - Nf need not be a power of two (Sec. 4.2, the case Nf != 2^k): iteration
 *     l pairs sub-bands 2j and 2j+1 of the previous one, sub-band j holding
 *     channels j*2^l .. min((j+1)*2^l, Nf) - 1, for ceil(log2 Nf) iterations;
 *     halves of unequal width meet at their border frequency, f2 being the
 *     upper edge of the sub-band's last channel, and a sub-band whose upper
 *     half holds no channel is its lower half unchanged.
 *
 * Layout: all device arrays are dense, row-major, time fastest:
 *   forward input   [batch][Nf][Nt]   of the plan's input dtype
 *   forward output  [batch][Nd][Nt]   of the plan's accumulation dtype
 *   adjoint input   [batch][Nd][Nt]   accumulation dtype
 *   adjoint output  [batch][Nf][Nt]   accumulation dtype
 *
 * Ownership: the caller owns every input, output and workspace buffer (device
 * memory of the plan's device, e.g. tensors of a framework's allocator). The
 * plan owns its host tables and one device table buffer, allocated by
 * fdmt_plan() and released by fdmt_plan_destroy(). fdmt_forward() and
 * fdmt_adjoint() allocate nothing, never synchronise the host, and enqueue
 * their kernels on the given HIP stream (NULL = the null stream), so they are
 * stream-ordered and may be captured into a HIP graph. A plan is immutable
 * after creation and may be used from several threads and streams at once,
 * each call with its own workspace.
 *
 * Errors: every call returns a status; nothing aborts or throws across the
 * ABI. All argument checks happen before any launch, so a call that returns an
 * error other than FDMT_E_DEVICE has enqueued nothing. fdmt_last_error()
 * returns a thread-local description of the most recent failure.
 */
#ifndef FDMT_H_
#define FDMT_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fdmt_plan_s *fdmt_plan_t;
typedef struct fdmt_ragged_s *fdmt_ragged_t;

typedef enum {
  FDMT_OK = 0,
  FDMT_E_INVALID = 1,     /* null pointer, size out of range, f_min >= f_max, f_min <= 0, ... */
  FDMT_E_UNSUPPORTED = 2, /* unsupported dtype pair or schedule, host-only plan */
  FDMT_E_NOMEM = 3,       /* host or device allocation failed inside fdmt_plan() */
  FDMT_E_DEVICE = 4,      /* a HIP call or kernel launch failed */
  FDMT_E_WORKSPACE = 5    /* workspace null or smaller than fdmt_workspace_bytes() */
} fdmt_status_t;

typedef enum {
  FDMT_F32 = 0, /* IEEE binary32 */
  FDMT_F16 = 1, /* IEEE binary16 (input only) */
  FDMT_U8 = 2,  /* unsigned 8-bit integer (input only) */
  FDMT_I32 = 3  /* signed 32-bit integer */
} fdmt_dtype_t;

/* Supported (in_dtype -> acc_dtype) pairs:
 *   F32 -> F32, F16 -> F32, U8 -> F32   (FP32 accumulation; U8 -> F32 is exact
 *                                         while every path sum stays below 2^24)
 *   U8 -> I32, I32 -> I32                (integer path, exact barring int32 overflow)
 * The adjoint always reads and writes the accumulation dtype. */

#define FDMT_PLAN_HOST_ONLY 0x1u /* build the tables only; no device memory is touched
                                    and forward/adjoint return FDMT_E_UNSUPPORTED */
#define FDMT_PLAN_UNFUSED 0x2u   /* run one kernel per iteration (reference schedule,
                                    same results; used to cross-check the fused one) */
#define FDMT_PLAN_WIDE_PLANES 0x4u /* keep every intermediate plane in the accumulation
                                      dtype. By default a uint8-input plan stores the
                                      planes between two cache gathers as uint16 while
                                      every sum on them is below 2^16 (exact integers,
                                      same results, half the bytes) */
#define FDMT_PLAN_FFT 0x8u         /* also build the FFT-FDMT state (Sec. 5, Algorithm 2)
                                      for fdmt_forward_fft(): FP32 accumulation only, the
                                      padded FFT length (the smallest 2^a 3^b 5^c >=
                                      Nt + Nd - 1) at most 2^24; allocates its shift-vector
                                      table and hipFFT plans with the plan */

/* Options of a plan. Zero in any schedule field selects the built-in default;
 * schedule fields change only the kernel schedule, never the results. */
typedef struct {
  int32_t in_dtype;       /* fdmt_dtype_t of the forward input */
  int32_t acc_dtype;      /* FDMT_F32 or FDMT_I32 */
  uint32_t flags;         /* FDMT_PLAN_* bits */
  int32_t first_levels;   /* iterations fused with the initialisation, 1..8 */
  int32_t later_levels;   /* iterations per later fused pass, 1..8 */
  int32_t tile;           /* output samples per work block, 64..8192, multiple of 64 */
  int32_t lds_kib;        /* LDS budget per work block, 16..160 KiB */
  int32_t max_block_rows; /* cap on the output rows of one work block, 1..4096 */
  int32_t first_kernel;   /* kernel form of the first pass: 1 staged gather,
                             2 level-by-level merges in LDS, 3 gather through the
                             caches straight from the input (0 = default: 2) */
  int32_t later_kernel;   /* kernel form of later passes: 1 staged gather, 2 level-by-level
                             merges in LDS, 3 gather through the caches (0 = default: 3) */
  int32_t stream_tiles;   /* consecutive time tiles one LDS workgroup runs, 1..65535
                             (0 = default: 1 for staged gathers, 8 for level-by-level merges) */
  int32_t gather_rows;    /* output rows per cache-gather workgroup: 1, 2, 4, 8 or 16 */
  int32_t adjoint_levels; /* iterations per adjoint pass, 1..5 (0 = default 2) */
  int32_t adjoint_last_levels; /* iterations folded into the last adjoint pass with the
                                  transposed initialisation, 1..4 (0 = default 2) */
  int32_t gather_vecs;    /* runs of 4 samples per lane in cache gathers: 1, 2 or 4; the
                             forward gathers take at most 2, and 1 in passes of four
                             iterations (0 = default 1) */
  int32_t adjoint_last_rows; /* output rows (channels) per workgroup of the last adjoint
                                pass: 1, 2, 4, 8 or 16 (0 = adjoint_rows). Channels of one
                                sub-band read the same rows, so a workgroup of one whole
                                sub-band reads them through one L1 */
  double gamma;           /* delay law dt ~ f^gamma (Sec. 4.2, other functional forms: the
                             power -2 of Eq. Cf2f0 becomes gamma); finite, nonzero
                             (0 = default: -2, the cold-plasma law). Changes the tables
                             and so the results */
  int32_t d_min;          /* smallest total delay searched, in samples, 0..2^30 with
                             Nt + d_min + 2 Nd < 2^31 - 8192 (Sec. 4.2,
                             different range of dispersions): channel k's input is
                             delayed by pre_k = round(d_min * phi(c_k)), phi the fraction
                             of the band delay at its centre c_k, so output row dt
                             follows delay d_min + dt. Needs the first pass to gather from
                             the input (first_kernel 3, the default when d_min > 0) or
                             the unfused schedule. Changes the results */
  uint32_t adjoint_tile_major; /* bit i set: adjoint gather pass i (launch order) runs each row
                                  group's time tiles back to back on one XCD instead of all
                                  groups of a tile together; suits passes whose leaves sit at
                                  large shifts (0 = default: none). Uniform batches only:
                                  ragged launches follow their tile maps */
  int32_t gather_threads;  /* workgroup size of the forward cache gathers: 64, 128, 256, 512 or
                              1024 threads, at least 64 * gather_rows (0 = default 1024). A
                              workgroup covers its rows over (threads / 64 / rows) waves per
                              row; smaller workgroups let a CU start new work as single
                              waves finish */
  int32_t adjoint_threads; /* the same for the adjoint gathers into planes, at least
                              64 * adjoint_rows (0 = default 1024) */
  int32_t adjoint_last_threads; /* the same for the last adjoint pass (into the channels), at
                                   least 64 times its rows per workgroup (0 = adjoint_threads) */
  int32_t rule;           /* delay-table rule (Sec. 4.2, rounding and binning): 0 = one C per
                             merge at the border frequency, the halves sharing the sample t1;
                             1 = two C's: a channel is the point of its label (lower edge), a
                             sub-band spans its first to its last label, the lower half's
                             delay uses C at the lower sub-band's end label and the upper
                             half's shift C at the upper sub-band's start label, so each
                             output adds one sample per channel. Changes the results */
  int32_t search_rows;    /* fdmt_forward_search(): 0 (default) runs the boxcar search after
                             the transform, over its output; 1, 2 or 4 runs it inside the
                             last forward pass (a register gather into FP32) on each
                             workgroup's output tile in LDS, with that many rows per
                             workgroup and tiles of 2048 samples. Same results either way;
                             after the transform is the faster on MI355X at Nf = 4096 */
  int32_t first_rows;     /* output rows per workgroup of a first pass that gathers from the
                             input: 1, 2, 4, 8 or 16 (0 = gather_rows) */
  int32_t first_threads;  /* its workgroup size: 64 .. 1024, a power of two, at least
                             64 * its rows (0 = gather_threads). The first pass reads
                             input channels and the later ones planes, so their best
                             shapes differ */
  int32_t adjoint_rows;   /* output rows per workgroup of the adjoint gathers into planes:
                             1, 2, 4, 8 or 16 (0 = gather_rows); adjoint_threads must be at
                             least 64 times it */
} fdmt_options_t;

/* Build a plan: the delay tables of every iteration (Sec. 4: the rows each
 * sub-band needs are fixed before any data is seen) and the kernel schedule, then upload
 * the tables to the current HIP device.
 *   nf     channels, 1 <= nf <= 65536 (not a power of two: the forward first
 *          copies the input into the workspace with zero rows up to the next
 *          power of two, and every schedule runs on that copy)
 *   nt     samples per beam, 1 <= nt <= 2^31 - 1
 *   nd     delay trials (output rows), 1 <= nd <= 65536
 *   f_min, f_max  band edges in any one unit, 0 < f_min < f_max
 *   opt    NULL = F32 -> F32, no flags
 * On success *out holds the plan; on failure *out is NULL. */
fdmt_status_t fdmt_plan(fdmt_plan_t *out, int32_t nf, int64_t nt, int32_t nd, double f_min,
                        double f_max, const fdmt_options_t *opt);

/* Device workspace (bytes) that fdmt_forward/fdmt_adjoint need for `batch`
 * beams of the plan's Nt; 0 if the plan is NULL or batch < 1. The workspace
 * must be 256-byte aligned; its contents on entry are irrelevant. */
size_t fdmt_workspace_bytes(fdmt_plan_t p, int32_t batch);

/* Forward transform (Algorithm 1) of `batch` independent beams.
 * in  : device [batch][Nf][Nt], plan input dtype, read only
 * out : device [batch][Nd][Nt], plan accumulation dtype, fully overwritten
 * in and out must not overlap each other or the workspace. */
fdmt_status_t fdmt_forward(fdmt_plan_t p, const void *in, void *out, int32_t batch, void *ws,
                           size_t ws_bytes, void *hip_stream);

/* Adjoint (transpose) of the forward map, i.e. the gradient of a scalar loss
 * with respect to I given its gradient with respect to A: term by term the
 * transpose of the Option-1 sums and of the addition rule, evaluated as a
 * gather over precomputed inverse delay tables (no atomics; deterministic).
 * grad_out : device [batch][Nd][Nt], accumulation dtype, read only
 * grad_in  : device [batch][Nf][Nt], accumulation dtype, fully overwritten */
fdmt_status_t fdmt_adjoint(fdmt_plan_t p, const void *grad_out, void *grad_in, int32_t batch,
                           void *ws, size_t ws_bytes, void *hip_stream);

/* Kernel steps. A transform is a fixed sequence of kernel launches ("steps");
 * running steps 0 .. count-1 in order with the same arguments and workspace is
 * exactly one fdmt_forward() (adjoint = 0) or fdmt_adjoint() (adjoint = 1)
 * call. This exists to time and profile individual kernels. */
typedef struct {
  int32_t kind;          /* 0 init, 1 one iteration, 2 iterations merged level by level
                            in LDS, 3 transpose of one iteration, 4 transpose of the
                            init, 5 iterations as a gather through the caches, 6 the init
                            and iterations as a gather from the input, 7 iterations as a
                            staged gather, 8 transposes of several iterations (and of the
                            init, in the last pass) as a gather, 9 copy of the input into
                            the workspace with a zero row for each channel position past
                            Nf (Nf not a power of two) */
  int32_t level_first;   /* first iteration covered (0 = the initialisation) */
  int32_t level_last;    /* last iteration covered */
  int32_t work_items;    /* workgroups per beam */
  int64_t lds_bytes;     /* dynamic LDS per workgroup */
  int64_t bytes_read;    /* algorithmic bytes per beam: each consumed element once */
  int64_t bytes_written; /* algorithmic bytes per beam: each produced element once */
  int64_t staged_bytes;  /* bytes per beam the step's work items load, overlaps included */
  int64_t adds;          /* additions per beam */
  int32_t in_elem_bytes; /* bytes per element of what the step reads (input or plane) */
  int32_t out_elem_bytes;/* bytes per element of what the step writes */
} fdmt_step_info_t;

/* FFT-FDMT (Sec. 5, Algorithm 2): the same transform as fdmt_forward(), with
 * the time axis Fourier transformed so that every shift is a product with a
 * shift vector exp(-2 pi i w s / n). The Option-1 rows are zero-padded to n
 * samples (n >= Nt + Nd - 1, so no path wraps), transformed by hipFFT, merged
 * per frequency bin over all iterations, transformed back and scaled by 1/n.
 * Results equal fdmt_forward()'s up to FP32 rounding of the transforms (not
 * bit for bit). The plan must have been created with FDMT_PLAN_FFT; beams run
 * one after another through the workspace, whose size does not depend on
 * batch. Calls on one plan must not overlap (the hipFFT plans hold one work
 * area). Arguments and layouts as for fdmt_forward().
 * FDMT_E_INVALID for a plan without the FFT state. */
size_t fdmt_fft_workspace_bytes(fdmt_plan_t p, int32_t batch);
fdmt_status_t fdmt_forward_fft(fdmt_plan_t p, const void *in, void *out, int32_t batch, void *ws,
                               size_t ws_bytes, void *hip_stream);

/* Number of steps of the forward (adjoint = 0) or adjoint (adjoint = 1)
 * transform; -1 if p is NULL. */
int32_t fdmt_step_count(fdmt_plan_t p, int32_t adjoint);

/* Describes one step (see fdmt_step_info_t). */
fdmt_status_t fdmt_step_info(fdmt_plan_t p, int32_t adjoint, int32_t step, fdmt_step_info_t *info);

/* Enqueues one step; arguments as for fdmt_forward()/fdmt_adjoint(). */
fdmt_status_t fdmt_run_step(fdmt_plan_t p, int32_t adjoint, int32_t step, const void *in, void *out,
                            int32_t batch, void *ws, size_t ws_bytes, void *hip_stream);

/* Host copy of one sub-band's delay table (for inspection and table tests).
 * level 0: sub = channel, *n_rows = rows of its Option-1 partial sums, no
 *          triples are written.
 * level l in 1..levels: sub = sub-band index (0 .. 2^(levels-l) - 1); for
 *          each row dt < *n_rows, d_lo[dt] = t0 - t1, s[dt] = shift of the
 *          upper half, d_hi[dt] = t1 - t2, written only if cap >= *n_rows
 *          (pointers may be NULL when cap = 0). A sub-band without channels
 *          has no rows; one whose upper half has none reports (dt, 0, -1).
 * FDMT_E_INVALID for a level or sub-band out of range. */
fdmt_status_t fdmt_plan_tables(fdmt_plan_t p, int32_t level, int32_t sub, int32_t *d_lo,
                               int32_t *s, int32_t *d_hi, int32_t cap, int32_t *n_rows);

/* Plan shape: *levels = ceil(log2(Nf)); rows_per_level[l] (l = 0..levels, if
 * not NULL and cap > levels) = total rows of iteration l's planes, including
 * the single zero row kept for each sub-band position without channels. */
fdmt_status_t fdmt_plan_info(fdmt_plan_t p, int32_t *levels, int64_t *rows_per_level, int32_t cap);

/* Release the plan and its device tables (must not be in use by queued work). NULL is a no-op. */
fdmt_status_t fdmt_plan_destroy(fdmt_plan_t p);

/* Ragged batches. Beams of different lengths (a survey's beams, or records
 * cut at different places) run through one plan's kernels together: every
 * step of a transform is one launch over all beams (a further launch per
 * 65535 time tiles of that step), so the beam count does not multiply the
 * launch count. Beam b has nt[b] samples (0 allowed); the delay tables and
 * schedule are the plan's, whose own Nt is not used. Results per beam are
 * bit-identical to fdmt_forward()/fdmt_adjoint() of a plan with Nt = nt[b].
 *
 * Packed layout (dense, time fastest): beam b's [rows][nt[b]] block starts at
 * element rows * (nt[0] + ... + nt[b-1]) of the buffer, rows = Nf for the
 * forward input and the adjoint output, Nd for the forward output and the
 * adjoint input. The plan must outlive the ragged plan, which owns one small
 * device buffer (beam table and tile maps) and nothing else; the forward and
 * adjoint calls allocate nothing and may be captured into a HIP graph.
 * Many beams per device are the workload of Sec. 8 (an interferometer's
 * synthesized beams, each dedispersed on its own).
 *
 * Each step is an ordinary launch over the flattened (beam, time tile) map,
 * not a persistent work-queue kernel: on MI355X, for 256 beams of Nf = 1024,
 * Nd = 512 and 3.1 M samples in all, the gaps between a forward's four
 * launches add about 0.01 ms to its 14 ms, and two half batches cost at most
 * 0.05 ms more than one call, so a single resident kernel could save well
 * under 1% while adding spin waits between passes.
 *
 * fdmt_ragged_plan errors: FDMT_E_INVALID (NULL pointer, nbeams < 1, an nt[b]
 * outside [0, 2^31 - 1], device mismatch), FDMT_E_UNSUPPORTED (host-only plan,
 * a plan whose passes use the staged-gather kernel, more than 2^31 - 1 padded
 * samples in total), FDMT_E_NOMEM. */
fdmt_status_t fdmt_ragged_plan(fdmt_ragged_t *out, fdmt_plan_t p, int32_t nbeams, const int64_t *nt);

/* Workspace (bytes, 256-byte aligned) of a ragged forward or adjoint; 0 if r is NULL. */
size_t fdmt_ragged_workspace_bytes(fdmt_ragged_t r);

/* Forward transform of every beam of the batch.
 * in  : device, packed [Nf][nt[b]] blocks, the plan's input dtype, read only
 * out : device, packed [Nd][nt[b]] blocks, the accumulation dtype, fully overwritten
 * A batch with no samples at all enqueues nothing and accepts NULL buffers. */
fdmt_status_t fdmt_ragged_forward(fdmt_ragged_t r, const void *in, void *out, void *ws, size_t ws_bytes,
                                  void *hip_stream);

/* Adjoint of every beam: grad_out packed [Nd][nt[b]], grad_in packed [Nf][nt[b]],
 * both in the accumulation dtype. */
fdmt_status_t fdmt_ragged_adjoint(fdmt_ragged_t r, const void *grad_out, void *grad_in, void *ws,
                                  size_t ws_bytes, void *hip_stream);

/* Enqueues one step of a ragged forward (adjoint = 0) or adjoint (adjoint = 1);
 * steps and their order are the plan's (fdmt_step_count). */
fdmt_status_t fdmt_ragged_run_step(fdmt_ragged_t r, int32_t adjoint, int32_t step, const void *in, void *out,
                                   void *ws, size_t ws_bytes, void *hip_stream);

/* Shape of a ragged plan: beams, total samples, and the kernel launches of one
 * forward plus one adjoint (any pointer may be NULL). */
fdmt_status_t fdmt_ragged_info(fdmt_ragged_t r, int32_t *nbeams, int64_t *total_nt, int32_t *launches);

/* Release the ragged plan's device buffer (must not be in use by queued work). NULL is a no-op. */
fdmt_status_t fdmt_ragged_destroy(fdmt_ragged_t r);

/* Boxcar search (Sec. 4.2, pulse profile: a profile shared by every frequency
 * commutes with the transform, so boxcars of several widths run on its output
 * instead of on the input, one transform for all widths).
 * For every beam, row dt of plane[b] and width w = 2^j, j = 0..max_log2:
 *   b_w[t] = y[t] + y[t-1] + ... + y[t-w+1], y = plane[b][dt], zero before t = 0,
 * summed in FP32 as b_2w[t] = b_w[t] + b_w[t-w] from b_1 = y, and reports its
 * largest value `peak`, the first t where it occurs, the mean and (population)
 * standard deviation of b_w over t = 0..nt-1, accumulated in FP64, and
 * snr = (peak - mean) / stdev (0 when stdev is 0). NaN samples are never a
 * peak. */
typedef struct {
  float peak;
  int32_t t;
  float mean;
  float stdev;
  float snr;
} fdmt_boxcar_t;

/* A candidate event of fdmt_forward_search(): in beam `beam`, row `dt`, the
 * width-2^width_log2 running sum's largest value `peak` inside one block of
 * 2048 samples (first at time t), with snr = (peak - mean) / stdev against
 * the row's statistics of that width over the whole record. */
typedef struct {
  int32_t beam;
  int32_t dt;
  int32_t t;
  int32_t width_log2;
  float peak;
  float snr;
} fdmt_candidate_t;

/* Workspace (bytes) of fdmt_boxcar_search; 0 for invalid sizes. */
size_t fdmt_boxcar_workspace_bytes(int32_t batch, int32_t nd, int64_t nt, int32_t max_log2);

/* plane : device, [batch][nd][nt] FP32 (an FDMT output), read only
 * out   : device, [batch][max_log2 + 1][nd] results, fully overwritten
 * ws    : device scratch of fdmt_boxcar_workspace_bytes()
 * Sizes: batch, nd in [1, 65535], nt in [1, 2^31 - 1], max_log2 in [0, 10].
 * Errors: FDMT_E_INVALID (NULL pointer, a size out of range),
 * FDMT_E_WORKSPACE, FDMT_E_DEVICE. Enqueued on hip_stream; allocates nothing. */
fdmt_status_t fdmt_boxcar_search(const float *plane, int32_t batch, int32_t nd, int64_t nt, int32_t max_log2,
                                 fdmt_boxcar_t *out, void *ws, size_t ws_bytes, void *hip_stream);

/* Streaming device copy of `bytes` bytes (16-byte aligned, non-overlapping
 * device buffers), enqueued on hip_stream. Not part of the transform: a
 * kernel that reads and writes every byte once, coalesced, 16 bytes per lane,
 * so its bandwidth is the practical ceiling of the transform's HBM-bound
 * gathers on the same device (the HBM peak is the other reference).
 * FDMT_E_INVALID for NULL, misaligned or overlapping buffers; bytes = 0 is a
 * no-op. Allocates nothing. */
fdmt_status_t fdmt_copy_bytes(void *dst, const void *src, size_t bytes, void *hip_stream);

/* Streaming device kernel with a given read/write mix: reads read_bytes of src
 * once and writes write_bytes of dst once, with the copy's access shape. Not
 * part of the transform: its bandwidth is the practical ceiling of a kernel
 * that moves the same bytes in each direction, since HBM serves writes more
 * slowly than reads (a kernel writing more than it reads cannot reach the
 * copy's rate). dst unit i (16 bytes) is src unit i, or i - read_units past
 * the end of src, when writing at least as much as reading; otherwise src
 * unit i xor src unit i + write_units (the latter only inside src).
 * FDMT_E_INVALID for NULL, misaligned or overlapping buffers, byte counts not
 * multiples of 16, or one count above twice the other; both counts 0 is a
 * no-op. Allocates nothing. */
fdmt_status_t fdmt_stream_mix(void *dst, size_t write_bytes, const void *src, size_t read_bytes,
                              void *hip_stream);

/* Tuned schedule lookup. The package's autotuner times candidate schedules
 * on the GPU and stores the fastest per workload in a JSON cache; this call
 * lets a C caller start from that schedule as the Python layer does. The
 * schedule only changes speed, never results (Sec. 4.2 leaves memory access
 * and fusion to the implementation).
 *   cache_path  JSON cache; NULL = $FDMT_TUNE_CACHE if set, else the cache
 *               shipped beside the library, <dir of libfdmt.so>/tuning/<arch>.json
 *   arch        architecture name ("gfx950"); NULL = the current device's
 *   opt         in: in_dtype, acc_dtype, gamma, d_min and any explicit schedule
 *               fields (nonzero ones are kept); out: every zero schedule field
 *               that the cache entry sets is filled in (with d_min > 0 a
 *               cached first_kernel of 1 or 2 becomes 3, the gather from the
 *               input that applies the pre-shift)
 *   found       (may be NULL) 1 if the cache held this workload, else 0
 * The key is the architecture, Nf, Nd, the band, gamma when not -2, the
 * dtypes and Nt rounded up to a power of two. A missing cache file is not an
 * error (found = 0). FDMT_E_INVALID: NULL opt, sizes < 1, a malformed cache
 * or an unknown field in the matching entry; FDMT_E_DEVICE: arch NULL and no
 * current device. Touches no device memory; pass the result to fdmt_plan(). */
fdmt_status_t fdmt_tuned_options(const char *cache_path, const char *arch, int32_t nf, int64_t nt, int32_t nd,
                                 double f_min, double f_max, fdmt_options_t *opt, int32_t *found);

/* Forward transform followed by the boxcar search of its output and a list
 * of candidate events (Sec. 1: a detection is a statistic above a
 * threshold; Sec. 4.2, pulse profile: one transform serves every width).
 * out receives the forward output as fdmt_forward() (FP32 plans only);
 * stats (device, [batch][max_log2 + 1][Nd]) the per-row results of
 * fdmt_boxcar_search() on it. Every block of 2048 samples of every beam, row
 * and width whose largest running sum has snr = (peak - mean) / stdev >=
 * threshold (row statistics of that width; 0 when stdev is 0) is one
 * candidate (fdmt_candidate_t, its first time in the block): up to `cap` of
 * them are written to cands (device) in no particular order, and *count
 * (device int32) receives how many there were (it may exceed cap).
 * When fdmt_search_fused() is 1 (options.search_rows > 0 and a last pass
 * that is a register gather) the search runs inside the last forward pass on
 * each workgroup's output tile while it is in LDS, plus one small kernel for
 * the windows that cross tile starts; otherwise the standalone search
 * kernels read the transform's output back. Either way the running
 * sums are the same doubling tree as fdmt_boxcar_search(), so peaks and
 * their times are identical. ws: fdmt_search_workspace_bytes() of device
 * memory (256-byte aligned). Allocates nothing; graph-capturable (the count
 * is cleared by a kernel). Errors: those of fdmt_forward(), FDMT_E_UNSUPPORTED
 * for an int32 plan, FDMT_E_INVALID for max_log2 outside [0, 10], a NaN
 * threshold, NULL stats or count, cap < 0 or NULL cands with cap > 0. */
size_t fdmt_search_workspace_bytes(fdmt_plan_t p, int32_t batch, int32_t max_log2);
int32_t fdmt_search_fused(fdmt_plan_t p, int32_t max_log2);
fdmt_status_t fdmt_forward_search(fdmt_plan_t p, const void *in, void *out, int32_t batch, int32_t max_log2,
                                  float threshold, fdmt_boxcar_t *stats, fdmt_candidate_t *cands, int32_t cap,
                                  int32_t *count, void *ws, size_t ws_bytes, void *hip_stream);

/* The boxcar search above without a workspace argument, for callers that
 * cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid allocation): the partials live in a static
 * 32 MiB device buffer of the library, one per GPU, held until the process
 * ends. Same arguments, results and stream order as fdmt_boxcar_search();
 * allocates nothing and calls no allocating routine. The buffer keeps the
 * last call's contents (every partial is written before it is read), and
 * calls that overlap on one GPU (other streams, other threads) race on it:
 * serialise them. FDMT_E_WORKSPACE when the search needs more than 32 MiB
 * (fdmt_boxcar_workspace_bytes() > 33554432, e.g. more than 2048 rows x
 * 65536 samples x 11 widths); FDMT_E_INVALID as fdmt_boxcar_search();
 * FDMT_E_DEVICE when the buffer's device address cannot be found. */
fdmt_status_t fdmt_boxcar_search_noalloc(const float *plane, int32_t batch, int32_t nd, int64_t nt,
                                         int32_t max_log2, fdmt_boxcar_t *out, void *hip_stream);

/* Static description of a status code. */
const char *fdmt_status_string(fdmt_status_t s);

/* Thread-local detail of the last failed call on this thread ("" if none). */
const char *fdmt_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FDMT_H_ */
