// C ABI of the FDMT library: argument validation, plan lifetime, table
// upload and error reporting. See include/fdmt.h for the contract.
#include <hip/hip_runtime.h>

#include <dlfcn.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <map>
#include <new>
#include <string>

#include "../../include/fdmt.h"
#include "fdmt_boxcar.h"
#include "fdmt_copy.h"
#include "fdmt_fft.h"
#include "fdmt_plan.h"
#include "fdmt_tune.h"

struct fdmt_plan_s {
  fdmt::Plan plan;
};

struct fdmt_ragged_s {
  fdmt_plan_t plan = nullptr;  // borrowed; must outlive the ragged plan
  fdmt::RaggedBatch rb;
  void *dbuf = nullptr;        // beam table and tile maps
  int device = -1;
};

namespace {

thread_local std::string g_last_error;

fdmt_status_t fail(fdmt_status_t s, const std::string &msg) {
  g_last_error = msg;
  return s;
}

fdmt_status_t device_fail(hipError_t e, const char *where) {
  return fail(FDMT_E_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

bool pair_supported(int in, int acc) {
  if (acc == FDMT_F32) return in == FDMT_F32 || in == FDMT_F16 || in == FDMT_U8;
  if (acc == FDMT_I32) return in == FDMT_U8 || in == FDMT_I32;
  return false;
}

// Copies every table into one device allocation and records typed pointers.
fdmt_status_t upload(fdmt::Plan &p) {
  const fdmt::Tables &T = p.tab;
  size_t bytes = 0;
  auto reserve = [&](size_t n) {
    size_t off = bytes;
    bytes += fdmt::round_up(static_cast<int64_t>(n), 256);
    return off;
  };
  size_t off_merge[32] = {}, off_adj[32] = {};
  for (int l = 1; l <= T.levels; ++l) {
    off_merge[l] = reserve(T.merge[l].size() * sizeof(fdmt::MergeRow));
    off_adj[l] = reserve(T.adj[l].size() * sizeof(fdmt::AdjRow));
  }
  const size_t off_leaf_off = reserve(T.leaf_off.size() * sizeof(int32_t));
  const size_t off_leaf_rows = reserve(T.leaf_rows.size() * sizeof(int32_t));
  const size_t off_pre = reserve(T.pre.size() * sizeof(int32_t));
  const size_t off_recs = reserve(p.fwd.recs.size() * sizeof(fdmt::Rec));
  const size_t off_heads = reserve(p.fwd.heads.size() * sizeof(int32_t));
  const size_t off_terms = reserve(p.fwd.terms.size() * sizeof(fdmt::Term));
  const size_t off_iterms = reserve(p.fwd.iterms.size() * sizeof(fdmt::InTerm));
  const size_t off_stage = reserve(p.fwd.stage.size() * sizeof(fdmt::Rec));
  const size_t off_psums = reserve(p.fwd.psums.size() * sizeof(fdmt::Rec));
  const size_t off_adj_leaves = reserve((p.adj.leaves.size() + fdmt::kAdjLeafPad) * sizeof(fdmt::AdjLeaf));
  const size_t off_adj_starts = reserve(p.adj.starts.size() * sizeof(int32_t));
  const size_t off_adj_order = reserve(p.adj.order.size() * sizeof(int32_t));
  const size_t off_sterms = reserve(p.fwd.sterms.size() * sizeof(fdmt::StagedTerm));
  const size_t off_sheads = reserve(p.fwd.sheads.size() * sizeof(int32_t));

  std::vector<unsigned char> host(bytes, 0);
  for (int l = 1; l <= T.levels; ++l) {
    std::memcpy(host.data() + off_merge[l], T.merge[l].data(), T.merge[l].size() * sizeof(fdmt::MergeRow));
    std::memcpy(host.data() + off_adj[l], T.adj[l].data(), T.adj[l].size() * sizeof(fdmt::AdjRow));
  }
  std::memcpy(host.data() + off_leaf_off, T.leaf_off.data(), T.leaf_off.size() * sizeof(int32_t));
  std::memcpy(host.data() + off_leaf_rows, T.leaf_rows.data(), T.leaf_rows.size() * sizeof(int32_t));
  std::memcpy(host.data() + off_pre, T.pre.data(), T.pre.size() * sizeof(int32_t));
  if (!p.fwd.recs.empty())
    std::memcpy(host.data() + off_recs, p.fwd.recs.data(), p.fwd.recs.size() * sizeof(fdmt::Rec));
  if (!p.fwd.heads.empty())
    std::memcpy(host.data() + off_heads, p.fwd.heads.data(), p.fwd.heads.size() * sizeof(int32_t));
  if (!p.fwd.terms.empty())
    std::memcpy(host.data() + off_terms, p.fwd.terms.data(), p.fwd.terms.size() * sizeof(fdmt::Term));
  if (!p.fwd.iterms.empty())
    std::memcpy(host.data() + off_iterms, p.fwd.iterms.data(), p.fwd.iterms.size() * sizeof(fdmt::InTerm));
  if (!p.fwd.stage.empty())
    std::memcpy(host.data() + off_stage, p.fwd.stage.data(), p.fwd.stage.size() * sizeof(fdmt::Rec));
  if (!p.fwd.psums.empty())
    std::memcpy(host.data() + off_psums, p.fwd.psums.data(), p.fwd.psums.size() * sizeof(fdmt::Rec));
  if (!p.adj.leaves.empty())
    std::memcpy(host.data() + off_adj_leaves, p.adj.leaves.data(), p.adj.leaves.size() * sizeof(fdmt::AdjLeaf));
  if (!p.adj.starts.empty())
    std::memcpy(host.data() + off_adj_starts, p.adj.starts.data(), p.adj.starts.size() * sizeof(int32_t));
  if (!p.adj.order.empty())
    std::memcpy(host.data() + off_adj_order, p.adj.order.data(), p.adj.order.size() * sizeof(int32_t));
  if (!p.fwd.sterms.empty())
    std::memcpy(host.data() + off_sterms, p.fwd.sterms.data(), p.fwd.sterms.size() * sizeof(fdmt::StagedTerm));
  if (!p.fwd.sheads.empty())
    std::memcpy(host.data() + off_sheads, p.fwd.sheads.data(), p.fwd.sheads.size() * sizeof(int32_t));

  hipError_t e = hipGetDevice(&p.device);
  if (e != hipSuccess) return device_fail(e, "hipGetDevice");
  e = hipMalloc(&p.dbuf, bytes);
  if (e != hipSuccess) {
    p.dbuf = nullptr;
    return fail(FDMT_E_NOMEM, std::string("hipMalloc of delay tables: ") + hipGetErrorString(e));
  }
  e = hipMemcpy(p.dbuf, host.data(), bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) return device_fail(e, "hipMemcpy of delay tables");
  auto *base = static_cast<unsigned char *>(p.dbuf);
  for (int l = 1; l <= T.levels; ++l) {
    p.dev.merge[l] = reinterpret_cast<const int4 *>(base + off_merge[l]);
    p.dev.adj[l] = reinterpret_cast<const int4 *>(base + off_adj[l]);
  }
  p.dev.leaf_off = reinterpret_cast<const int32_t *>(base + off_leaf_off);
  p.dev.leaf_rows = reinterpret_cast<const int32_t *>(base + off_leaf_rows);
  p.dev.pre = reinterpret_cast<const int32_t *>(base + off_pre);
  p.dev_recs = reinterpret_cast<const fdmt::Rec *>(base + off_recs);
  p.dev_heads = reinterpret_cast<const int32_t *>(base + off_heads);
  p.dev_terms = reinterpret_cast<const int2 *>(base + off_terms);
  p.dev_iterms = reinterpret_cast<const int4 *>(base + off_iterms);
  p.dev_stage = reinterpret_cast<const fdmt::Rec *>(base + off_stage);
  p.dev_psums = reinterpret_cast<const fdmt::Rec *>(base + off_psums);
  p.dev_adj_leaves = reinterpret_cast<const int4 *>(base + off_adj_leaves);
  p.dev_adj_starts = reinterpret_cast<const int32_t *>(base + off_adj_starts);
  p.dev_adj_order = reinterpret_cast<const int32_t *>(base + off_adj_order);
  p.dev_sterms = reinterpret_cast<const int2 *>(base + off_sterms);
  p.dev_sheads = reinterpret_cast<const int32_t *>(base + off_sheads);
  e = fdmt::prepare_kernels(p);
  if (e != hipSuccess) return device_fail(e, "hipFuncSetAttribute (dynamic LDS)");
  return FDMT_OK;
}

fdmt_status_t check_call(fdmt_plan_t p, const void *a, const void *b, int32_t batch, void *ws,
                         size_t ws_bytes) {
  if (!p) return fail(FDMT_E_INVALID, "plan is NULL");
  if (!a || !b) return fail(FDMT_E_INVALID, "input or output pointer is NULL");
  if (a == b) return fail(FDMT_E_INVALID, "input and output alias");
  if (batch < 1 || batch > 65535) return fail(FDMT_E_INVALID, "batch must be in [1, 65535]");
  const size_t need = fdmt::workspace_bytes(p->plan, batch);
  if (need > 0 && (!ws || ws_bytes < need))
    return fail(FDMT_E_WORKSPACE, "workspace needs " + std::to_string(need) + " bytes, got " +
                                      std::to_string(ws ? ws_bytes : 0));
  if (need > 0 && (reinterpret_cast<uintptr_t>(ws) & 255u) != 0)
    return fail(FDMT_E_WORKSPACE, "workspace must be 256-byte aligned");
  if (p->plan.flags & FDMT_PLAN_HOST_ONLY)
    return fail(FDMT_E_UNSUPPORTED, "plan was built with FDMT_PLAN_HOST_ONLY");
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return device_fail(e, "hipGetDevice");
  if (dev != p->plan.device)
    return fail(FDMT_E_INVALID, "current device differs from the plan's device");
  return FDMT_OK;
}

fdmt_status_t check_ragged(fdmt_ragged_t r, const void *a, const void *b, void *ws, size_t ws_bytes) {
  if (!r) return fail(FDMT_E_INVALID, "ragged plan is NULL");
  if (r->rb.sum_nt == 0) return FDMT_OK;  // nothing to read or write
  if (!a || !b) return fail(FDMT_E_INVALID, "input or output pointer is NULL");
  if (a == b) return fail(FDMT_E_INVALID, "input and output alias");
  const size_t need = fdmt::ragged_workspace_bytes(r->plan->plan, r->rb);
  if (need > 0 && (!ws || ws_bytes < need))
    return fail(FDMT_E_WORKSPACE, "workspace needs " + std::to_string(need) + " bytes, got " +
                                      std::to_string(ws ? ws_bytes : 0));
  if (need > 0 && (reinterpret_cast<uintptr_t>(ws) & 255u) != 0)
    return fail(FDMT_E_WORKSPACE, "workspace must be 256-byte aligned");
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return device_fail(e, "hipGetDevice");
  if (dev != r->device) return fail(FDMT_E_INVALID, "current device differs from the plan's device");
  return FDMT_OK;
}

} // namespace

extern "C" {

fdmt_status_t fdmt_plan(fdmt_plan_t *out, int32_t nf, int64_t nt, int32_t nd, double f_min,
                        double f_max, const fdmt_options_t *opt) {
  if (!out) return fail(FDMT_E_INVALID, "out is NULL");
  *out = nullptr;
  fdmt_options_t o{FDMT_F32, FDMT_F32, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
  if (opt) o = *opt;
  if (nf < 1 || nf > 65536) return fail(FDMT_E_INVALID, "Nf must be in [1, 65536]");
  if (nt < 1 || nt > INT32_MAX) return fail(FDMT_E_INVALID, "Nt must be in [1, 2^31 - 1]");
  if (nd < 1 || nd > 65536) return fail(FDMT_E_INVALID, "Nd must be in [1, 65536]");
  if (!(f_min > 0.0) || !(f_max > f_min) || !std::isfinite(f_max))
    return fail(FDMT_E_INVALID, "need 0 < f_min < f_max (finite)");
  if (o.first_levels < 0 || o.first_levels > 8 || o.later_levels < 0 || o.later_levels > 8)
    return fail(FDMT_E_INVALID, "fused iterations per pass must be in [1, 8]");
  if (o.tile < 0 || (o.tile && (o.tile < 64 || o.tile > 8192 || o.tile % 64)))
    return fail(FDMT_E_INVALID, "tile must be a multiple of 64 in [64, 8192]");
  if (o.lds_kib < 0 || (o.lds_kib && (o.lds_kib < 16 || o.lds_kib > 160)))
    return fail(FDMT_E_INVALID, "lds_kib must be in [16, 160]");
  if (o.first_kernel < 0 || o.first_kernel > 3 || o.later_kernel < 0 || o.later_kernel > 3)
    return fail(FDMT_E_INVALID, "unknown pass kernel");
  if (o.stream_tiles < 0 || o.stream_tiles > 65535)
    return fail(FDMT_E_INVALID, "stream_tiles must be in [1, 65535]");
  if (o.gather_rows < 0 || o.gather_rows > 16 || (o.gather_rows & (o.gather_rows - 1)))
    return fail(FDMT_E_INVALID, "gather_rows must be 1, 2, 4, 8 or 16");
  if (o.adjoint_levels < 0 || o.adjoint_levels > 5 || o.adjoint_last_levels < 0 || o.adjoint_last_levels > 4)
    return fail(FDMT_E_INVALID, "adjoint_levels must be in [1, 5], adjoint_last_levels in [1, 4]");
  if (o.gather_vecs < 0 || o.gather_vecs > 4 || o.gather_vecs == 3)
    return fail(FDMT_E_INVALID, "gather_vecs must be 1, 2 or 4");
  for (int32_t rw : {o.adjoint_last_rows, o.first_rows, o.adjoint_rows})
    if (rw < 0 || rw > 16 || (rw & (rw - 1)))
      return fail(FDMT_E_INVALID, "adjoint_last_rows, first_rows and adjoint_rows must be 1, 2, 4, 8 or 16");
  for (int32_t th : {o.gather_threads, o.adjoint_threads, o.adjoint_last_threads, o.first_threads})
    if (th < 0 || th > 1024 || (th && (th < 64 || (th & (th - 1)))))
      return fail(FDMT_E_INVALID, "gather_threads, adjoint_threads, adjoint_last_threads and first_threads must be "
                                  "64, 128, 256, 512 or 1024");
  {
    const int rows = o.gather_rows ? o.gather_rows : 8;
    const int threads = o.gather_threads ? o.gather_threads : 1024;
    const int adj_rows = o.adjoint_rows ? o.adjoint_rows : rows;
    const int last_rows = o.adjoint_last_rows ? o.adjoint_last_rows : adj_rows;
    const int adj = o.adjoint_threads ? o.adjoint_threads : 1024;
    if (64 * rows > threads) return fail(FDMT_E_INVALID, "gather_threads must be at least 64 * gather_rows");
    if (64 * (o.first_rows ? o.first_rows : rows) > (o.first_threads ? o.first_threads : threads))
      return fail(FDMT_E_INVALID, "the first pass's workgroup must hold at least 64 * its rows threads");
    if (64 * adj_rows > adj) return fail(FDMT_E_INVALID, "adjoint_threads must be at least 64 * adjoint_rows");
    if (64 * last_rows > (o.adjoint_last_threads ? o.adjoint_last_threads : adj))
      return fail(FDMT_E_INVALID, "the last adjoint pass's workgroup must hold at least 64 * its rows threads");
  }
  // Shifts, sample indices and their sums stay int32 in the kernels: d_min is
  // at most 2^30, and Nt + d_min + 2 Nd leaves 2^13 samples of headroom.
  if (o.d_min < 0 || o.d_min > (1 << 30)) return fail(FDMT_E_INVALID, "d_min must be in [0, 2^30]");
  if (o.rule != 0 && o.rule != 1) return fail(FDMT_E_INVALID, "rule must be 0 (one C) or 1 (two C's)");
  if (o.search_rows < 0 || o.search_rows > 4 || (o.search_rows & (o.search_rows - 1)))
    return fail(FDMT_E_INVALID, "search_rows must be 1, 2 or 4");
  if (nt + o.d_min + 2 * static_cast<int64_t>(nd) > INT32_MAX - 8192)
    return fail(FDMT_E_INVALID, "Nt + d_min + 2 Nd must stay below 2^31 - 8192");
  if (o.max_block_rows < 0 || o.max_block_rows > 4096)
    return fail(FDMT_E_INVALID, "max_block_rows must be in [1, 4096]");
  if (o.flags & ~(FDMT_PLAN_HOST_ONLY | FDMT_PLAN_UNFUSED | FDMT_PLAN_WIDE_PLANES | FDMT_PLAN_FFT))
    return fail(FDMT_E_INVALID, "unknown option flag");
  if ((o.flags & FDMT_PLAN_FFT) && o.acc_dtype != FDMT_F32)
    return fail(FDMT_E_UNSUPPORTED, "FFT-FDMT accumulates in FP32 only");
  if (!pair_supported(o.in_dtype, o.acc_dtype))
    return fail(FDMT_E_UNSUPPORTED, "unsupported (input, accumulation) dtype pair");

  auto *h = new (std::nothrow) fdmt_plan_s;
  if (!h) return fail(FDMT_E_NOMEM, "host allocation of the plan failed");
  fdmt::Plan &p = h->plan;
  try {
    const std::string err =
        fdmt::build_tables(p.tab, nf, nd, f_min, f_max, o.gamma != 0.0 ? o.gamma : -2.0, o.d_min, o.rule);
    if (!err.empty()) {
      delete h;
      return fail(FDMT_E_INVALID, err);
    }
  } catch (const std::bad_alloc &) {
    delete h;
    return fail(FDMT_E_NOMEM, "host allocation of the delay tables failed");
  }
  p.nt = nt;
  p.ntp = fdmt::round_up(nt, fdmt::kRowAlign);
  p.in_dtype = o.in_dtype;
  p.acc_dtype = o.acc_dtype;
  p.flags = o.flags;
  if (o.stream_tiles) p.tiles_per_wg = p.rec_tiles = o.stream_tiles;
  if (o.gather_rows) p.gather_rows = o.gather_rows;
  if (o.gather_vecs) p.gather_vecs = o.gather_vecs;
  if (o.gather_threads) p.gather_threads = o.gather_threads;
  if (o.adjoint_threads) p.adjoint_threads = o.adjoint_threads;
  p.adjoint_last_threads = o.adjoint_last_threads;
  if (o.search_rows) p.search_rows = o.search_rows;
  p.adjoint_last_rows = o.adjoint_last_rows;
  p.first_rows = o.first_rows;
  p.first_threads = o.first_threads;
  p.adjoint_rows = o.adjoint_rows;
  p.adjoint_tile_major = o.adjoint_tile_major;
  for (int64_t r : p.tab.total) p.rmax = r > p.rmax ? r : p.rmax;
  if (!(o.flags & FDMT_PLAN_UNFUSED)) {
    fdmt::ScheduleParams sp;
    if (o.first_levels) {
      sp.first_levels = o.first_levels;
      sp.first_auto = false;
    }
    if (o.later_levels) {
      sp.later_levels = o.later_levels;
      sp.later_auto = false;
    }
    if (o.tile) sp.tile = o.tile;
    if (o.lds_kib) sp.lds_bytes = o.lds_kib * 1024;
    if (o.max_block_rows) sp.max_block_rows = o.max_block_rows;
    static const fdmt::PassKind kinds[] = {fdmt::PassKind::Staged, fdmt::PassKind::Staged,
                                           fdmt::PassKind::Recursive, fdmt::PassKind::Register};
    if (o.first_kernel) sp.first_kind = kinds[o.first_kernel];
    // the d_min pre-shift rides on the input terms of a gather from the input
    else if (o.d_min > 0) sp.first_kind = fdmt::PassKind::Register;
    if (o.later_kernel) sp.later_kind = kinds[o.later_kernel];
    try {
      const std::string err = fdmt::build_schedule(p.fwd, p.tab, sp);
      if (!err.empty()) {
        delete h;
        return fail(FDMT_E_UNSUPPORTED, "schedule: " + err);
      }
    } catch (const std::bad_alloc &) {
      delete h;
      return fail(FDMT_E_NOMEM, "host allocation of the schedule failed");
    }
  }
  if (!(o.flags & FDMT_PLAN_UNFUSED)) {
    try {
      const int per = o.adjoint_levels ? o.adjoint_levels : 2;
      const int last = o.adjoint_last_levels ? o.adjoint_last_levels : 2;
      const std::string err = fdmt::build_adjoint_schedule(p.adj, p.tab, per, last);
      if (!err.empty()) {
        delete h;
        return fail(FDMT_E_UNSUPPORTED, "adjoint schedule: " + err);
      }
    } catch (const std::bad_alloc &) {
      delete h;
      return fail(FDMT_E_NOMEM, "host allocation of the adjoint schedule failed");
    }
  }
  // uint16 planes between two cache gathers of a uint8-input plan: plane l
  // sums at most 2^l + dt input samples per element (one per channel plus the
  // chain lengths), so it is exact in 16 bits while 255 * (2^l + rows - 1)
  // stays below 2^16. A run of such planes starts at the gather from the
  // input: each narrow plane is made from the input or from a narrow plane.
  p.narrow.assign(p.fwd.passes.size(), 0);
  if (o.in_dtype == FDMT_U8 && !(o.flags & FDMT_PLAN_WIDE_PLANES)) {
    for (size_t i = 0; i + 1 < p.fwd.passes.size(); ++i) {
      const fdmt::Pass &a = p.fwd.passes[i], &b = p.fwd.passes[i + 1];
      if (!a.gather || !b.gather || b.from_input) continue;
      if (!a.from_input && !(i > 0 && p.narrow[i - 1])) continue;
      int64_t rows = 0;
      for (int32_t r : p.tab.rows[a.l1]) rows = std::max<int64_t>(rows, r);
      if (255 * ((int64_t(1) << a.l1) + rows - 1) <= 65535) p.narrow[i] = 1;
    }
  }
  // Gathers over uint8 input or uint16 planes whose sums stay integers below
  // 2^24 (every plane-l value is at most 255 * (2^l + rows - 1)) may add in
  // any order: int32 lanes, wide per-lane loads.
  p.int_sums.assign(p.fwd.passes.size(), 0);
  for (size_t i = 0; i < p.fwd.passes.size(); ++i) {
    const fdmt::Pass &a = p.fwd.passes[i];
    if (!a.gather) continue;
    if (!(a.from_input ? o.in_dtype == FDMT_U8 : i > 0 && p.narrow[i - 1])) continue;
    int64_t rows = 0;
    for (int32_t r : p.tab.rows[a.l1]) rows = std::max<int64_t>(rows, r);
    if (o.acc_dtype == FDMT_I32 || 255 * ((int64_t(1) << a.l1) + rows - 1) < (int64_t(1) << 24)) p.int_sums[i] = 1;
  }
  p.pad_input = p.tab.slots != p.tab.nf;
  fdmt::plan_steps(p);
  // Time tiles of uniform batches run along the grid's y dimension (at most
  // 65535 workgroups).
  int64_t min_tile = INT32_MAX;
  for (int adj = 0; adj < 2; ++adj) {
    const int n = static_cast<int>(adj ? p.adj_steps.size() : p.fwd_steps.size());
    for (int i = 0; i < n; ++i) {
      const int w = fdmt::step_tile(p, adj != 0, i);
      if (w > 0) min_tile = std::min<int64_t>(min_tile, w);
    }
  }
  if ((nt + min_tile - 1) / min_tile > 65535) {
    delete h;
    return fail(FDMT_E_UNSUPPORTED, "Nt too long for the time tile (more than 65535 tiles)");
  }
  if ((o.flags & FDMT_PLAN_FFT) && fdmt::fft_length(nt, nd) > fdmt::kFftMaxLength) {
    delete h;
    return fail(FDMT_E_UNSUPPORTED, "FFT-FDMT length Nt + Nd - 1 above 2^24 samples");
  }
  if (!(o.flags & FDMT_PLAN_HOST_ONLY)) {
    fdmt_status_t s = upload(p);
    if (s == FDMT_OK && (o.flags & FDMT_PLAN_FFT)) {
      const std::string err = fdmt::fft_create(p);
      if (!err.empty()) s = fail(FDMT_E_DEVICE, "FFT-FDMT: " + err);
    }
    if (s != FDMT_OK) {
      fdmt::fft_destroy(p);
      if (p.dbuf) (void)hipFree(p.dbuf);
      delete h;
      return s;
    }
  }
  *out = h;
  return FDMT_OK;
}

size_t fdmt_fft_workspace_bytes(fdmt_plan_t p, int32_t batch) {
  if (!p || batch < 1) return 0;
  return fdmt::fft_workspace_bytes(p->plan);
}

fdmt_status_t fdmt_forward_fft(fdmt_plan_t p, const void *in, void *out, int32_t batch, void *ws,
                               size_t ws_bytes, void *hip_stream) {
  if (!p) return fail(FDMT_E_INVALID, "plan is NULL");
  if (!p->plan.fft) return fail(FDMT_E_INVALID, "plan was built without FDMT_PLAN_FFT");
  if (!in || !out) return fail(FDMT_E_INVALID, "input or output pointer is NULL");
  if (in == out) return fail(FDMT_E_INVALID, "input and output alias");
  if (batch < 1 || batch > 65535) return fail(FDMT_E_INVALID, "batch must be in [1, 65535]");
  const size_t need = fdmt::fft_workspace_bytes(p->plan);
  if (!ws || ws_bytes < need)
    return fail(FDMT_E_WORKSPACE, "workspace needs " + std::to_string(need) + " bytes, got " +
                                      std::to_string(ws ? ws_bytes : 0));
  if ((reinterpret_cast<uintptr_t>(ws) & 255u) != 0) return fail(FDMT_E_WORKSPACE, "workspace must be 256-byte aligned");
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return device_fail(e, "hipGetDevice");
  if (dev != p->plan.device) return fail(FDMT_E_INVALID, "current device differs from the plan's device");
  const std::string err = fdmt::launch_forward_fft(p->plan, in, out, batch, ws, static_cast<hipStream_t>(hip_stream));
  if (!err.empty()) return fail(FDMT_E_DEVICE, "fdmt_forward_fft: " + err);
  return FDMT_OK;
}

size_t fdmt_workspace_bytes(fdmt_plan_t p, int32_t batch) {
  if (!p || batch < 1) return 0;
  return fdmt::workspace_bytes(p->plan, batch);
}

fdmt_status_t fdmt_forward(fdmt_plan_t p, const void *in, void *out, int32_t batch, void *ws,
                           size_t ws_bytes, void *hip_stream) {
  fdmt_status_t s = check_call(p, in, out, batch, ws, ws_bytes);
  if (s != FDMT_OK) return s;
  hipError_t e = fdmt::launch_forward(p->plan, in, out, batch, ws, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return device_fail(e, "fdmt_forward launch");
  return FDMT_OK;
}

fdmt_status_t fdmt_adjoint(fdmt_plan_t p, const void *grad_out, void *grad_in, int32_t batch,
                           void *ws, size_t ws_bytes, void *hip_stream) {
  fdmt_status_t s = check_call(p, grad_out, grad_in, batch, ws, ws_bytes);
  if (s != FDMT_OK) return s;
  hipError_t e = fdmt::launch_adjoint(p->plan, grad_out, grad_in, batch, ws, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return device_fail(e, "fdmt_adjoint launch");
  return FDMT_OK;
}

int32_t fdmt_step_count(fdmt_plan_t p, int32_t adjoint) {
  if (!p) return -1;
  return static_cast<int32_t>(adjoint ? p->plan.adj_steps.size() : p->plan.fwd_steps.size());
}

fdmt_status_t fdmt_step_info(fdmt_plan_t p, int32_t adjoint, int32_t step, fdmt_step_info_t *info) {
  if (!p || !info) return fail(FDMT_E_INVALID, "plan or info is NULL");
  const fdmt::Plan &P = p->plan;
  const auto &steps = adjoint ? P.adj_steps : P.fwd_steps;
  if (step < 0 || step >= static_cast<int32_t>(steps.size()))
    return fail(FDMT_E_INVALID, "step out of range");
  const fdmt::Step &st = steps[step];
  const fdmt::Tables &T = P.tab;
  const int64_t nt = P.nt;
  const int64_t in_b = P.in_dtype == FDMT_U8 ? 1 : (P.in_dtype == FDMT_F16 ? 2 : 4);
  *info = fdmt_step_info_t{};
  info->kind = static_cast<int32_t>(st.kind);
  // unless set below: reads the input (init) or a 4-byte plane, writes 4-byte elements
  info->in_elem_bytes =
      st.kind == fdmt::Step::Init || st.kind == fdmt::Step::PadIn ? static_cast<int32_t>(in_b) : 4;
  info->out_elem_bytes = 4;
  auto init_adds = [&]() {
    int64_t a = 0;
    for (int k = 0; k < T.nf; ++k) a += T.leaf_rows[k] - 1;
    return a * nt;
  };
  switch (st.kind) {
    case fdmt::Step::PadIn:
      info->kind = 9;
      info->work_items = T.slots;
      info->bytes_read = static_cast<int64_t>(T.nf) * nt * in_b;
      info->bytes_written = static_cast<int64_t>(T.slots) * nt * in_b;
      info->staged_bytes = info->bytes_read;
      info->out_elem_bytes = static_cast<int32_t>(in_b);
      break;
    case fdmt::Step::Init:
      info->level_first = info->level_last = 0;
      info->work_items = T.slots;
      info->bytes_read = static_cast<int64_t>(T.nf) * nt * in_b;
      info->bytes_written = T.total[0] * nt * 4;
      info->staged_bytes = info->bytes_read;
      info->adds = init_adds();
      break;
    case fdmt::Step::Merge:
      info->level_first = info->level_last = st.index;
      info->work_items = static_cast<int32_t>(T.total[st.index]);
      info->bytes_read = T.total[st.index - 1] * nt * 4;
      info->bytes_written = T.total[st.index] * nt * 4;
      info->staged_bytes = 2 * T.total[st.index] * nt * 4;
      info->adds = T.total[st.index] * nt;
      break;
    case fdmt::Step::Fused: {
      const fdmt::Pass &ps = P.fwd.passes[st.index];
      info->kind = ps.kind == fdmt::PassKind::Staged ? 7 : !ps.gather ? 2 : ps.from_input ? 6 : 5;
      info->level_first = ps.from_input ? 0 : ps.l0 + 1;
      info->level_last = ps.l1;
      const int64_t gt = fdmt::step_tile(P, false, step);  // samples per gather workgroup
      const int rows = fdmt::forward_rows(P, ps);
      info->work_items = ps.gather ? static_cast<int32_t>(((ps.nblocks + rows - 1) / rows) * ((nt + gt - 1) / gt))
                                   : static_cast<int32_t>(
                                         ps.nblocks *
                                         ((nt + ps.tile - 1) / ps.tile +
                                          (ps.kind == fdmt::PassKind::Staged ? P.tiles_per_wg : P.rec_tiles) - 1) /
                                         (ps.kind == fdmt::PassKind::Staged ? P.tiles_per_wg : P.rec_tiles));
      info->lds_bytes = ps.gather ? 0
                        : ps.kind == fdmt::PassKind::Staged
                            ? static_cast<int64_t>(ps.lds_a + ps.lds_p + ps.lds_b + ps.max_recs) * 4
                            : static_cast<int64_t>(ps.lds_a + ps.lds_b + 2 * fdmt::kLdsSlack) * 4;
      const bool narrow_in = st.index > 0 && P.narrow[st.index - 1];
      const int64_t eb = ps.from_input ? in_b : narrow_in ? 2 : 4;
      const int64_t ob = P.narrow[st.index] ? 2 : 4;
      info->in_elem_bytes = static_cast<int32_t>(eb);
      info->out_elem_bytes = static_cast<int32_t>(ob);
      info->bytes_read = ps.rows_in * nt * eb;
      info->bytes_written = ps.rows_out * nt * ob;
      info->staged_bytes = ps.staged_rows * nt * eb;
      for (int l = ps.l0 + 1; l <= ps.l1; ++l) info->adds += T.total[l] * nt;
      if (ps.from_input) info->adds += init_adds();
      break;
    }
    case fdmt::Step::MergeAdj:
      info->level_first = info->level_last = st.index;
      info->work_items = static_cast<int32_t>(T.total[st.index - 1]);
      info->bytes_read = T.total[st.index] * nt * 4;
      info->bytes_written = T.total[st.index - 1] * nt * 4;
      info->staged_bytes = 2 * T.total[st.index] * nt * 4;
      info->adds = (T.total[st.index] * 2 - T.total[st.index - 1]) * nt;
      break;
    case fdmt::Step::AdjGather: {
      const fdmt::AdjPass &ps = P.adj.passes[st.index];
      info->kind = 8;
      info->level_first = ps.to_input ? 0 : ps.l_lo + 1;
      info->level_last = ps.l_hi;
      const int rows = fdmt::adjoint_rows(P, st.index);
      const int64_t tile = fdmt::step_tile(P, true, step);
      info->work_items = static_cast<int32_t>(((ps.nrows + rows - 1) / rows) * ((nt + tile - 1) / tile));
      info->bytes_read = T.total[ps.l_hi] * nt * 4;
      info->bytes_written = static_cast<int64_t>(ps.nrows) * nt * 4;
      info->staged_bytes = ps.leaves * nt * 4;
      info->adds = ps.leaves * nt;
      break;
    }
    case fdmt::Step::InitAdj:
      info->level_first = info->level_last = 0;
      info->work_items = T.nf;
      info->bytes_read = T.total[0] * nt * 4;
      info->bytes_written = static_cast<int64_t>(T.nf) * nt * 4;
      info->staged_bytes = info->bytes_read;
      for (int k = 0; k < T.nf; ++k)
        info->adds += (static_cast<int64_t>(T.leaf_rows[k]) * (T.leaf_rows[k] + 1) / 2 - 1) * nt;
      break;
  }
  return FDMT_OK;
}

fdmt_status_t fdmt_run_step(fdmt_plan_t p, int32_t adjoint, int32_t step, const void *in, void *out,
                            int32_t batch, void *ws, size_t ws_bytes, void *hip_stream) {
  fdmt_status_t s = check_call(p, in, out, batch, ws, ws_bytes);
  if (s != FDMT_OK) return s;
  const auto &steps = adjoint ? p->plan.adj_steps : p->plan.fwd_steps;
  if (step < 0 || step >= static_cast<int32_t>(steps.size()))
    return fail(FDMT_E_INVALID, "step out of range");
  hipError_t e = fdmt::run_step(p->plan, adjoint != 0, step, in, out, batch, ws,
                                static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return device_fail(e, "fdmt_run_step launch");
  return FDMT_OK;
}

fdmt_status_t fdmt_plan_tables(fdmt_plan_t p, int32_t level, int32_t sub, int32_t *d_lo, int32_t *s,
                               int32_t *d_hi, int32_t cap, int32_t *n_rows) {
  if (!p || !n_rows) return fail(FDMT_E_INVALID, "plan or n_rows is NULL");
  const fdmt::Tables &T = p->plan.tab;
  if (level < 0 || level > T.levels) return fail(FDMT_E_INVALID, "level out of range");
  if (sub < 0 || sub >= (T.slots >> level)) return fail(FDMT_E_INVALID, "sub-band out of range");
  // positions without channels keep one zero row internally; reported as none
  const bool empty = (static_cast<int64_t>(sub) << level) >= T.nf;
  const bool copy = level > 0 && (static_cast<int64_t>(2 * sub + 1) << (level - 1)) >= T.nf;
  const int32_t n = empty ? 0 : T.rows[level][sub];
  *n_rows = n;
  if (level == 0 || cap <= 0) return FDMT_OK;
  if (cap < n) return fail(FDMT_E_INVALID, "cap smaller than the row count");
  if (!d_lo || !s || !d_hi) return fail(FDMT_E_INVALID, "table pointer is NULL");
  const int64_t base = T.row_off[level][sub];
  for (int32_t dt = 0; dt < n; ++dt) {
    d_lo[dt] = T.d_lo[level][base + dt];
    s[dt] = copy ? 0 : T.shift[level][base + dt];
    d_hi[dt] = copy ? -1 : T.d_hi[level][base + dt];
  }
  return FDMT_OK;
}

fdmt_status_t fdmt_plan_info(fdmt_plan_t p, int32_t *levels, int64_t *rows_per_level, int32_t cap) {
  if (!p || !levels) return fail(FDMT_E_INVALID, "plan or levels is NULL");
  const fdmt::Tables &T = p->plan.tab;
  *levels = T.levels;
  if (rows_per_level && cap > T.levels)
    for (int l = 0; l <= T.levels; ++l) rows_per_level[l] = T.total[l];
  return FDMT_OK;
}

fdmt_status_t fdmt_plan_destroy(fdmt_plan_t p) {
  if (!p) return FDMT_OK;
  fdmt_status_t s = FDMT_OK;
  fdmt::fft_destroy(p->plan);
  if (p->plan.dbuf) {
    hipError_t e = hipFree(p->plan.dbuf);
    if (e != hipSuccess) s = device_fail(e, "hipFree of delay tables");
  }
  delete p;
  return s;
}

fdmt_status_t fdmt_ragged_plan(fdmt_ragged_t *out, fdmt_plan_t p, int32_t nbeams, const int64_t *nt) {
  if (!out) return fail(FDMT_E_INVALID, "out is NULL");
  *out = nullptr;
  if (!p) return fail(FDMT_E_INVALID, "plan is NULL");
  if (!nt) return fail(FDMT_E_INVALID, "nt is NULL");
  if (nbeams < 1) return fail(FDMT_E_INVALID, "nbeams must be at least 1");
  const fdmt::Plan &P = p->plan;
  int64_t sum = 0, sump = 0;
  for (int32_t b = 0; b < nbeams; ++b) {
    if (nt[b] < 0 || nt[b] > INT32_MAX)
      return fail(FDMT_E_INVALID, "beam " + std::to_string(b) + ": Nt must be in [0, 2^31 - 1]");
    sum += nt[b];
    sump += fdmt::round_up(nt[b], fdmt::kRowAlign);
    if (sump > INT32_MAX) return fail(FDMT_E_UNSUPPORTED, "total samples of the batch exceed 2^31 - 1");
  }
  // Tile widths of every step of both transforms.
  std::vector<int> widths;
  for (int adj = 0; adj < 2; ++adj) {
    const int n = static_cast<int>(adj ? P.adj_steps.size() : P.fwd_steps.size());
    for (int i = 0; i < n; ++i) {
      const int w = fdmt::step_tile(P, adj != 0, i);
      if (w <= 0) return fail(FDMT_E_UNSUPPORTED, "the plan's staged-gather passes have no ragged form");
      if (std::find(widths.begin(), widths.end(), w) == widths.end()) widths.push_back(w);
    }
  }
  if (P.flags & FDMT_PLAN_HOST_ONLY)
    return fail(FDMT_E_UNSUPPORTED, "plan was built with FDMT_PLAN_HOST_ONLY");
  auto *h = new (std::nothrow) fdmt_ragged_s;
  if (!h) return fail(FDMT_E_NOMEM, "host allocation of the ragged plan failed");
  std::vector<int4> beams(nbeams);
  std::vector<std::vector<int2>> maps(widths.size());
  try {
    int64_t off = 0, poff = 0;
    for (int32_t b = 0; b < nbeams; ++b) {
      const int64_t ntp = fdmt::round_up(nt[b], fdmt::kRowAlign);
      beams[b] = make_int4(static_cast<int>(nt[b]), static_cast<int>(ntp), static_cast<int>(off),
                           static_cast<int>(poff));
      off += nt[b];
      poff += ntp;
      for (size_t m = 0; m < widths.size(); ++m)
        for (int64_t j = 0; j * widths[m] < nt[b]; ++j) maps[m].push_back(make_int2(b, static_cast<int>(j)));
    }
  } catch (const std::bad_alloc &) {
    delete h;
    return fail(FDMT_E_NOMEM, "host allocation of the tile maps failed");
  }
  size_t bytes = fdmt::round_up(static_cast<int64_t>(beams.size() * sizeof(int4)), 256);
  std::vector<size_t> map_off(widths.size());
  for (size_t m = 0; m < widths.size(); ++m) {
    map_off[m] = bytes;
    bytes += fdmt::round_up(static_cast<int64_t>(std::max<size_t>(1, maps[m].size()) * sizeof(int2)), 256);
  }
  std::vector<unsigned char> host(bytes, 0);
  std::memcpy(host.data(), beams.data(), beams.size() * sizeof(int4));
  for (size_t m = 0; m < widths.size(); ++m)
    if (!maps[m].empty()) std::memcpy(host.data() + map_off[m], maps[m].data(), maps[m].size() * sizeof(int2));
  hipError_t e = hipGetDevice(&h->device);
  if (e != hipSuccess) {
    delete h;
    return device_fail(e, "hipGetDevice");
  }
  if (h->device != P.device) {
    delete h;
    return fail(FDMT_E_INVALID, "current device differs from the plan's device");
  }
  e = hipMalloc(&h->dbuf, bytes);
  if (e != hipSuccess) {
    delete h;
    return fail(FDMT_E_NOMEM, std::string("hipMalloc of the tile maps: ") + hipGetErrorString(e));
  }
  e = hipMemcpy(h->dbuf, host.data(), bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    (void)hipFree(h->dbuf);
    delete h;
    return device_fail(e, "hipMemcpy of the tile maps");
  }
  auto *base = static_cast<unsigned char *>(h->dbuf);
  h->plan = p;
  h->rb.nbeams = nbeams;
  h->rb.sum_nt = sum;
  h->rb.sum_ntp = sump;
  h->rb.beam = reinterpret_cast<const int4 *>(base);
  for (size_t m = 0; m < widths.size(); ++m)
    h->rb.maps.push_back({widths[m], static_cast<int64_t>(maps[m].size()),
                          reinterpret_cast<const int2 *>(base + map_off[m])});
  *out = h;
  return FDMT_OK;
}

size_t fdmt_ragged_workspace_bytes(fdmt_ragged_t r) {
  if (!r) return 0;
  return fdmt::ragged_workspace_bytes(r->plan->plan, r->rb);
}

fdmt_status_t fdmt_ragged_forward(fdmt_ragged_t r, const void *in, void *out, void *ws, size_t ws_bytes,
                                  void *hip_stream) {
  fdmt_status_t s = check_ragged(r, in, out, ws, ws_bytes);
  if (s != FDMT_OK) return s;
  hipError_t e = fdmt::launch_forward(r->plan->plan, in, out, 1, ws, static_cast<hipStream_t>(hip_stream), &r->rb);
  if (e != hipSuccess) return device_fail(e, "fdmt_ragged_forward launch");
  return FDMT_OK;
}

fdmt_status_t fdmt_ragged_adjoint(fdmt_ragged_t r, const void *grad_out, void *grad_in, void *ws,
                                  size_t ws_bytes, void *hip_stream) {
  fdmt_status_t s = check_ragged(r, grad_out, grad_in, ws, ws_bytes);
  if (s != FDMT_OK) return s;
  hipError_t e = fdmt::launch_adjoint(r->plan->plan, grad_out, grad_in, 1, ws, static_cast<hipStream_t>(hip_stream), &r->rb);
  if (e != hipSuccess) return device_fail(e, "fdmt_ragged_adjoint launch");
  return FDMT_OK;
}

fdmt_status_t fdmt_ragged_run_step(fdmt_ragged_t r, int32_t adjoint, int32_t step, const void *in, void *out,
                                   void *ws, size_t ws_bytes, void *hip_stream) {
  fdmt_status_t s = check_ragged(r, in, out, ws, ws_bytes);
  if (s != FDMT_OK) return s;
  const fdmt::Plan &P = r->plan->plan;
  const auto &steps = adjoint ? P.adj_steps : P.fwd_steps;
  if (step < 0 || step >= static_cast<int32_t>(steps.size()))
    return fail(FDMT_E_INVALID, "step out of range");
  hipError_t e = fdmt::run_step(P, adjoint != 0, step, in, out, 1, ws, static_cast<hipStream_t>(hip_stream), &r->rb);
  if (e != hipSuccess) return device_fail(e, "fdmt_ragged_run_step launch");
  return FDMT_OK;
}

fdmt_status_t fdmt_ragged_info(fdmt_ragged_t r, int32_t *nbeams, int64_t *total_nt, int32_t *launches) {
  if (!r) return fail(FDMT_E_INVALID, "ragged plan is NULL");
  if (nbeams) *nbeams = r->rb.nbeams;
  if (total_nt) *total_nt = r->rb.sum_nt;
  if (launches) {
    const fdmt::Plan &P = r->plan->plan;
    int32_t n = 0;
    for (int adj = 0; adj < 2; ++adj) {
      const int k = static_cast<int>(adj ? P.adj_steps.size() : P.fwd_steps.size());
      for (int i = 0; i < k; ++i) {
        const int w = fdmt::step_tile(P, adj != 0, i);
        for (const fdmt::RaggedBatch::Map &m : r->rb.maps)
          if (m.tile == w) n += static_cast<int32_t>((m.count + 65534) / 65535);
      }
    }
    *launches = n;
  }
  return FDMT_OK;
}

fdmt_status_t fdmt_ragged_destroy(fdmt_ragged_t r) {
  if (!r) return FDMT_OK;
  fdmt_status_t s = FDMT_OK;
  if (r->dbuf) {
    hipError_t e = hipFree(r->dbuf);
    if (e != hipSuccess) s = device_fail(e, "hipFree of the tile maps");
  }
  delete r;
  return s;
}

namespace {

bool boxcar_sizes_ok(int32_t batch, int32_t nd, int64_t nt, int32_t max_log2) {
  return batch >= 1 && batch <= 65535 && nd >= 1 && nd <= 65535 && nt >= 1 && nt <= INT32_MAX && max_log2 >= 0 &&
         max_log2 <= fdmt::kBoxMaxLog2;
}

} // namespace

size_t fdmt_boxcar_workspace_bytes(int32_t batch, int32_t nd, int64_t nt, int32_t max_log2) {
  return boxcar_sizes_ok(batch, nd, nt, max_log2) ? fdmt::boxcar_workspace_bytes(batch, nd, nt, max_log2) : 0;
}

fdmt_status_t fdmt_boxcar_search(const float *plane, int32_t batch, int32_t nd, int64_t nt, int32_t max_log2,
                                 fdmt_boxcar_t *out, void *ws, size_t ws_bytes, void *hip_stream) {
  if (!plane || !out || !ws) return fail(FDMT_E_INVALID, "plane, out or workspace is NULL");
  if (!boxcar_sizes_ok(batch, nd, nt, max_log2))
    return fail(FDMT_E_INVALID, "need batch, nd in [1, 65535], nt in [1, 2^31 - 1], max_log2 in [0, 10]");
  const size_t need = fdmt::boxcar_workspace_bytes(batch, nd, nt, max_log2);
  if (ws_bytes < need)
    return fail(FDMT_E_WORKSPACE, "boxcar workspace needs " + std::to_string(need) + " bytes, got " +
                                      std::to_string(ws_bytes));
  const hipError_t e =
      fdmt::launch_boxcar(plane, batch, nd, nt, max_log2, out, ws, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return device_fail(e, "boxcar search launch");
  return FDMT_OK;
}

size_t fdmt_search_workspace_bytes(fdmt_plan_t p, int32_t batch, int32_t max_log2) {
  if (!p || batch < 1 || batch > 65535 || max_log2 < 0 || max_log2 > fdmt::kBoxMaxLog2) return 0;
  const fdmt::Plan &P = p->plan;
  const size_t fwd = fdmt::round_up(static_cast<int64_t>(fdmt::workspace_bytes(P, batch)), 256);
  const size_t part = fdmt::round_up(
      static_cast<int64_t>(fdmt::boxcar_workspace_bytes(batch, P.tab.nd, P.nt, max_log2)), 256);
  return fwd + part + static_cast<size_t>(batch) * (max_log2 + 1) * P.tab.nd * sizeof(double2);
}

int32_t fdmt_search_fused(fdmt_plan_t p, int32_t max_log2) {
  return p && fdmt::search_fusable(p->plan, max_log2) ? 1 : 0;
}

fdmt_status_t fdmt_forward_search(fdmt_plan_t p, const void *in, void *out, int32_t batch, int32_t max_log2,
                                  float threshold, fdmt_boxcar_t *stats, fdmt_candidate_t *cands, int32_t cap,
                                  int32_t *count, void *ws, size_t ws_bytes, void *hip_stream) {
  if (!p) return fail(FDMT_E_INVALID, "plan is NULL");
  if (p->plan.acc_dtype != FDMT_F32) return fail(FDMT_E_UNSUPPORTED, "the search reads an FP32 output plane");
  if (max_log2 < 0 || max_log2 > fdmt::kBoxMaxLog2) return fail(FDMT_E_INVALID, "max_log2 must be in [0, 10]");
  if (!stats || !count || cap < 0 || (cap > 0 && !cands))
    return fail(FDMT_E_INVALID, "stats or count is NULL, cap < 0, or cands NULL with cap > 0");
  if (!(threshold == threshold)) return fail(FDMT_E_INVALID, "threshold is NaN");
  const size_t need = fdmt_search_workspace_bytes(p, batch, max_log2);
  if (need == 0) return fail(FDMT_E_INVALID, "batch must be in [1, 65535]");
  if (!ws || ws_bytes < need)
    return fail(FDMT_E_WORKSPACE, "search workspace needs " + std::to_string(need) + " bytes, got " +
                                      std::to_string(ws ? ws_bytes : 0));
  const fdmt_status_t st = check_call(p, in, out, batch, ws, ws_bytes);
  if (st != FDMT_OK) return st;
  const fdmt::Plan &P = p->plan;
  auto *base = static_cast<unsigned char *>(ws);
  const size_t fwd = fdmt::round_up(static_cast<int64_t>(fdmt::workspace_bytes(P, batch)), 256);
  const size_t partb = fdmt::round_up(
      static_cast<int64_t>(fdmt::boxcar_workspace_bytes(batch, P.tab.nd, P.nt, max_log2)), 256);
  auto *part = reinterpret_cast<fdmt::BoxPartial *>(base + fwd);
  auto *mean_sd = reinterpret_cast<double2 *>(base + fwd + partb);
  auto stream = static_cast<hipStream_t>(hip_stream);
  float *plane = static_cast<float *>(out);
  hipError_t e;
  if (fdmt::search_fusable(P, max_log2)) {
    e = fdmt::launch_forward_search(P, in, plane, batch, ws, part, max_log2, stream);
  } else {
    e = fdmt::launch_forward(P, in, out, batch, ws, stream);
    if (e == hipSuccess) e = fdmt::launch_boxcar_tiles(plane, batch, P.tab.nd, P.nt, max_log2, part, stream);
  }
  if (e == hipSuccess) e = fdmt::launch_boxcar_combine(part, batch, P.tab.nd, P.nt, max_log2, stats, mean_sd, stream);
  if (e == hipSuccess)
    e = fdmt::launch_boxcar_candidates(part, mean_sd, batch, P.tab.nd, P.nt, max_log2, threshold, cands, cap, count,
                                       stream);
  if (e != hipSuccess) return device_fail(e, "forward search launch");
  return FDMT_OK;
}

fdmt_status_t fdmt_boxcar_search_noalloc(const float *plane, int32_t batch, int32_t nd, int64_t nt,
                                         int32_t max_log2, fdmt_boxcar_t *out, void *hip_stream) {
  if (!plane || !out) return fail(FDMT_E_INVALID, "plane or out is NULL");
  if (!boxcar_sizes_ok(batch, nd, nt, max_log2))
    return fail(FDMT_E_INVALID, "need batch, nd in [1, 65535], nt in [1, 2^31 - 1], max_log2 in [0, 10]");
  const size_t need = fdmt::boxcar_workspace_bytes(batch, nd, nt, max_log2);
  if (need > fdmt::kBoxScratchBytes)
    return fail(FDMT_E_WORKSPACE, "the search needs " + std::to_string(need) + " bytes of scratch, more than the " +
                                      std::to_string(fdmt::kBoxScratchBytes) +
                                      " of the static buffer: use fdmt_boxcar_search with a workspace");
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return device_fail(e, "hipGetDevice");
  void *ws = nullptr;
  e = fdmt::boxcar_static_scratch(dev, &ws);
  if (e != hipSuccess) return device_fail(e, "static boxcar scratch");
  e = fdmt::launch_boxcar(plane, batch, nd, nt, max_log2, out, ws, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return device_fail(e, "boxcar search launch");
  return FDMT_OK;
}

fdmt_status_t fdmt_copy_bytes(void *dst, const void *src, size_t bytes, void *hip_stream) {
  if (bytes == 0) return FDMT_OK;
  if (!dst || !src) return fail(FDMT_E_INVALID, "src or dst is NULL");
  if (((reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src)) & 15u) != 0)
    return fail(FDMT_E_INVALID, "src and dst must be 16-byte aligned");
  const uintptr_t d = reinterpret_cast<uintptr_t>(dst), s = reinterpret_cast<uintptr_t>(src);
  if (d < s + bytes && s < d + bytes) return fail(FDMT_E_INVALID, "src and dst overlap");
  const hipError_t e = fdmt::launch_stream_copy(dst, src, bytes, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return device_fail(e, "stream copy launch");
  return FDMT_OK;
}

fdmt_status_t fdmt_stream_mix(void *dst, size_t write_bytes, const void *src, size_t read_bytes,
                              void *hip_stream) {
  if (write_bytes == 0 && read_bytes == 0) return FDMT_OK;
  if (!dst || !src) return fail(FDMT_E_INVALID, "src or dst is NULL");
  if (((reinterpret_cast<uintptr_t>(dst) | reinterpret_cast<uintptr_t>(src)) & 15u) != 0)
    return fail(FDMT_E_INVALID, "src and dst must be 16-byte aligned");
  if ((write_bytes | read_bytes) & 15u) return fail(FDMT_E_INVALID, "byte counts must be multiples of 16");
  if (write_bytes == 0 || read_bytes == 0 || write_bytes > 2 * read_bytes || read_bytes > 2 * write_bytes)
    return fail(FDMT_E_INVALID, "each byte count must be at least half the other");
  const uintptr_t d = reinterpret_cast<uintptr_t>(dst), s = reinterpret_cast<uintptr_t>(src);
  if (d < s + read_bytes && s < d + write_bytes) return fail(FDMT_E_INVALID, "src and dst overlap");
  const hipError_t e =
      fdmt::launch_stream_mix(dst, write_bytes, src, read_bytes, static_cast<hipStream_t>(hip_stream));
  if (e != hipSuccess) return device_fail(e, "stream mix launch");
  return FDMT_OK;
}

fdmt_status_t fdmt_tuned_options(const char *cache_path, const char *arch, int32_t nf, int64_t nt, int32_t nd,
                                 double f_min, double f_max, fdmt_options_t *opt, int32_t *found) {
  if (found) *found = 0;
  if (!opt) return fail(FDMT_E_INVALID, "opt is NULL");
  if (nf < 1 || nt < 1 || nd < 1) return fail(FDMT_E_INVALID, "Nf, Nt and Nd must be >= 1");
  std::string a;
  if (arch) {
    a = arch;
  } else {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return device_fail(e, "hipGetDevice");
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return device_fail(e, "hipGetDeviceProperties");
    a = prop.gcnArchName;
  }
  a = a.substr(0, a.find(':'));  // "gfx950:sramecc+:xnack-" -> "gfx950"
  std::string path;
  if (cache_path) {
    path = cache_path;
  } else if (const char *env = std::getenv("FDMT_TUNE_CACHE"); env && *env) {
    path = env;
  } else {
    // the cache shipped beside the library: <directory of libfdmt.so>/tuning/<arch>.json
    Dl_info info;
    if (!dladdr(reinterpret_cast<void *>(&fdmt_tuned_options), &info) || !info.dli_fname)
      return fail(FDMT_E_INVALID, "cannot locate the library to find its tuning cache");
    std::string lib = info.dli_fname;
    const size_t slash = lib.rfind('/');
    path = (slash == std::string::npos ? std::string(".") : lib.substr(0, slash)) + "/tuning/" + a + ".json";
  }
  const double gamma = opt->gamma != 0.0 ? opt->gamma : -2.0;
  const std::string key =
      fdmt::tune_key(a, nf, nt, nd, f_min, f_max, opt->in_dtype, opt->acc_dtype, gamma, opt->rule);
  std::map<std::string, double> o;
  bool hit = false;
  std::string err;
  try {
    err = fdmt::tune_lookup(path, key, o, hit);
  } catch (const std::bad_alloc &) {
    return fail(FDMT_E_NOMEM, "host allocation while reading the tuning cache");
  }
  if (!err.empty()) return fail(FDMT_E_INVALID, "tuning cache: " + err);
  if (!hit) return FDMT_OK;
  struct Field {
    const char *name;
    int32_t *i;
    uint32_t *u;
  };
  const Field fields[] = {{"first_levels", &opt->first_levels, nullptr},
                          {"later_levels", &opt->later_levels, nullptr},
                          {"tile", &opt->tile, nullptr},
                          {"lds_kib", &opt->lds_kib, nullptr},
                          {"max_block_rows", &opt->max_block_rows, nullptr},
                          {"first_kernel", &opt->first_kernel, nullptr},
                          {"later_kernel", &opt->later_kernel, nullptr},
                          {"stream_tiles", &opt->stream_tiles, nullptr},
                          {"gather_rows", &opt->gather_rows, nullptr},
                          {"adjoint_levels", &opt->adjoint_levels, nullptr},
                          {"adjoint_last_levels", &opt->adjoint_last_levels, nullptr},
                          {"gather_vecs", &opt->gather_vecs, nullptr},
                          {"adjoint_last_rows", &opt->adjoint_last_rows, nullptr},
                          {"adjoint_tile_major", nullptr, &opt->adjoint_tile_major},
                          {"gather_threads", &opt->gather_threads, nullptr},
                          {"adjoint_threads", &opt->adjoint_threads, nullptr},
                          {"adjoint_last_threads", &opt->adjoint_last_threads, nullptr},
                          {"search_rows", &opt->search_rows, nullptr},
                          {"first_rows", &opt->first_rows, nullptr},
                          {"first_threads", &opt->first_threads, nullptr},
                          {"adjoint_rows", &opt->adjoint_rows, nullptr}};
  for (const auto &kv : o) {
    const Field *f = nullptr;
    for (const Field &c : fields)
      if (kv.first == c.name) f = &c;
    if (!f) return fail(FDMT_E_INVALID, "tuning cache entry " + key + ": unknown schedule field " + kv.first);
    const double v = kv.second;
    if (!(v >= 0.0 && v <= 4294967295.0 && v == std::floor(v)))
      return fail(FDMT_E_INVALID, "tuning cache entry " + key + ": bad value of " + kv.first);
    // explicit (nonzero) fields of the caller win over the cache
    if (f->i && *f->i == 0) *f->i = static_cast<int32_t>(v);
    if (f->u && *f->u == 0) *f->u = static_cast<uint32_t>(v);
  }
  // the d_min pre-shift rides on the input terms: keep a gather from the input
  if (opt->d_min > 0 && (opt->first_kernel == 1 || opt->first_kernel == 2)) opt->first_kernel = 3;
  if (found) *found = 1;
  return FDMT_OK;
}

const char *fdmt_status_string(fdmt_status_t s) {
  switch (s) {
    case FDMT_OK: return "ok";
    case FDMT_E_INVALID: return "invalid argument";
    case FDMT_E_UNSUPPORTED: return "unsupported request";
    case FDMT_E_NOMEM: return "out of memory";
    case FDMT_E_DEVICE: return "device error";
    case FDMT_E_WORKSPACE: return "workspace missing or too small";
  }
  return "unknown status";
}

const char *fdmt_last_error(void) { return g_last_error.c_str(); }

} // extern "C"
