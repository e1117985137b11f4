"""Python binding of libfdmt.so (argument marshalling only).

Every step of the transform runs in the HIP library; PyTorch supplies device
memory (tensors, the workspace) and the current HIP stream. The functions
carry the C ABI's names; `Plan` and `FDMTFunction` are thin tensor-level
conveniences over them. If the library is not built this module raises on
first use: there is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

import torch  # imported first so the library binds to torch's HIP runtime

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libfdmt.so")
_lib = None

FDMT_OK, FDMT_E_INVALID, FDMT_E_UNSUPPORTED, FDMT_E_NOMEM, FDMT_E_DEVICE, FDMT_E_WORKSPACE = range(6)
FDMT_F32, FDMT_F16, FDMT_U8, FDMT_I32 = range(4)
FDMT_PLAN_HOST_ONLY = 0x1
FDMT_PLAN_UNFUSED = 0x2
FDMT_PLAN_WIDE_PLANES = 0x4
FDMT_PLAN_FFT = 0x8

EXPORTED = ("fdmt_plan", "fdmt_workspace_bytes", "fdmt_forward", "fdmt_adjoint",
            "fdmt_step_count", "fdmt_step_info", "fdmt_run_step",
            "fdmt_plan_tables", "fdmt_plan_info", "fdmt_plan_destroy",
            "fdmt_ragged_plan", "fdmt_ragged_workspace_bytes", "fdmt_ragged_forward",
            "fdmt_ragged_adjoint", "fdmt_ragged_run_step", "fdmt_ragged_info",
            "fdmt_ragged_destroy", "fdmt_boxcar_workspace_bytes", "fdmt_boxcar_search",
            "fdmt_fft_workspace_bytes", "fdmt_forward_fft", "fdmt_search_workspace_bytes", "fdmt_search_fused", "fdmt_forward_search",
            "fdmt_boxcar_search_noalloc", "fdmt_copy_bytes", "fdmt_stream_mix", "fdmt_tuned_options",
            "fdmt_status_string",
            "fdmt_last_error")

STEP_KINDS = ("init", "iteration", "lds_levels", "iteration_adjoint", "init_adjoint", "gather",
              "input_gather", "staged_gather", "adjoint_gather", "pad_input")

_TORCH_TO_CODE = {torch.float32: FDMT_F32, torch.float16: FDMT_F16,
                  torch.uint8: FDMT_U8, torch.int32: FDMT_I32}
_CODE_TO_TORCH = {v: k for k, v in _TORCH_TO_CODE.items()}


class FDMTError(RuntimeError):
    def __init__(self, status, message):
        super().__init__(message)
        self.status = status


class _Options(ctypes.Structure):
    _fields_ = [("in_dtype", ctypes.c_int32), ("acc_dtype", ctypes.c_int32),
                ("flags", ctypes.c_uint32), ("first_levels", ctypes.c_int32),
                ("later_levels", ctypes.c_int32), ("tile", ctypes.c_int32),
                ("lds_kib", ctypes.c_int32), ("max_block_rows", ctypes.c_int32),
                ("first_kernel", ctypes.c_int32), ("later_kernel", ctypes.c_int32),
                ("stream_tiles", ctypes.c_int32), ("gather_rows", ctypes.c_int32),
                ("adjoint_levels", ctypes.c_int32), ("adjoint_last_levels", ctypes.c_int32),
                ("gather_vecs", ctypes.c_int32), ("adjoint_last_rows", ctypes.c_int32),
                ("gamma", ctypes.c_double), ("d_min", ctypes.c_int32),
                ("adjoint_tile_major", ctypes.c_uint32), ("gather_threads", ctypes.c_int32),
                ("adjoint_threads", ctypes.c_int32), ("adjoint_last_threads", ctypes.c_int32),
                ("rule", ctypes.c_int32), ("search_rows", ctypes.c_int32),
                ("first_rows", ctypes.c_int32), ("first_threads", ctypes.c_int32),
                ("adjoint_rows", ctypes.c_int32)]


class _StepInfo(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("level_first", ctypes.c_int32),
                ("level_last", ctypes.c_int32), ("work_items", ctypes.c_int32),
                ("lds_bytes", ctypes.c_int64), ("bytes_read", ctypes.c_int64),
                ("bytes_written", ctypes.c_int64), ("staged_bytes", ctypes.c_int64),
                ("adds", ctypes.c_int64), ("in_elem_bytes", ctypes.c_int32),
                ("out_elem_bytes", ctypes.c_int32)]


def library_path():
    return _LIB_PATH


def load():
    """Load libfdmt.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is missing: build it with python paper_1411_5373_amd/build.py; "
                          "there is no fallback path")
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i32, i64, sz = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    p_i32 = ctypes.POINTER(ctypes.c_int32)
    lib.fdmt_plan.argtypes = [ctypes.POINTER(vp), i32, i64, i32, ctypes.c_double, ctypes.c_double,
                              ctypes.POINTER(_Options)]
    lib.fdmt_plan.restype = ctypes.c_int
    lib.fdmt_workspace_bytes.argtypes = [vp, i32]
    lib.fdmt_workspace_bytes.restype = sz
    for name in ("fdmt_forward", "fdmt_adjoint"):
        f = getattr(lib, name)
        f.argtypes = [vp, vp, vp, i32, vp, sz, vp]
        f.restype = ctypes.c_int
    lib.fdmt_step_count.argtypes = [vp, i32]
    lib.fdmt_step_count.restype = ctypes.c_int32
    lib.fdmt_step_info.argtypes = [vp, i32, i32, ctypes.POINTER(_StepInfo)]
    lib.fdmt_step_info.restype = ctypes.c_int
    lib.fdmt_run_step.argtypes = [vp, i32, i32, vp, vp, i32, vp, sz, vp]
    lib.fdmt_run_step.restype = ctypes.c_int
    lib.fdmt_plan_tables.argtypes = [vp, i32, i32, p_i32, p_i32, p_i32, i32, p_i32]
    lib.fdmt_plan_tables.restype = ctypes.c_int
    lib.fdmt_plan_info.argtypes = [vp, p_i32, ctypes.POINTER(ctypes.c_int64), i32]
    lib.fdmt_plan_info.restype = ctypes.c_int
    lib.fdmt_plan_destroy.argtypes = [vp]
    lib.fdmt_plan_destroy.restype = ctypes.c_int
    lib.fdmt_ragged_plan.argtypes = [ctypes.POINTER(vp), vp, i32, ctypes.POINTER(ctypes.c_int64)]
    lib.fdmt_ragged_plan.restype = ctypes.c_int
    lib.fdmt_ragged_workspace_bytes.argtypes = [vp]
    lib.fdmt_ragged_workspace_bytes.restype = sz
    for name in ("fdmt_ragged_forward", "fdmt_ragged_adjoint"):
        f = getattr(lib, name)
        f.argtypes = [vp, vp, vp, vp, sz, vp]
        f.restype = ctypes.c_int
    lib.fdmt_ragged_run_step.argtypes = [vp, i32, i32, vp, vp, vp, sz, vp]
    lib.fdmt_ragged_run_step.restype = ctypes.c_int
    lib.fdmt_ragged_info.argtypes = [vp, p_i32, ctypes.POINTER(ctypes.c_int64), p_i32]
    lib.fdmt_ragged_info.restype = ctypes.c_int
    lib.fdmt_ragged_destroy.argtypes = [vp]
    lib.fdmt_ragged_destroy.restype = ctypes.c_int
    lib.fdmt_fft_workspace_bytes.argtypes = [vp, i32]
    lib.fdmt_fft_workspace_bytes.restype = sz
    lib.fdmt_forward_fft.argtypes = [vp, vp, vp, i32, vp, sz, vp]
    lib.fdmt_forward_fft.restype = ctypes.c_int
    lib.fdmt_boxcar_workspace_bytes.argtypes = [i32, i32, i64, i32]
    lib.fdmt_boxcar_workspace_bytes.restype = sz
    lib.fdmt_boxcar_search.argtypes = [vp, i32, i32, i64, i32, vp, vp, sz, vp]
    lib.fdmt_boxcar_search.restype = ctypes.c_int
    lib.fdmt_search_workspace_bytes.argtypes = [vp, i32, i32]
    lib.fdmt_search_workspace_bytes.restype = sz
    lib.fdmt_search_fused.argtypes = [vp, i32]
    lib.fdmt_search_fused.restype = ctypes.c_int32
    lib.fdmt_forward_search.argtypes = [vp, vp, vp, i32, i32, ctypes.c_float, vp, vp, i32, vp, vp, sz, vp]
    lib.fdmt_forward_search.restype = ctypes.c_int
    lib.fdmt_boxcar_search_noalloc.argtypes = [vp, i32, i32, i64, i32, vp, vp]
    lib.fdmt_boxcar_search_noalloc.restype = ctypes.c_int
    lib.fdmt_copy_bytes.argtypes = [vp, vp, sz, vp]
    lib.fdmt_copy_bytes.restype = ctypes.c_int
    lib.fdmt_stream_mix.argtypes = [vp, sz, vp, sz, vp]
    lib.fdmt_stream_mix.restype = ctypes.c_int
    lib.fdmt_tuned_options.argtypes = [ctypes.c_char_p, ctypes.c_char_p, i32, i64, i32, ctypes.c_double,
                                       ctypes.c_double, ctypes.POINTER(_Options), p_i32]
    lib.fdmt_tuned_options.restype = ctypes.c_int
    lib.fdmt_status_string.argtypes = [ctypes.c_int]
    lib.fdmt_status_string.restype = ctypes.c_char_p
    lib.fdmt_last_error.argtypes = []
    lib.fdmt_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _check(status, what):
    if status != FDMT_OK:
        lib = load()
        raise FDMTError(status, f"{what}: {lib.fdmt_status_string(status).decode()}: "
                                f"{lib.fdmt_last_error().decode()}")


# ----------------------------------------------------------------- C ABI names

def fdmt_status_string(status):
    return load().fdmt_status_string(int(status)).decode()


def fdmt_last_error():
    return load().fdmt_last_error().decode()


def fdmt_plan(nf, nt, nd, f_min, f_max, in_dtype=FDMT_F32, acc_dtype=FDMT_F32, flags=0,
              first_levels=0, later_levels=0, tile=0, lds_kib=0, max_block_rows=0,
              first_kernel=0, later_kernel=0, stream_tiles=0, gather_rows=0, adjoint_levels=0,
              adjoint_last_levels=0, gather_vecs=0, adjoint_last_rows=0, gamma=0.0, d_min=0,
              adjoint_tile_major=0, gather_threads=0, adjoint_threads=0, adjoint_last_threads=0, rule=0,
              search_rows=0, first_rows=0, first_threads=0, adjoint_rows=0):
    """Returns an opaque plan handle (int); raises FDMTError on failure."""
    h = ctypes.c_void_p()
    opt = _Options(int(in_dtype), int(acc_dtype), int(flags), int(first_levels),
                   int(later_levels), int(tile), int(lds_kib), int(max_block_rows),
                   int(first_kernel), int(later_kernel), int(stream_tiles), int(gather_rows),
                   int(adjoint_levels), int(adjoint_last_levels), int(gather_vecs),
                   int(adjoint_last_rows), float(gamma), int(d_min), int(adjoint_tile_major),
                   int(gather_threads), int(adjoint_threads), int(adjoint_last_threads), int(rule),
                   int(search_rows), int(first_rows), int(first_threads), int(adjoint_rows))
    _check(load().fdmt_plan(ctypes.byref(h), int(nf), int(nt), int(nd), float(f_min), float(f_max),
                            ctypes.byref(opt)), "fdmt_plan")
    return h.value


def fdmt_copy_bytes(dst_ptr, src_ptr, nbytes, stream):
    _check(load().fdmt_copy_bytes(dst_ptr, src_ptr, int(nbytes), stream), "fdmt_copy_bytes")


def copy_bytes(dst, src):
    """Streaming copy of src's bytes into dst (device tensors of equal byte
    size) with the library's copy kernel, on the current stream."""
    n = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != n or not (src.is_contiguous() and dst.is_contiguous()):
        raise ValueError("dst and src must be contiguous and of equal byte size")
    fdmt_copy_bytes(ctypes.c_void_p(dst.data_ptr()), ctypes.c_void_p(src.data_ptr()), n, _stream_handle(src.device))
    return dst


def fdmt_stream_mix(dst_ptr, write_bytes, src_ptr, read_bytes, stream):
    _check(load().fdmt_stream_mix(dst_ptr, int(write_bytes), src_ptr, int(read_bytes), stream), "fdmt_stream_mix")


def stream_mix(dst, src):
    """The library's read/write-mix stream: reads all of src's bytes once and
    writes all of dst's once (contiguous device tensors; each byte count a
    multiple of 16 and at most twice the other), on the current stream."""
    if not (src.is_contiguous() and dst.is_contiguous()):
        raise ValueError("dst and src must be contiguous")
    fdmt_stream_mix(ctypes.c_void_p(dst.data_ptr()), dst.numel() * dst.element_size(),
                    ctypes.c_void_p(src.data_ptr()), src.numel() * src.element_size(), _stream_handle(src.device))
    return dst


SCHEDULE_FIELDS = ("first_levels", "later_levels", "tile", "lds_kib", "max_block_rows", "first_kernel",
                   "later_kernel", "stream_tiles", "gather_rows", "adjoint_levels", "adjoint_last_levels",
                   "gather_vecs", "adjoint_last_rows", "adjoint_tile_major", "gather_threads", "adjoint_threads",
                   "adjoint_last_threads", "search_rows", "first_rows", "first_threads", "adjoint_rows")


def fdmt_tuned_options(nf, nt, nd, f_min, f_max, in_dtype=FDMT_F32, acc_dtype=FDMT_F32, gamma=0.0, d_min=0,
                       rule=0, cache_path=None, arch=None, **explicit):
    """The autotuner's schedule for this workload through the C ABI: a dict of
    the schedule fields the cache sets (explicit nonzero fields kept as given),
    or None when the cache has no entry."""
    opt = _Options(int(in_dtype), int(acc_dtype), 0, *([0] * 13), float(gamma), int(d_min), 0, 0, 0, 0, int(rule), 0,
                   0, 0, 0)
    for k, v in explicit.items():
        setattr(opt, k, int(v))
    found = ctypes.c_int32()
    _check(load().fdmt_tuned_options(None if cache_path is None else os.fsencode(cache_path),
                                     None if arch is None else arch.encode(), int(nf), int(nt), int(nd),
                                     float(f_min), float(f_max), ctypes.byref(opt), ctypes.byref(found)),
           "fdmt_tuned_options")
    if not found.value:
        return None
    return {k: getattr(opt, k) for k in SCHEDULE_FIELDS if getattr(opt, k) != 0}


def fdmt_workspace_bytes(plan, batch):
    return int(load().fdmt_workspace_bytes(plan, int(batch)))


def fdmt_forward(plan, in_ptr, out_ptr, batch, ws_ptr, ws_bytes, stream):
    _check(load().fdmt_forward(plan, in_ptr, out_ptr, int(batch), ws_ptr, int(ws_bytes), stream),
           "fdmt_forward")


def fdmt_adjoint(plan, grad_out_ptr, grad_in_ptr, batch, ws_ptr, ws_bytes, stream):
    _check(load().fdmt_adjoint(plan, grad_out_ptr, grad_in_ptr, int(batch), ws_ptr, int(ws_bytes),
                               stream), "fdmt_adjoint")


def fdmt_fft_workspace_bytes(plan, batch=1):
    return int(load().fdmt_fft_workspace_bytes(plan, int(batch)))


def fdmt_forward_fft(plan, in_ptr, out_ptr, batch, ws_ptr, ws_bytes, stream):
    _check(load().fdmt_forward_fft(plan, in_ptr, out_ptr, int(batch), ws_ptr, int(ws_bytes), stream),
           "fdmt_forward_fft")


def fdmt_boxcar_workspace_bytes(batch, nd, nt, max_log2):
    return int(load().fdmt_boxcar_workspace_bytes(int(batch), int(nd), int(nt), int(max_log2)))


def fdmt_boxcar_search(plane_ptr, batch, nd, nt, max_log2, out_ptr, ws_ptr, ws_bytes, stream):
    _check(load().fdmt_boxcar_search(plane_ptr, int(batch), int(nd), int(nt), int(max_log2), out_ptr, ws_ptr,
                                     int(ws_bytes), stream), "fdmt_boxcar_search")


def fdmt_search_workspace_bytes(plan, batch, max_log2):
    return int(load().fdmt_search_workspace_bytes(plan, int(batch), int(max_log2)))


def fdmt_search_fused(plan, max_log2):
    return bool(load().fdmt_search_fused(plan, int(max_log2)))


def fdmt_forward_search(plan, in_ptr, out_ptr, batch, max_log2, threshold, stats_ptr, cands_ptr, cap, count_ptr,
                        ws_ptr, ws_bytes, stream):
    _check(load().fdmt_forward_search(plan, in_ptr, out_ptr, int(batch), int(max_log2), float(threshold),
                                      stats_ptr, cands_ptr, int(cap), count_ptr, ws_ptr, int(ws_bytes), stream),
           "fdmt_forward_search")


def fdmt_boxcar_search_noalloc(plane_ptr, batch, nd, nt, max_log2, out_ptr, stream):
    _check(load().fdmt_boxcar_search_noalloc(plane_ptr, int(batch), int(nd), int(nt), int(max_log2), out_ptr,
                                             stream), "fdmt_boxcar_search_noalloc")


def fdmt_step_count(plan, adjoint=False):
    return int(load().fdmt_step_count(plan, int(bool(adjoint))))


def fdmt_step_info(plan, adjoint, step):
    info = _StepInfo()
    _check(load().fdmt_step_info(plan, int(bool(adjoint)), int(step), ctypes.byref(info)),
           "fdmt_step_info")
    d = {f: getattr(info, f) for f, _ in _StepInfo._fields_}
    d["kind"] = STEP_KINDS[d["kind"]]
    return d


def fdmt_run_step(plan, adjoint, step, in_ptr, out_ptr, batch, ws_ptr, ws_bytes, stream):
    _check(load().fdmt_run_step(plan, int(bool(adjoint)), int(step), in_ptr, out_ptr, int(batch),
                                ws_ptr, int(ws_bytes), stream), "fdmt_run_step")


def fdmt_plan_tables(plan, level, sub):
    """Returns (d_lo, s, d_hi) as lists (empty for level 0) and the row count."""
    n = ctypes.c_int32()
    _check(load().fdmt_plan_tables(plan, int(level), int(sub), None, None, None, 0, ctypes.byref(n)),
           "fdmt_plan_tables")
    if level == 0:
        return [], [], [], n.value
    arr = ctypes.c_int32 * n.value
    a, b, c = arr(), arr(), arr()
    _check(load().fdmt_plan_tables(plan, int(level), int(sub), a, b, c, n.value, ctypes.byref(n)),
           "fdmt_plan_tables")
    return list(a), list(b), list(c), n.value


def fdmt_plan_info(plan):
    lv = ctypes.c_int32()
    _check(load().fdmt_plan_info(plan, ctypes.byref(lv), None, 0), "fdmt_plan_info")
    rows = (ctypes.c_int64 * (lv.value + 1))()
    _check(load().fdmt_plan_info(plan, ctypes.byref(lv), rows, lv.value + 1), "fdmt_plan_info")
    return lv.value, list(rows)


def fdmt_plan_destroy(plan):
    if plan:
        _check(load().fdmt_plan_destroy(plan), "fdmt_plan_destroy")


def fdmt_ragged_plan(plan, nts):
    """Ragged batch over `plan`'s kernels: beams of nts[b] samples. Returns a handle."""
    h = ctypes.c_void_p()
    arr = (ctypes.c_int64 * max(1, len(nts)))(*[int(n) for n in nts])
    _check(load().fdmt_ragged_plan(ctypes.byref(h), plan, len(nts), arr), "fdmt_ragged_plan")
    return h.value


def fdmt_ragged_workspace_bytes(ragged):
    return int(load().fdmt_ragged_workspace_bytes(ragged))


def fdmt_ragged_forward(ragged, in_ptr, out_ptr, ws_ptr, ws_bytes, stream):
    _check(load().fdmt_ragged_forward(ragged, in_ptr, out_ptr, ws_ptr, int(ws_bytes), stream),
           "fdmt_ragged_forward")


def fdmt_ragged_adjoint(ragged, grad_out_ptr, grad_in_ptr, ws_ptr, ws_bytes, stream):
    _check(load().fdmt_ragged_adjoint(ragged, grad_out_ptr, grad_in_ptr, ws_ptr, int(ws_bytes), stream),
           "fdmt_ragged_adjoint")


def fdmt_ragged_run_step(ragged, adjoint, step, in_ptr, out_ptr, ws_ptr, ws_bytes, stream):
    _check(load().fdmt_ragged_run_step(ragged, int(bool(adjoint)), int(step), in_ptr, out_ptr, ws_ptr,
                                       int(ws_bytes), stream), "fdmt_ragged_run_step")


def fdmt_ragged_info(ragged):
    """Returns (beams, total samples, launches of one forward plus one adjoint)."""
    nb, tot, nl = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int32()
    _check(load().fdmt_ragged_info(ragged, ctypes.byref(nb), ctypes.byref(tot), ctypes.byref(nl)),
           "fdmt_ragged_info")
    return nb.value, tot.value, nl.value


def fdmt_ragged_destroy(ragged):
    if ragged:
        _check(load().fdmt_ragged_destroy(ragged), "fdmt_ragged_destroy")


# ----------------------------------------------------------------- tensor layer

def _stream_handle(device):
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Plan:
    """Owns one plan handle. forward/adjoint take and return device tensors
    shaped [Nf][Nt] / [Nd][Nt], or with a leading batch dimension."""

    def __init__(self, nf, nt, nd, f_min, f_max, in_dtype=torch.float32, acc_dtype=torch.float32,
                 host_only=False, unfused=False, tuned=False, wide_planes=False, gamma=-2.0, d_min=0,
                 fft=False, rule=0, **schedule):
        """`gamma`: the delay law dt ~ f^gamma (-2: cold plasma). `d_min`: the
        smallest delay searched (row dt is delay d_min + dt). `rule`: the
        delay-table rule (0: one C per merge; 1: two C's, see
        fdmt_options_t). `fft`: also build
        the FFT-FDMT state for forward_fft(). `schedule`:
        fdmt_options_t schedule fields (first_kernel, first_levels, ...).
        tuned=True first takes the autotuner's stored options for this
        workload, if any; explicit schedule fields override them."""
        self.nf, self.nt, self.nd = int(nf), int(nt), int(nd)
        self.f_min, self.f_max = float(f_min), float(f_max)
        self.gamma = float(gamma)
        self.d_min = int(d_min)
        self.rule = int(rule)
        self.in_dtype, self.acc_dtype = in_dtype, acc_dtype
        flags = ((FDMT_PLAN_HOST_ONLY if host_only else 0) | (FDMT_PLAN_UNFUSED if unfused else 0) |
                 (FDMT_PLAN_WIDE_PLANES if wide_planes else 0) | (FDMT_PLAN_FFT if fft else 0))
        self.device = None if host_only else torch.device("cuda", torch.cuda.current_device())
        self.tuned = None
        if tuned and not host_only and not unfused:
            # the cache lookup is the library's (fdmt_tuned_options); explicit
            # schedule fields override the cached ones
            self.tuned = fdmt_tuned_options(nf, nt, nd, f_min, f_max, _TORCH_TO_CODE[in_dtype],
                                            _TORCH_TO_CODE[acc_dtype], gamma=self.gamma, d_min=self.d_min,
                                            rule=self.rule)
            if self.tuned:
                schedule = dict(self.tuned, **schedule)
        self.options = dict(schedule)
        self.handle = None
        self.handle = fdmt_plan(nf, nt, nd, f_min, f_max, _TORCH_TO_CODE[in_dtype],
                                _TORCH_TO_CODE[acc_dtype], flags, gamma=self.gamma, d_min=self.d_min,
                                rule=self.rule, **schedule)

    def __del__(self):
        h, self.handle = getattr(self, "handle", None), None
        if h and _lib is not None:
            _lib.fdmt_plan_destroy(h)

    def workspace_bytes(self, batch=1):
        return fdmt_workspace_bytes(self.handle, batch)

    def workspace(self, batch=1):
        n = self.workspace_bytes(batch)
        return torch.empty(max(n, 1), dtype=torch.uint8, device=self.device)

    def _run(self, fn, x, out, rows_in, rows_out, dtype_in, dtype_out, ws):
        if x.device != self.device:
            raise ValueError(f"tensor on {x.device}, plan on {self.device}")
        if x.dtype != dtype_in:
            raise TypeError(f"expected {dtype_in}, got {x.dtype}")
        if x.shape[-2:] != (rows_in, self.nt):
            raise ValueError(f"expected [..., {rows_in}, {self.nt}], got {tuple(x.shape)}")
        if x.dim() not in (2, 3):
            raise ValueError("expected a 2-D or 3-D tensor")
        x = x.contiguous()
        batch = 1 if x.dim() == 2 else x.shape[0]
        shape = (rows_out, self.nt) if x.dim() == 2 else (batch, rows_out, self.nt)
        if out is None:
            out = torch.empty(shape, dtype=dtype_out, device=self.device)
        elif out.shape != shape or out.dtype != dtype_out or not out.is_contiguous():
            raise ValueError("out has the wrong shape, dtype or layout")
        if ws is None:
            ws = self.workspace(batch)
        fn(self.handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()), batch,
           ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_handle(self.device))
        return out

    def forward(self, x, out=None, ws=None):
        return self._run(fdmt_forward, x, out, self.nf, self.nd, self.in_dtype, self.acc_dtype, ws)

    def adjoint(self, g, out=None, ws=None):
        return self._run(fdmt_adjoint, g, out, self.nd, self.nf, self.acc_dtype, self.acc_dtype, ws)

    def fft_workspace(self):
        return torch.empty(max(fdmt_fft_workspace_bytes(self.handle), 1), dtype=torch.uint8, device=self.device)

    def forward_fft(self, x, out=None, ws=None):
        """FFT-FDMT (Algorithm 2) of x; the plan needs fft=True."""
        return self._run(fdmt_forward_fft, x, out, self.nf, self.nd, self.in_dtype, self.acc_dtype,
                         self.fft_workspace() if ws is None else ws)

    def search_workspace(self, batch=1, max_log2=8):
        n = fdmt_search_workspace_bytes(self.handle, batch, max_log2)
        return torch.empty(max(n, 1), dtype=torch.uint8, device=self.device)

    def search_fused(self, max_log2=8):
        """True when forward_search runs the boxcar search inside the last
        forward pass (otherwise it reads the output back)."""
        return fdmt_search_fused(self.handle, max_log2)

    def forward_search(self, x, max_log2=8, threshold=6.0, cap=65536, out=None, ws=None):
        """Forward transform plus boxcar search (fdmt_forward_search). Returns
        (output, stats, candidates, count): stats as boxcar_search() returns
        them, candidates an int32 tensor [min(count, cap)][6] of (beam, dt, t,
        width_log2, peak bits, snr bits) - view columns 4 and 5 as float32 -
        and count the number of candidates found (possibly above cap)."""
        if x.device != self.device or x.dtype != self.in_dtype or x.shape[-2:] != (self.nf, self.nt):
            raise ValueError("input does not match the plan")
        x = x.contiguous()
        batch = 1 if x.dim() == 2 else x.shape[0]
        shape = (self.nd, self.nt) if x.dim() == 2 else (batch, self.nd, self.nt)
        if out is None:
            out = torch.empty(shape, dtype=self.acc_dtype, device=self.device)
        if ws is None:
            ws = self.search_workspace(batch, max_log2)
        stats = torch.empty((batch, max_log2 + 1, self.nd, 5), dtype=torch.int32, device=self.device)
        cands = torch.empty((max(cap, 1), 6), dtype=torch.int32, device=self.device)
        count = torch.zeros(1, dtype=torch.int32, device=self.device)
        fdmt_forward_search(self.handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()), batch,
                            max_log2, threshold, ctypes.c_void_p(stats.data_ptr()),
                            ctypes.c_void_p(cands.data_ptr()), cap, ctypes.c_void_p(count.data_ptr()),
                            ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_handle(self.device))
        n = int(count.item())
        f = stats.view(torch.float32)
        res = {"peak": f[..., 0], "t": stats[..., 1], "mean": f[..., 2], "stdev": f[..., 3], "snr": f[..., 4]}
        if x.dim() == 2:
            res = {k: v[0] for k, v in res.items()}
        return out, res, cands[:min(n, cap)], n

    def steps(self, adjoint=False):
        """Per-kernel description of the forward (or adjoint) launch sequence."""
        return [fdmt_step_info(self.handle, adjoint, i)
                for i in range(fdmt_step_count(self.handle, adjoint))]

    def run_step(self, adjoint, step, x, out, ws, batch=None):
        """Enqueue one kernel of the sequence on the current stream (x, out, ws
        preallocated, as for forward/adjoint)."""
        if batch is None:
            batch = 1 if x.dim() == 2 else x.shape[0]
        fdmt_run_step(self.handle, adjoint, step, ctypes.c_void_p(x.data_ptr()),
                      ctypes.c_void_p(out.data_ptr()), batch, ctypes.c_void_p(ws.data_ptr()),
                      ws.numel(), _stream_handle(self.device))

    def tables(self, level, sub):
        return fdmt_plan_tables(self.handle, level, sub)

    def info(self):
        return fdmt_plan_info(self.handle)


class RaggedPlan:
    """Beams of different lengths through one plan's kernels, one launch per
    step for the whole batch. Buffers are packed: beam b's [rows][nt[b]] block
    starts at element rows * (nt[0] + ... + nt[b-1]) of a 1-D tensor."""

    def __init__(self, plan, lengths):
        self.plan = plan  # keeps the plan alive while this handle exists
        self.lengths = [int(n) for n in lengths]
        self.total = sum(self.lengths)
        self.offsets = [0]
        for n in self.lengths:
            self.offsets.append(self.offsets[-1] + n)
        self.device = plan.device
        self.handle = None
        self.handle = fdmt_ragged_plan(plan.handle, self.lengths)

    def __del__(self):
        h, self.handle = getattr(self, "handle", None), None
        if h and _lib is not None:
            _lib.fdmt_ragged_destroy(h)

    def workspace_bytes(self):
        return fdmt_ragged_workspace_bytes(self.handle)

    def workspace(self):
        return torch.empty(max(self.workspace_bytes(), 1), dtype=torch.uint8, device=self.device)

    def pack(self, beams):
        """Concatenate [rows][nt[b]] tensors into one packed 1-D tensor."""
        if len(beams) != len(self.lengths):
            raise ValueError(f"expected {len(self.lengths)} beams, got {len(beams)}")
        for b, (x, n) in enumerate(zip(beams, self.lengths)):
            if x.dim() != 2 or x.shape[1] != n:
                raise ValueError(f"beam {b}: expected [rows, {n}], got {tuple(x.shape)}")
        return torch.cat([x.reshape(-1) for x in beams])

    def unpack(self, packed, rows):
        """Views [rows][nt[b]] of a packed tensor, one per beam."""
        return [packed[rows * a:rows * b].view(rows, b - a)
                for a, b in zip(self.offsets[:-1], self.offsets[1:])]

    def _run(self, fn, x, out, rows_in, rows_out, dtype_in, dtype_out, ws):
        if x.device != self.device:
            raise ValueError(f"tensor on {x.device}, plan on {self.device}")
        if x.dtype != dtype_in:
            raise TypeError(f"expected {dtype_in}, got {x.dtype}")
        if x.dim() != 1 or x.numel() != rows_in * self.total or not x.is_contiguous():
            raise ValueError(f"expected a contiguous 1-D tensor of {rows_in * self.total} elements")
        if out is None:
            out = torch.empty(rows_out * self.total, dtype=dtype_out, device=self.device)
        elif (out.dim() != 1 or out.numel() != rows_out * self.total or out.dtype != dtype_out
              or not out.is_contiguous()):
            raise ValueError("out has the wrong size, dtype or layout")
        if ws is None:
            ws = self.workspace()
        fn(self.handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
           ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_handle(self.device))
        return out

    def forward(self, x, out=None, ws=None):
        p = self.plan
        return self._run(fdmt_ragged_forward, x, out, p.nf, p.nd, p.in_dtype, p.acc_dtype, ws)

    def adjoint(self, g, out=None, ws=None):
        p = self.plan
        return self._run(fdmt_ragged_adjoint, g, out, p.nd, p.nf, p.acc_dtype, p.acc_dtype, ws)

    def run_step(self, adjoint, step, x, out, ws):
        fdmt_ragged_run_step(self.handle, adjoint, step, ctypes.c_void_p(x.data_ptr()),
                             ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(ws.data_ptr()),
                             ws.numel(), _stream_handle(self.device))

    def info(self):
        return fdmt_ragged_info(self.handle)


class FDMTFunction(torch.autograd.Function):
    """y = FDMT(x); the backward pass is the hand-written adjoint."""

    @staticmethod
    def forward(ctx, x, plan):
        ctx.plan = plan
        return plan.forward(x)

    @staticmethod
    def backward(ctx, grad_y):
        return ctx.plan.adjoint(grad_y.contiguous()), None


def fdmt(x, plan):
    return FDMTFunction.apply(x, plan)


def boxcar_search(plane, max_log2=8, ws=None):
    """Boxcar search over FDMT output planes ([Nd][Nt] or [B][Nd][Nt], FP32, on
    the GPU): widths 2^0 .. 2^max_log2. Returns a dict of tensors shaped
    [B][max_log2 + 1][Nd] (no B for a 2-D plane): peak, t (first time of the
    peak), mean and stdev of each width's running sum, and snr =
    (peak - mean) / stdev (0 where stdev is 0), all from fdmt_boxcar_search."""
    if plane.dtype != torch.float32 or plane.device.type != "cuda":
        raise TypeError("plane must be a float32 CUDA tensor")
    squeeze = plane.dim() == 2
    x = (plane.unsqueeze(0) if squeeze else plane).contiguous()
    if x.dim() != 3:
        raise ValueError("plane must be [Nd][Nt] or [B][Nd][Nt]")
    b, nd, nt = x.shape
    out = torch.empty((b, max_log2 + 1, nd, 5), dtype=torch.int32, device=x.device)
    need = fdmt_boxcar_workspace_bytes(b, nd, nt, max_log2)
    if ws is None or ws.numel() < need:
        ws = torch.empty(max(need, 1), dtype=torch.uint8, device=x.device)
    fdmt_boxcar_search(ctypes.c_void_p(x.data_ptr()), b, nd, nt, max_log2, ctypes.c_void_p(out.data_ptr()),
                       ctypes.c_void_p(ws.data_ptr()), ws.numel(), _stream_handle(x.device))
    f = out.view(torch.float32)
    res = {"peak": f[..., 0], "t": out[..., 1], "mean": f[..., 2], "stdev": f[..., 3], "snr": f[..., 4]}
    if squeeze:
        res = {k: v[0] for k, v in res.items()}
    return res
