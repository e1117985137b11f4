"""The allocation-free boxcar search (fdmt_boxcar_search_noalloc) against the
workspace entry point (fdmt_boxcar_search), through the C ABI: identical
results on two calls in a row, the second on a smaller plane (the static
scratch keeps the first call's partials; the second must not read them), and
a plane too large for the static buffer refused before any launch."""
import ctypes

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1411_5373_amd as F  # noqa: E402
from paper_1411_5373_amd import binding as B  # noqa: E402

DEV = torch.device("cuda", 0)


def _noalloc(plane, m):
    b, nd, nt = plane.shape
    out = torch.empty((b, m + 1, nd, 5), dtype=torch.int32, device=DEV)
    B.fdmt_boxcar_search_noalloc(ctypes.c_void_p(plane.data_ptr()), b, nd, nt, m, ctypes.c_void_p(out.data_ptr()),
                                 B._stream_handle(DEV))
    return out


def _with_ws(plane, m):
    b, nd, nt = plane.shape
    out = torch.empty((b, m + 1, nd, 5), dtype=torch.int32, device=DEV)
    ws = torch.empty(max(1, B.fdmt_boxcar_workspace_bytes(b, nd, nt, m)), dtype=torch.uint8, device=DEV)
    B.fdmt_boxcar_search(ctypes.c_void_p(plane.data_ptr()), b, nd, nt, m, ctypes.c_void_p(out.data_ptr()),
                         ctypes.c_void_p(ws.data_ptr()), ws.numel(), B._stream_handle(DEV))
    return out


def test_noalloc_boxcar_matches_workspace_entry_point():
    print("no-alloc boxcar: [2][300][20000] then [1][7][4097]", flush=True)
    big = torch.from_numpy(W.random_input((2, 300, 20000), np.float32, seed=91)).to(DEV)
    small = torch.from_numpy(W.random_input((1, 7, 4097), np.float32, seed=92)).to(DEV)
    a1 = _noalloc(big, 8)
    a2 = _noalloc(small, 10)
    torch.cuda.synchronize()
    assert torch.equal(a1, _with_ws(big, 8))
    assert torch.equal(a2, _with_ws(small, 10))
    # the full Nf=4096 workload's plane size fits the static buffer
    assert B.fdmt_boxcar_workspace_bytes(1, 2048, 65536, 10) <= 32 << 20


def test_noalloc_boxcar_refuses_oversized_plane():
    print("no-alloc boxcar: oversized request refused", flush=True)
    nd, nt, m = 4096, 1 << 20, 10
    assert B.fdmt_boxcar_workspace_bytes(1, nd, nt, m) > 32 << 20
    tiny = torch.zeros(16, device=DEV)
    out = torch.zeros(16, dtype=torch.int32, device=DEV)
    with pytest.raises(F.FDMTError) as e:
        B.fdmt_boxcar_search_noalloc(ctypes.c_void_p(tiny.data_ptr()), 1, nd, nt, m, ctypes.c_void_p(out.data_ptr()),
                                     B._stream_handle(DEV))
    assert e.value.status == B.FDMT_E_WORKSPACE
