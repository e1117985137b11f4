"""Host-only checks of the C ABI (no GPU needed): the library loads and exports
every function include/fdmt.h declares, the C++ delay tables equal the
oracle's element by element, and every documented error status is returned
before anything is launched."""
import ctypes
import os
import re

import pytest

from conftest import ROOT
from oracle import build_tables

import paper_1411_5373_amd as F
from paper_1411_5373_amd import binding as B


def _declared_functions():
    text = open(os.path.join(ROOT, "include", "fdmt.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fdmt_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_symbol():
    lib = F.load()
    names = _declared_functions()
    assert len(names) >= 9
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(F.EXPORTED)


def _host_plan(nf, nd, f_min, f_max, nt=64, **kw):
    return F.Plan(nf, nt, nd, f_min, f_max, host_only=True, **kw)


def _triples(trip):
    """The oracle's (d_lo, s, d_hi) with a copy row's missing upper half as -1,
    as the library reports it."""
    return [(a, b, -1 if c is None else c) for a, b, c in trip]


def _plane_rows(ref):
    """Rows of each plane in the library: the oracle's plus one zero row per
    sub-band position without channels (Nf not a power of two)."""
    return [sum(r) + sum(1 for j in range(len(r)) if j << l >= ref.nf) for l, r in enumerate(ref.rows)]


@pytest.mark.parametrize("nf,nd,band", [
    (1, 7, (1.2, 1.6)), (2, 3, (1.0, 2.0)), (64, 64, (1.2, 1.6)), (1024, 1024, (1.2, 1.6)),
    (4096, 2048, (1.2, 1.6)), (1024, 512, (1.2, 1.6)), (1024, 1024, (0.4, 0.8)),
    (32, 32, (0.4, 0.8)), (256, 1000, (0.11, 0.19)), (8192, 300, (1.0, 1.5)),
    (3, 4, (1.0, 2.0)), (5, 40, (1.2, 1.6)), (100, 90, (1.2, 1.6)), (336, 500, (0.4, 0.8)),
    (1000, 1024, (1.2, 1.6)), (4095, 2048, (1.2, 1.6)), (2049, 700, (0.11, 0.19)),
])
def test_tables_match_oracle(nf, nd, band):
    ref = build_tables(nf, nd, *band)
    p = _host_plan(nf, nd, *band)
    levels, rows = p.info()
    assert levels == ref.levels
    assert rows == _plane_rows(ref)
    for k in range(nf):
        assert p.tables(0, k)[3] == ref.rows[0][k]
    for l in range(1, levels + 1):
        for j in range(len(ref.rows[l])):
            d_lo, s, d_hi, n = p.tables(l, j)
            assert n == ref.rows[l][j]
            assert list(zip(d_lo, s, d_hi)) == _triples(ref.split[l][j]), (l, j)


@pytest.mark.parametrize("gamma", [-1.0, 1.0, 2.5, -4.0])
@pytest.mark.parametrize("nf,nd,band", [(64, 64, (1.2, 1.6)), (1024, 700, (0.4, 0.8)), (4096, 2048, (1.2, 1.6)),
                                        (600, 700, (0.4, 0.8))])
def test_power_law_tables_match_oracle(gamma, nf, nd, band):
    """Delay law dt ~ f^gamma: the library's tables equal the oracle's
    (the same float64 expression and pow), and differ from the -2 law's."""
    ref = build_tables(nf, nd, *band, gamma=gamma)
    p = F.Plan(nf, 1000, nd, *band, host_only=True, gamma=gamma)
    levels, rows = p.info()
    assert rows == _plane_rows(ref)
    differs = False
    default = build_tables(nf, nd, *band)
    for l in range(1, levels + 1):
        for j in range(len(ref.rows[l])):
            d_lo, s, d_hi, n = p.tables(l, j)
            assert list(zip(d_lo, s, d_hi)) == _triples(ref.split[l][j]), (l, j)
            differs |= ref.split[l][j] != default.split[l][j]
    assert differs
    for bad in (float("inf"), float("nan")):
        with pytest.raises(F.FDMTError) as e:
            F.Plan(nf, 1000, nd, *band, host_only=True, gamma=bad)
        assert e.value.status == B.FDMT_E_INVALID


@pytest.mark.parametrize("nf,nd,band,gamma", [(2, 9, (1.0, 2.0), -2.0), (64, 64, (1.2, 1.6), -2.0),
                                              (4096, 2048, (1.2, 1.6), -2.0), (1024, 1024, (0.4, 0.8), -2.0),
                                              (3, 40, (1.0, 2.0), -2.0), (100, 90, (1.2, 1.6), -2.0),
                                              (1000, 1024, (1.2, 1.6), -2.0), (600, 700, (0.4, 0.8), 2.0),
                                              (5, 300, (1.2, 1.6), -3.0)])
def test_two_c_tables_match_oracle(nf, nd, band, gamma):
    """The two-C rule (rule=1, Sec. 4.2 rounding and binning): the library's
    tables equal the oracle's element by element, with the upper half's
    shift differing from the lower half's delay; channels keep row 0 only."""
    ref = build_tables(nf, nd, *band, gamma=gamma, rule=1)
    p = F.Plan(nf, 1000, nd, *band, host_only=True, gamma=gamma, rule=1)
    levels, rows = p.info()
    assert levels == ref.levels and rows == _plane_rows(ref)
    for k in range(nf):
        assert p.tables(0, k)[3] == 1
    gaps = 0
    for l in range(1, levels + 1):
        for j in range(len(ref.rows[l])):
            d_lo, s, d_hi, n = p.tables(l, j)
            assert n == ref.rows[l][j]
            assert list(zip(d_lo, s, d_hi)) == _triples(ref.split[l][j]), (l, j)
            gaps += sum(1 for a, b, c in zip(d_lo, s, d_hi) if c >= 0 and b != a)
    assert gaps > 0 or nd < 3
    with pytest.raises(F.FDMTError) as e:
        F.Plan(nf, 1000, nd, *band, host_only=True, rule=2)
    assert e.value.status == B.FDMT_E_INVALID


def test_dmin_plan_rules():
    """d_min >= 0; the pre-shift needs the first pass to gather from the
    input, which a d_min plan picks by default; LDS first passes are refused."""
    with pytest.raises(F.FDMTError) as e:
        F.Plan(64, 1000, 64, 1.2, 1.6, host_only=True, d_min=-1)
    assert e.value.status == B.FDMT_E_INVALID
    p = F.Plan(64, 1000, 64, 1.2, 1.6, host_only=True, d_min=500)
    assert p.steps()[0]["kind"] == B.STEP_KINDS[6]      # gather from the input
    for fk in (1, 2):
        with pytest.raises(F.FDMTError) as e:
            F.Plan(64, 1000, 64, 1.2, 1.6, host_only=True, d_min=500, first_kernel=fk)
        assert e.value.status == B.FDMT_E_UNSUPPORTED and "d_min" in F.fdmt_last_error()
    F.Plan(64, 1000, 64, 1.2, 1.6, host_only=True, d_min=500, unfused=True)
    F.Plan(64, 1000, 64, 1.2, 1.6, host_only=True, d_min=0, first_kernel=2)


def test_huge_dmin_refused():
    """Shifts and sample indices stay int32 in the kernels: d_min above 2^30,
    or Nt + d_min + 2 Nd within 8192 of 2^31, is refused before any table is
    built (a host-only plan shows it)."""
    for nt, d_min in ((1000, 2 ** 30 + 1), (1000, 2 ** 31 - 1), (2 ** 31 - 2 ** 30, 2 ** 30)):
        with pytest.raises(F.FDMTError) as e:
            F.Plan(64, nt, 64, 1.2, 1.6, host_only=True, d_min=d_min)
        assert e.value.status == B.FDMT_E_INVALID and "d_min" in F.fdmt_last_error()
    F.Plan(64, 1000, 64, 1.2, 1.6, host_only=True, d_min=2 ** 30)


def test_boxcar_argument_errors_before_launch():
    """fdmt_boxcar_search validates pointers, sizes and the workspace before
    it touches the device."""
    lib = B.load()
    x, o, ws = ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000), ctypes.c_void_p(0x3000)
    need = F.fdmt_boxcar_workspace_bytes(2, 8, 10000, 5)
    assert need == 2 * 6 * 8 * 5 * 24      # beams * widths * rows * 2048-sample tiles * partial
    for args in [(1, 0, 100, 3), (0, 4, 100, 3), (1, 4, 0, 3), (1, 4, 100, 11), (1, 4, 100, -1),
                 (1, 70000, 100, 3)]:
        assert F.fdmt_boxcar_workspace_bytes(*args) == 0
        assert lib.fdmt_boxcar_search(x, *args, o, ws, 1 << 30, None) == B.FDMT_E_INVALID
    assert lib.fdmt_boxcar_search(None, 2, 8, 10000, 5, o, ws, need, None) == B.FDMT_E_INVALID
    assert lib.fdmt_boxcar_search(x, 2, 8, 10000, 5, o, None, need, None) == B.FDMT_E_INVALID
    assert lib.fdmt_boxcar_search(x, 2, 8, 10000, 5, o, ws, need - 1, None) == B.FDMT_E_WORKSPACE
    assert "workspace" in F.fdmt_last_error()


def test_random_bands_match_oracle():
    import numpy as np
    rng = np.random.default_rng(99)
    for _ in range(20):
        nf = int(2 ** rng.integers(0, 11)) if _ % 2 else int(rng.integers(1, 3000))
        nd = int(rng.integers(1, 2000))
        f_min = float(rng.uniform(0.05, 3.0))
        f_max = f_min * float(rng.uniform(1.01, 4.0))
        ref = build_tables(nf, nd, f_min, f_max)
        p = _host_plan(nf, nd, f_min, f_max)
        assert p.info()[1] == _plane_rows(ref)
        for l in range(1, ref.levels + 1):
            subs = len(ref.rows[l])
            for j in list(range(0, subs, max(1, subs // 8))) + [subs - 1]:
                d_lo, s, d_hi, _ = p.tables(l, j)
                assert list(zip(d_lo, s, d_hi)) == _triples(ref.split[l][j])


@pytest.mark.parametrize("args,status", [
    ((0, 64, 8, 1.2, 1.6), B.FDMT_E_INVALID),
    ((131072, 64, 8, 1.2, 1.6), B.FDMT_E_INVALID),
    ((8, 0, 8, 1.2, 1.6), B.FDMT_E_INVALID),          # Nt < 1
    ((8, 64, 0, 1.2, 1.6), B.FDMT_E_INVALID),         # Nd < 1
    ((8, 64, 8, 1.6, 1.2), B.FDMT_E_INVALID),         # f_min >= f_max
    ((8, 64, 8, 1.2, 1.2), B.FDMT_E_INVALID),
    ((8, 64, 8, 0.0, 1.2), B.FDMT_E_INVALID),         # f_min <= 0
    ((8, 64, 8, -1.0, 1.2), B.FDMT_E_INVALID),
    ((8, 64, 8, 1.2, float("inf")), B.FDMT_E_INVALID),
    ((8, 64, 8, float("nan"), 1.2), B.FDMT_E_INVALID),
])
def test_plan_argument_errors(args, status):
    with pytest.raises(F.FDMTError) as e:
        B.fdmt_plan(*args, flags=B.FDMT_PLAN_HOST_ONLY)
    assert e.value.status == status
    assert F.fdmt_last_error() != ""


@pytest.mark.parametrize("in_dt,acc_dt", [(B.FDMT_F16, B.FDMT_I32), (B.FDMT_F32, B.FDMT_I32),
                                          (B.FDMT_I32, B.FDMT_F32), (B.FDMT_F32, B.FDMT_F16), (7, 0)])
def test_unsupported_dtype_pairs(in_dt, acc_dt):
    with pytest.raises(F.FDMTError) as e:
        B.fdmt_plan(8, 64, 8, 1.2, 1.6, in_dt, acc_dt, B.FDMT_PLAN_HOST_ONLY)
    assert e.value.status == B.FDMT_E_UNSUPPORTED


def test_unknown_flag_rejected():
    with pytest.raises(F.FDMTError) as e:
        B.fdmt_plan(8, 64, 8, 1.2, 1.6, flags=0x80 | B.FDMT_PLAN_HOST_ONLY)
    assert e.value.status == B.FDMT_E_INVALID


def test_call_argument_errors_before_launch():
    """Fake (never dereferenced) pointers: every check fails before any launch."""
    lib = F.load()
    unfused = _host_plan(64, 64, 1.2, 1.6, nt=1000, unfused=True)
    # per-iteration schedule: two planes of the tallest (127-row) plane, padded Nt, per beam
    assert unfused.workspace_bytes(2) == 2 * 2 * 127 * 1024 * 4
    p = _host_plan(64, 64, 1.2, 1.6, nt=1000)
    h = p.handle
    need = F.fdmt_workspace_bytes(h, 2)
    assert need == 2 * F.fdmt_workspace_bytes(h, 1) > 0
    assert F.fdmt_workspace_bytes(h, 0) == 0 and F.fdmt_workspace_bytes(None, 1) == 0
    x, y, ws = ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000), ctypes.c_void_p(0x100000)
    for fn in (lib.fdmt_forward, lib.fdmt_adjoint):
        assert fn(None, x, y, 1, ws, need, None) == B.FDMT_E_INVALID
        assert fn(h, None, y, 1, ws, need, None) == B.FDMT_E_INVALID
        assert fn(h, x, None, 1, ws, need, None) == B.FDMT_E_INVALID
        assert fn(h, x, x, 1, ws, need, None) == B.FDMT_E_INVALID
        assert fn(h, x, y, 0, ws, need, None) == B.FDMT_E_INVALID
        assert fn(h, x, y, 2, None, need, None) == B.FDMT_E_WORKSPACE
        assert fn(h, x, y, 2, ws, need - 1, None) == B.FDMT_E_WORKSPACE
        assert fn(h, x, y, 2, ctypes.c_void_p(0x100010), need, None) == B.FDMT_E_WORKSPACE
        assert fn(h, x, y, 2, ws, need, None) == B.FDMT_E_UNSUPPORTED  # host-only plan


def test_single_channel_needs_no_workspace():
    p = _host_plan(1, 10, 1.2, 1.6, nt=100)
    assert p.workspace_bytes(4) == 0


def test_table_query_errors():
    p = _host_plan(8, 8, 1.2, 1.6)
    with pytest.raises(F.FDMTError):
        p.tables(4, 0)
    with pytest.raises(F.FDMTError):
        p.tables(1, 4)
    with pytest.raises(F.FDMTError):
        p.tables(-1, 0)
    assert F.fdmt_status_string(B.FDMT_E_WORKSPACE).startswith("workspace")
    assert B.fdmt_plan_destroy(None) is None


def test_ragged_plan_errors_before_any_device_work():
    """Ragged plans validate beams and the plan's kernels first; a host-only
    plan is refused last (it has no device tables to run)."""
    lib = F.load()
    p = _host_plan(64, 64, 1.2, 1.6, nt=1000)
    with pytest.raises(F.FDMTError) as e:
        B.fdmt_ragged_plan(p.handle, [])
    assert e.value.status == B.FDMT_E_INVALID
    with pytest.raises(F.FDMTError) as e:
        B.fdmt_ragged_plan(p.handle, [100, -1])
    assert e.value.status == B.FDMT_E_INVALID and "beam 1" in F.fdmt_last_error()
    with pytest.raises(F.FDMTError) as e:
        B.fdmt_ragged_plan(p.handle, [2 ** 31])
    assert e.value.status == B.FDMT_E_INVALID
    with pytest.raises(F.FDMTError) as e:
        B.fdmt_ragged_plan(p.handle, [2 ** 30, 2 ** 30])  # padded total above 2^31 - 1
    assert e.value.status == B.FDMT_E_UNSUPPORTED
    with pytest.raises(F.FDMTError) as e:
        B.fdmt_ragged_plan(p.handle, [100, 0, 5000])
    assert e.value.status == B.FDMT_E_UNSUPPORTED and "HOST_ONLY" in F.fdmt_last_error()
    staged = _host_plan(64, 64, 1.2, 1.6, nt=1000, first_kernel=1)
    with pytest.raises(F.FDMTError) as e:
        B.fdmt_ragged_plan(staged.handle, [100])
    assert e.value.status == B.FDMT_E_UNSUPPORTED and "staged" in F.fdmt_last_error()
    with pytest.raises(F.FDMTError) as e:
        B.fdmt_ragged_plan(None, [100])
    assert e.value.status == B.FDMT_E_INVALID
    x, y, ws = ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000), ctypes.c_void_p(0x100000)
    for fn in (lib.fdmt_ragged_forward, lib.fdmt_ragged_adjoint):
        assert fn(None, x, y, ws, 1 << 20, None) == B.FDMT_E_INVALID
    assert lib.fdmt_ragged_run_step(None, 0, 0, x, y, ws, 1 << 20, None) == B.FDMT_E_INVALID
    assert F.fdmt_ragged_workspace_bytes(None) == 0
    assert lib.fdmt_ragged_info(None, None, None, None) == B.FDMT_E_INVALID
    assert B.fdmt_ragged_destroy(None) is None


def _lagged(plan, nf):
    """The last adjoint pass lists each partial-sum subtree once (lagged) when
    some channel has 2..4 partial-sum rows; its waves then store 4 samples
    fewer (the last lane's last run only feeds the lane exchange)."""
    return 1 < max(plan.tables(0, ch)[-1] for ch in range(nf)) <= 4


def test_nt_limit_follows_the_smallest_time_tile():
    """Uniform batches put time tiles on the grid's y axis (at most 65535):
    the plan refuses an Nt that the narrowest step's tile cannot cover."""
    # 16 rows per gather workgroup: 256-sample tiles, 252 in a lagged adjoint pass
    probe = F.Plan(64, 1000, 64, 1.2, 1.6, host_only=True)
    assert _lagged(probe, 64)
    ok = 65535 * 252
    F.Plan(64, ok, 64, 1.2, 1.6, host_only=True, gather_rows=16)
    with pytest.raises(F.FDMTError) as e:
        F.Plan(64, ok + 1, 64, 1.2, 1.6, host_only=True, gather_rows=16)
    assert e.value.status == B.FDMT_E_UNSUPPORTED
    # two runs of 4 samples per lane double the tile
    F.Plan(64, ok + 1, 64, 1.2, 1.6, host_only=True, gather_rows=16, gather_vecs=2)
    with pytest.raises(F.FDMTError) as e:
        B.fdmt_plan(64, 1000, 64, 1.2, 1.6, flags=B.FDMT_PLAN_HOST_ONLY, gather_vecs=3)
    assert e.value.status == B.FDMT_E_INVALID


def test_adjoint_last_rows_shapes_only_the_last_pass():
    """adjoint_last_rows sets the channels per workgroup of the adjoint pass
    into the channels alone: its tile, its work items and the Nt limit follow."""
    nf, nt = 64, 8192
    base = F.Plan(nf, nt, 64, 1.2, 1.6, host_only=True, gather_rows=4)
    wide = F.Plan(nf, nt, 64, 1.2, 1.6, host_only=True, gather_rows=4, adjoint_last_rows=16)
    a, b = base.steps(adjoint=True), wide.steps(adjoint=True)
    assert [s["kind"] for s in a] == [s["kind"] for s in b]
    assert a[-1]["kind"] == B.STEP_KINDS[8] and a[-1]["level_first"] == 0
    for s0, s1 in zip(a[:-1], b[:-1]):
        assert s0["work_items"] == s1["work_items"]
    # 4 rows: 1024-sample tiles; 16 rows: 256-sample tiles (4 fewer per wave if lagged)
    lag = 4 if _lagged(base, nf) else 0
    assert a[-1]["work_items"] == (nf // 4) * -(-nt // (4 * (256 - lag)))
    assert b[-1]["work_items"] == (nf // 16) * -(-nt // (256 - lag))
    ok = 65535 * 256
    F.Plan(64, ok + 1, 64, 1.2, 1.6, host_only=True, gather_rows=4)
    with pytest.raises(F.FDMTError) as e:
        F.Plan(64, ok + 1, 64, 1.2, 1.6, host_only=True, gather_rows=4, adjoint_last_rows=16)
    assert e.value.status == B.FDMT_E_UNSUPPORTED
    for bad in (3, 32, -1):
        with pytest.raises(F.FDMTError) as e:
            F.Plan(64, 1000, 64, 1.2, 1.6, host_only=True, adjoint_last_rows=bad)
        assert e.value.status == B.FDMT_E_INVALID


def test_first_pass_and_adjoint_shapes():
    """first_rows / first_threads shape only a first pass that gathers from the
    input, adjoint_rows only the adjoint gathers into planes: work items follow,
    every other step keeps its shape, and invalid shapes are refused."""
    nf, nt, nd = 4096, 65536, 2048
    kw = dict(first_kernel=3, first_levels=3, later_levels=3, gather_rows=8, gather_threads=512, gather_vecs=2)
    base = F.Plan(nf, nt, nd, 1.2, 1.6, host_only=True, **kw)
    shaped = F.Plan(nf, nt, nd, 1.2, 1.6, host_only=True, first_rows=2, first_threads=512, adjoint_rows=4, **kw)
    f0, f1 = base.steps(), shaped.steps()
    assert f0[0]["kind"] == f1[0]["kind"] == B.STEP_KINDS[6] and f0[0]["level_last"] == 3
    rows0 = f0[0]["bytes_written"] // f0[0]["out_elem_bytes"] // nt
    # 8 rows x 512 threads: one wave per row, 512-sample tiles; 2 rows: 4 waves per row, 2048 samples
    assert f0[0]["work_items"] == -(-rows0 // 8) * (nt // 512)
    assert f1[0]["work_items"] == -(-rows0 // 2) * (nt // 2048)
    for s0, s1 in zip(f0[1:], f1[1:]):
        assert s0["work_items"] == s1["work_items"]
    # adjoint gathers into planes: two 4-sample runs per lane, 1024 threads, so
    # (16 / rows) waves of 512 samples per row
    for steps, r in ((base.steps(adjoint=True), 8), (shaped.steps(adjoint=True), 4)):
        gathers = [st for st in steps[:-1] if st["kind"] == B.STEP_KINDS[8]]
        assert gathers
        for st in gathers:
            n = st["bytes_written"] // (4 * nt)
            assert st["work_items"] == -(-n // r) * -(-nt // (512 * 16 // r))
    for bad in (dict(first_rows=3), dict(first_rows=32), dict(adjoint_rows=-1), dict(first_threads=100),
                dict(first_threads=2048), dict(first_rows=16, first_threads=512),
                dict(adjoint_rows=16, adjoint_threads=512)):
        with pytest.raises(F.FDMTError) as e:
            F.Plan(64, 1000, 64, 1.2, 1.6, host_only=True, **bad)
        assert e.value.status == B.FDMT_E_INVALID, bad


def test_uint8_plans_store_exact_uint16_planes():
    """Planes between two cache gathers of a uint8-input plan are uint16 while
    255 * (2^l + rows - 1) < 2^16 (plane l sums at most 2^l + dt samples)."""
    import torch
    from oracle import build_tables
    kw = dict(first_kernel=3, first_levels=3, later_levels=3)
    p = F.Plan(4096, 65536, 2048, 1.2, 1.6, host_only=True, in_dtype=torch.uint8, **kw)
    steps = p.steps()
    assert [(s["in_elem_bytes"], s["out_elem_bytes"]) for s in steps] == [(1, 2), (2, 2), (2, 4), (4, 4)]
    tab = build_tables(4096, 2048, 1.2, 1.6)
    for s in steps[:-1]:
        l = s["level_last"]
        fits = 255 * (2 ** l + max(tab.rows[l]) - 1) < 2 ** 16
        assert (s["out_elem_bytes"] == 2) == fits
    wide = F.Plan(4096, 65536, 2048, 1.2, 1.6, host_only=True, in_dtype=torch.uint8, wide_planes=True, **kw)
    assert all(s["out_elem_bytes"] == 4 for s in wide.steps())
    f32 = F.Plan(4096, 65536, 2048, 1.2, 1.6, host_only=True, in_dtype=torch.float32, **kw)
    assert all(s["out_elem_bytes"] == 4 for s in f32.steps())


def test_uint16_planes_start_at_the_input_gather():
    """With a level-by-level first pass no plane is narrowed: a narrow plane is
    always made from the input or from another narrow plane."""
    import torch
    p = F.Plan(512, 2048, 96, 0.4, 0.8, host_only=True, in_dtype=torch.uint8, acc_dtype=torch.int32,
               first_kernel=2, later_kernel=3)
    assert all(s["out_elem_bytes"] == 4 for s in p.steps())
    q = F.Plan(512, 2048, 96, 0.4, 0.8, host_only=True, in_dtype=torch.uint8, acc_dtype=torch.int32,
               first_kernel=3, first_levels=2, later_levels=2)
    outs = [s["out_elem_bytes"] for s in q.steps()]
    ins = [s["in_elem_bytes"] for s in q.steps()]
    assert outs[0] == 2 and ins[1:] == outs[:-1]
    assert outs == sorted(outs)  # narrow planes form one run from the input


def test_fft_plan_rules():
    """FFT-FDMT plans: FP32 accumulation only, a length limit, and the entry
    point refuses a plan built without the FFT state before touching the device."""
    import torch
    with pytest.raises(F.FDMTError) as e:
        F.Plan(64, 1000, 64, 1.2, 1.6, host_only=True, fft=True, in_dtype=torch.int32, acc_dtype=torch.int32)
    assert e.value.status == B.FDMT_E_UNSUPPORTED and "FFT" in F.fdmt_last_error()
    with pytest.raises(F.FDMTError) as e:
        F.Plan(1, 16_770_000, 65536, 1.2, 1.6, host_only=True, fft=True)
    assert e.value.status == B.FDMT_E_UNSUPPORTED
    p = F.Plan(64, 1000, 64, 1.2, 1.6, host_only=True, fft=True)
    assert F.fdmt_fft_workspace_bytes(p.handle) == 0           # no FFT state without a device
    lib = B.load()
    x, o, ws = ctypes.c_void_p(0x1000), ctypes.c_void_p(0x2000), ctypes.c_void_p(0x3000)
    assert lib.fdmt_forward_fft(p.handle, x, o, 1, ws, 1 << 30, None) == B.FDMT_E_INVALID
    assert "FDMT_PLAN_FFT" in F.fdmt_last_error()
    assert lib.fdmt_forward_fft(None, x, o, 1, ws, 1 << 30, None) == B.FDMT_E_INVALID


def test_stream_mix_argument_checks():
    """The read/write-mix stream refuses what its kernel does not cover before
    touching the device: NULL, misaligned or overlapping buffers, counts not
    multiples of 16, one count above twice the other."""
    lib = F.load()
    a, b = ctypes.c_void_p(1 << 20), ctypes.c_void_p(1 << 30)
    assert lib.fdmt_stream_mix(a, 0, b, 0, None) == B.FDMT_OK
    assert lib.fdmt_stream_mix(None, 16, b, 16, None) == B.FDMT_E_INVALID
    assert lib.fdmt_stream_mix(ctypes.c_void_p((1 << 20) + 4), 16, b, 16, None) == B.FDMT_E_INVALID
    assert lib.fdmt_stream_mix(a, 24, b, 32, None) == B.FDMT_E_INVALID
    assert lib.fdmt_stream_mix(a, 16, b, 48, None) == B.FDMT_E_INVALID
    assert lib.fdmt_stream_mix(a, 48, b, 16, None) == B.FDMT_E_INVALID
    assert lib.fdmt_stream_mix(a, 16, b, 0, None) == B.FDMT_E_INVALID
    assert lib.fdmt_stream_mix(a, 1 << 20, ctypes.c_void_p((1 << 20) + 4096), 1 << 20, None) == B.FDMT_E_INVALID
    assert "overlap" in F.fdmt_last_error()
