"""GPU parity of ragged batches: beams of different lengths through one plan,
one launch per step for the whole batch, through the C ABI.

Bar: every beam's output equals, bit for bit, the oracle (int64 for integer
input, binary32 for FP32) and the uniform-batch path of a plan with that
beam's Nt; replays of a captured HIP graph equal eager calls."""
import numpy as np
import pytest

import workloads as W
from oracle import build_tables, brute_point, fdmt as ofdmt, fdmt_adjoint as oadj

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1411_5373_amd as F  # noqa: E402

DEV = torch.device("cuda", 0)

# Empty beams, single samples, exact and off-by-one multiples of every tile
# width (64, 256, 512, 1024) and one beam longer than the base plan's Nt.
LENGTHS = [1000, 1, 64, 0, 2049, 333, 4103, 256, 255, 257, 1024, 1025, 63, 0, 511, 513]

SHAPES = [  # nf, nd, band
    (1, 7, (1.2, 1.6)),
    (8, 12, (1.2, 1.6)),
    (64, 100, (1.2, 1.6)),
    (256, 128, (1.2, 1.6)),
    (2, 500, (0.4, 0.8)),
    (1024, 512, (1.2, 1.6)),
    (100, 128, (1.2, 1.6)),          # Nf not a power of two
]


def _beam_inputs(rows, lengths, dtype, seed):
    out = []
    for b, n in enumerate(lengths):
        out.append(W.random_input((rows, n), dtype, seed * 1000 + b))
    return out


def _pack(arrs, dtype):
    return torch.from_numpy(np.concatenate([a.reshape(-1) for a in arrs]).astype(dtype)).to(DEV)


def _unpack(packed, rows, lengths):
    res, off = [], 0
    for n in lengths:
        res.append(packed[rows * off:rows * (off + n)].reshape(rows, n))
        off += n
    return res


@pytest.mark.parametrize("nf,nd,band", SHAPES)
@pytest.mark.parametrize("unfused", [False, True])
def test_ragged_forward_integer_exact(nf, nd, band, unfused):
    print(f"ragged forward u8->i32 nf={nf} nd={nd} unfused={unfused}", flush=True)
    p = F.Plan(nf, 4096, nd, *band, in_dtype=torch.uint8, acc_dtype=torch.int32, unfused=unfused)
    r = F.RaggedPlan(p, LENGTHS)
    xs = _beam_inputs(nf, LENGTHS, np.uint8, nf + nd)
    y = r.forward(_pack(xs, np.uint8))
    ys = _unpack(y.cpu().numpy(), nd, LENGTHS)
    tab = build_tables(nf, nd, *band)
    for x, yb, n in zip(xs, ys, LENGTHS):
        if n == 0:
            assert yb.size == 0
            continue
        np.testing.assert_array_equal(yb.astype(np.int64), ofdmt(x, *band, nd, tab))


@pytest.mark.parametrize("nf,nd,band", SHAPES)
@pytest.mark.parametrize("unfused", [False, True])
def test_ragged_forward_f32_bitwise(nf, nd, band, unfused):
    """FP32: bit-exact against the binary32 oracle and the uniform path per beam."""
    print(f"ragged forward f32 nf={nf} nd={nd} unfused={unfused}", flush=True)
    p = F.Plan(nf, 4096, nd, *band, unfused=unfused)
    r = F.RaggedPlan(p, LENGTHS)
    xs = _beam_inputs(nf, LENGTHS, np.float32, 7 * nf + nd)
    y = r.forward(_pack(xs, np.float32))
    ys = _unpack(y, nd, LENGTHS)
    for x, yb, n in zip(xs, ys, LENGTHS):
        if n == 0:
            continue
        np.testing.assert_array_equal(yb.cpu().numpy(), ofdmt(x, *band, nd, acc=np.float32))
        uni = F.Plan(nf, n, nd, *band, unfused=unfused).forward(torch.from_numpy(x).to(DEV))
        assert torch.equal(yb, uni)


@pytest.mark.parametrize("nf,nd,band", SHAPES)
@pytest.mark.parametrize("unfused", [False, True])
def test_ragged_adjoint_bitwise(nf, nd, band, unfused):
    """Adjoint: int32 exact against the int64 oracle adjoint, FP32 bit-exact
    against the binary32 oracle adjoint, per beam."""
    print(f"ragged adjoint nf={nf} nd={nd} unfused={unfused}", flush=True)
    for acc, npdt in ((torch.int32, np.int32), (torch.float32, np.float32)):
        p = F.Plan(nf, 4096, nd, *band, in_dtype=acc, acc_dtype=acc, unfused=unfused)
        r = F.RaggedPlan(p, LENGTHS)
        gs = _beam_inputs(nd, LENGTHS, npdt, 11 * nf + nd)
        xb = r.adjoint(_pack(gs, npdt))
        xbs = _unpack(xb.cpu().numpy(), nf, LENGTHS)
        for g, xbb, n in zip(gs, xbs, LENGTHS):
            if n == 0:
                assert xbb.size == 0
                continue
            if acc == torch.int32:
                np.testing.assert_array_equal(xbb.astype(np.int64), oadj(g.astype(np.int64), *band, nf))
            else:
                np.testing.assert_array_equal(xbb, oadj(g, *band, nf, acc=np.float32))


@pytest.mark.parametrize("sched", [dict(first_kernel=3), dict(first_kernel=2, later_kernel=2, stream_tiles=3),
                                   dict(first_levels=2, first_kernel=3, later_levels=4, gather_rows=2),
                                   dict(first_levels=3, first_kernel=3, gather_vecs=2, gather_rows=4),
                                   dict(first_levels=3, first_kernel=3, gather_vecs=4, gather_rows=8),
                                   dict(gather_vecs=4, gather_rows=4, adjoint_levels=3, adjoint_last_levels=3,
                                        adjoint_last_rows=16),
                                   dict(first_levels=3, first_kernel=3, gather_vecs=2, gather_rows=8,
                                        gather_threads=512, first_rows=2, first_threads=512, adjoint_rows=4)])
@pytest.mark.parametrize("nf,nd,band", [(256, 128, (1.2, 1.6)), (8, 300, (0.4, 0.8))])
def test_ragged_other_kernel_forms(sched, nf, nd, band):
    """Other pass kernels: ragged forward and adjoint bit-identical to the oracle per beam."""
    print(f"ragged {sched} nf={nf} nd={nd}", flush=True)
    xs = _beam_inputs(nf, LENGTHS, np.float32, 3 * nf + nd)
    p = F.Plan(nf, 4096, nd, *band, **sched)
    y = _unpack(F.RaggedPlan(p, LENGTHS).forward(_pack(xs, np.float32)).cpu().numpy(), nd, LENGTHS)
    for x, yb, n in zip(xs, y, LENGTHS):
        if n:
            np.testing.assert_array_equal(yb, ofdmt(x, *band, nd, acc=np.float32))
    xu = _beam_inputs(nf, LENGTHS, np.uint8, 5 * nf + nd)
    pu = F.Plan(nf, 4096, nd, *band, in_dtype=torch.uint8, acc_dtype=torch.int32, **sched)
    yu = _unpack(F.RaggedPlan(pu, LENGTHS).forward(_pack(xu, np.uint8)).cpu().numpy(), nd, LENGTHS)
    for x, yb, n in zip(xu, yu, LENGTHS):
        if n:
            np.testing.assert_array_equal(yb.astype(np.int64), ofdmt(x, *band, nd))
    # uint8 -> FP32: integer sums below 2^24, exact
    pf = F.Plan(nf, 4096, nd, *band, in_dtype=torch.uint8, acc_dtype=torch.float32, **sched)
    yf = _unpack(F.RaggedPlan(pf, LENGTHS).forward(_pack(xu, np.uint8)).cpu().numpy(), nd, LENGTHS)
    for x, yb, n in zip(xu, yf, LENGTHS):
        if n:
            np.testing.assert_array_equal(yb.astype(np.int64), ofdmt(x, *band, nd))
    gs = _beam_inputs(nd, LENGTHS, np.float32, 9 * nf + nd)
    xb = _unpack(F.RaggedPlan(p, LENGTHS).adjoint(_pack(gs, np.float32)).cpu().numpy(), nf, LENGTHS)
    for g, xbb, n in zip(gs, xb, LENGTHS):
        if n:
            np.testing.assert_array_equal(xbb, oadj(g, *band, nf, acc=np.float32))


def test_ragged_all_empty_and_single_beam():
    p = F.Plan(64, 1000, 64, 1.2, 1.6)
    r = F.RaggedPlan(p, [0, 0])
    assert r.workspace_bytes() == 0
    assert r.info()[:2] == (2, 0)
    e = torch.empty(0, device=DEV)
    assert r.forward(e).numel() == 0
    x = torch.randn(64, 777, device=DEV)
    r1 = F.RaggedPlan(p, [777])
    assert torch.equal(r1.forward(x.reshape(-1)).view(64, 777), F.Plan(64, 777, 64, 1.2, 1.6).forward(x))


def test_ragged_one_launch_per_step():
    """The launch count of a forward plus an adjoint does not grow with the beams."""
    p = F.Plan(1024, 4096, 512, 1.2, 1.6)
    n_steps = len(p.steps(False)) + len(p.steps(True))
    for beams in (1, 16, 256):
        r = F.RaggedPlan(p, [3000 + 17 * b for b in range(beams)])
        assert r.info()[2] == n_steps


def test_ragged_graph_replays_match_eager():
    """A forward and an adjoint captured in one HIP graph: each replay, with
    fresh inputs and eager work between replays, equals the eager result."""
    nf, nd, band = 256, 128, (1.2, 1.6)
    p = F.Plan(nf, 4096, nd, *band, in_dtype=torch.uint8, acc_dtype=torch.float32)
    r = F.RaggedPlan(p, LENGTHS)
    tot = sum(LENGTHS)
    gen = torch.Generator(DEV).manual_seed(5)
    x = torch.randint(0, 256, (nf * tot,), device=DEV, dtype=torch.uint8, generator=gen)
    g = torch.randn(nd * tot, device=DEV, generator=gen)
    y = torch.empty(nd * tot, device=DEV)
    xb = torch.empty(nf * tot, device=DEV)
    ws = r.workspace()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):  # warm-up outside the capture
        r.forward(x, out=y, ws=ws)
        r.adjoint(g, out=xb, ws=ws)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        r.forward(x, out=y, ws=ws)
        r.adjoint(g, out=xb, ws=ws)
    for i in range(4):
        x.copy_(torch.randint(0, 256, x.shape, device=DEV, dtype=torch.uint8, generator=gen))
        g.copy_(torch.randn(g.shape, device=DEV, generator=gen))
        ref_y = r.forward(x)
        ref_xb = r.adjoint(g)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        assert torch.equal(y, ref_y), i
        assert torch.equal(xb, ref_xb), i


def test_c4_full_size():
    """The full ragged workload: 256 beams, Nf=1024, Nd=512, Nt log-uniform in
    [2048, 32768]. uint8 input with int32 accumulation: row 0 is each beam's
    channel sum; sampled points equal the oracle's path sums; sampled beams
    (shortest, longest and others) equal the uniform path bit for bit, in
    int32 and FP32."""
    w = W.WORKLOADS["c4"]
    lengths = [int(n) for n in W.c4_lengths()]
    tot = sum(lengths)
    tab = build_tables(w.nf, w.nd, w.f_min, w.f_max)
    xu8 = W.torch_noise((w.nf * tot,), W.SEED_BASE + 40, DEV, kind="u8")
    rng = np.random.default_rng(4)
    order = np.argsort(lengths)
    sample = sorted({int(order[0]), int(order[-1])} | {int(b) for b in rng.choice(len(lengths), 6, replace=False)})
    for acc in (torch.int32, torch.float32):
        print(f"c4 full u8 -> {acc}", flush=True)
        p = F.Plan(w.nf, 32768, w.nd, w.f_min, w.f_max, in_dtype=torch.uint8, acc_dtype=acc)
        r = F.RaggedPlan(p, lengths)
        y = r.forward(xu8)
        xs = _unpack(xu8, w.nf, lengths)
        ys = _unpack(y, w.nd, lengths)
        for b in range(len(lengths)):
            assert torch.equal(ys[b][0].to(torch.int64), xs[b].to(torch.int64).sum(0)), b
        for b in sample:
            uni = F.Plan(w.nf, lengths[b], w.nd, w.f_min, w.f_max, in_dtype=torch.uint8, acc_dtype=acc)
            assert torch.equal(ys[b], uni.forward(xs[b])), b
        if acc == torch.int32:
            for b in sample[:4]:
                xb = xs[b].cpu().numpy()
                yb = ys[b].cpu().numpy()
                for _ in range(10):
                    dt, t0 = int(rng.integers(w.nd)), int(rng.integers(lengths[b]))
                    assert int(yb[dt, t0]) == brute_point(xb, tab, dt, t0), (b, dt, t0)
        del y, ys, r, p
    print("c4 full adjoint f32", flush=True)
    p = F.Plan(w.nf, 32768, w.nd, w.f_min, w.f_max)
    r = F.RaggedPlan(p, lengths)
    g = W.torch_noise((w.nd * tot,), W.SEED_BASE + 41, DEV)
    xb = r.adjoint(g)
    gs, xbs = _unpack(g, w.nd, lengths), _unpack(xb, w.nf, lengths)
    for b in sample:
        assert torch.equal(xbs[b], F.Plan(w.nf, lengths[b], w.nd, w.f_min, w.f_max).adjoint(gs[b])), b


def test_c4_benchmark_configuration():
    """The ragged benchmark's launch configuration: the tuned FP32 plan (Nt =
    the longest beam) over all 256 beams, forward and adjoint; the shortest,
    the longest and a third beam equal the oracle's binary32 transform and
    adjoint bit for bit."""
    w = W.WORKLOADS["c4"]
    lengths = [int(n) for n in W.c4_lengths()]
    tot = sum(lengths)
    tab = build_tables(w.nf, w.nd, w.f_min, w.f_max)
    p = F.Plan(w.nf, max(lengths), w.nd, w.f_min, w.f_max, tuned=True)
    print(f"c4 tuned {p.options}", flush=True)
    r = F.RaggedPlan(p, lengths)
    order = np.argsort(lengths)
    sample = [int(order[0]), int(order[-1]), int(order[len(order) // 2])]
    x = W.torch_noise((w.nf * tot,), W.SEED_BASE + 42, DEV)
    ys = _unpack(r.forward(x), w.nd, lengths)
    xs = _unpack(x, w.nf, lengths)
    for b in sample:
        np.testing.assert_array_equal(ys[b].cpu().numpy(),
                                      ofdmt(xs[b].cpu().numpy(), w.f_min, w.f_max, w.nd, tab, acc=np.float32))
    del ys, xs, x
    g = W.torch_noise((w.nd * tot,), W.SEED_BASE + 43, DEV)
    xbs, gs = _unpack(r.adjoint(g), w.nf, lengths), _unpack(g, w.nd, lengths)
    for b in sample:
        np.testing.assert_array_equal(xbs[b].cpu().numpy(),
                                      oadj(gs[b].cpu().numpy(), w.f_min, w.f_max, w.nf, tab, acc=np.float32))
