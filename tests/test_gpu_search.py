"""The forward transform with the boxcar search and candidate list
(fdmt_forward_search) against the oracle.

Bar: the output plane equals fdmt_forward()'s bit for bit; the per-row
statistics lie within the rounding bounds of the float64 definition
(tests/numerics.py, check_boxcar_float64) and their peaks and times equal the
standalone search's (fdmt_boxcar_search) bit for bit; the candidate list
equals the oracle's (boxcar_candidates, float64) except where a block's S/N
lies within rounding of the threshold, each candidate's time holds a value
within rounding of its block's maximum, and its S/N agrees with the oracle's
to 1e-5 relative."""
import numpy as np
import pytest

import workloads as W
from numerics import check_boxcar_float64
from oracle import boxcar, boxcar_candidates, build_tables, fdmt as ofdmt

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1411_5373_amd as F  # noqa: E402

DEV = torch.device("cuda", 0)
BLOCK = 2048
FUSED = dict(first_kernel=3, first_levels=2, later_levels=2, gather_rows=4, gather_vecs=2, search_rows=1)


def _cand_rows(cands):
    c = cands.cpu().numpy()
    f = c.view(np.float32)
    return [(int(r[0]), int(r[1]), int(r[3]), int(r[2]), float(f[i, 4]), float(f[i, 5])) for i, r in enumerate(c)]


def check_candidates(gpu, plane, m, threshold):
    """gpu: list of (b, dt, j, t, peak, snr); plane [B][Nd][Nt] float32."""
    ref = boxcar_candidates(plane, m, threshold, BLOCK)
    y = np.asarray(plane, dtype=np.float64)
    key = lambda c: (c[0], c[1], c[2], c[3] // BLOCK)  # noqa: E731
    got = {key(c): c for c in gpu}
    assert len(got) == len(gpu), "two candidates for one block"
    want = {key(c): c for c in ref}
    u = 2.0 ** -24
    for k in set(got) | set(want):
        b, dt, j, blk = k
        bw = boxcar(y[b, dt], 1 << j)
        mean, sd = bw.mean(), bw.std()
        seg = bw[blk * BLOCK:(blk + 1) * BLOCK]
        snr = (seg.max() - mean) / sd if sd > 0 else 0.0
        e = j * u / (1 - j * u) * boxcar(np.abs(y[b, dt]), 1 << j).max()  # rounding of a window sum
        tol = 1e-5 * abs(snr) + (2 * e / sd if sd > 0 else 0.0) + 1e-6
        if k in want and k not in got:
            assert snr < threshold + tol, f"candidate {k} missing (snr {snr})"
        if k in got and k not in want:
            assert snr > threshold - tol, f"spurious candidate {k} (snr {snr})"
        if k in got:
            c = got[k]
            assert abs(c[5] - snr) <= tol, (k, c[5], snr)
            assert bw[c[3]] >= seg.max() - 2 * e and c[3] // BLOCK == blk, (k, c[3])
            assert abs(c[4] - seg.max()) <= e + 1e-30
    return len(got)


@pytest.mark.parametrize("nf,nt,nd,band,batch,m,sched", [
    (256, 9000, 300, (1.2, 1.6), 1, 8, FUSED),
    (256, 9000, 300, (1.2, 1.6), 1, 8, dict()),
    (128, 4097, 150, (0.4, 0.8), 2, 10, FUSED),
    (64, 2048, 64, (1.2, 1.6), 1, 5, FUSED),
    (64, 100, 64, (1.2, 1.6), 1, 8, FUSED),          # Nt shorter than one tile and than the widest boxcar
    (100, 6000, 120, (1.2, 1.6), 1, 0, FUSED),       # width 1 only; Nf not a power of two
    (512, 5000, 256, (1.2, 1.6), 1, 6, dict(first_levels=3, later_levels=3, gather_vecs=4, search_rows=2)),
    (256, 9000, 300, (1.2, 1.6), 1, 8, dict(FUSED, search_rows=4)),
])
def test_forward_search_matches_oracle(nf, nt, nd, band, batch, m, sched):
    print(f"forward search nf={nf} nt={nt} nd={nd} batch={batch} max_log2={m} {sched}", flush=True)
    rng = np.random.default_rng(nf + nt + m)
    x = rng.standard_normal((batch, nf, nt)).astype(np.float32)
    for b in range(batch):
        pulses = W.draw_pulses(rng, 3, nd, nt, amp_lo=2.0, amp_hi=4.0) if nt > nd else []
        for dt, t_end, amp in pulses:
            for i in range(8):
                W.inject_pulses(x[b], *band, [(dt, t_end - i, amp)])
    p = F.Plan(nf, nt, nd, *band, **sched)
    xd = torch.from_numpy(x).to(DEV)
    y, stats, cands, n = p.forward_search(xd, m, threshold=5.0, cap=100000)
    torch.cuda.synchronize()
    print(f"  fused={p.search_fused(m)} candidates={n}", flush=True)
    assert torch.equal(y, p.forward(xd))
    yn = y.cpu().numpy()
    np.testing.assert_array_equal(yn, np.stack([ofdmt(x[b], *band, nd, acc=np.float32) for b in range(batch)]))
    check_boxcar_float64(stats, yn, m)
    ref = F.boxcar_search(y, m)
    for k in ("peak", "t"):
        assert torch.equal(stats[k], ref[k]), k
    for k in ("mean", "stdev"):  # float64 sums in another order, stored as float32
        a, r = stats[k].cpu().numpy().astype(np.float64), ref[k].cpu().numpy().astype(np.float64)
        assert np.all(np.abs(a - r) <= 2.4e-7 * np.abs(r) + 1e-30), k
    assert n == len(cands)
    found = check_candidates(_cand_rows(cands), yn, m, 5.0)
    assert p.search_fused(m) == bool(sched.get("search_rows"))
    assert found == n


def test_forward_search_cap_and_threshold():
    """More candidates than `cap`: the count reports all of them and `cap`
    slots are filled with distinct ones; an unreachable threshold finds none."""
    nf, nt, nd, band = 64, 8192, 64, (1.2, 1.6)
    x = torch.from_numpy(W.random_input((nf, nt), np.float32, seed=5)).to(DEV)
    p = F.Plan(nf, nt, nd, *band, **FUSED)
    _, _, all_c, n = p.forward_search(x, 4, threshold=1.0, cap=100000)
    assert n > 10 and len(all_c) == n
    _, _, few, n2 = p.forward_search(x, 4, threshold=1.0, cap=7)
    assert n2 == n and len(few) == 7
    assert len({tuple(r) for r in few.cpu().numpy().tolist()}) == 7
    assert {tuple(r) for r in few.cpu().numpy().tolist()} <= {tuple(r) for r in all_c.cpu().numpy().tolist()}
    _, _, none, n3 = p.forward_search(x, 4, threshold=1e30, cap=10)
    assert n3 == 0 and len(none) == 0


def test_c3_forward_search_finds_injected_pulses():
    """The benchmark's workload at full size with its tuned plan: the output
    equals the plain forward, the peaks and times equal the standalone
    search's, and so do the search fused into the last pass (search_rows 1)
    and its candidate list; sampled rows are within the float64 bounds, and
    every injected pulse whose block reaches the threshold is a candidate
    within 2 samples of its (dt, T)."""
    w = W.WORKLOADS["c3"]
    u8, _, pulses = W.make_c3()
    p = F.Plan(w.nf, w.nt, w.nd, w.f_min, w.f_max, in_dtype=torch.uint8, tuned=True)
    m = 8
    assert not p.search_fused(m)
    xd = torch.from_numpy(u8).to(DEV)
    y, stats, cands, n = p.forward_search(xd, m, threshold=7.0, cap=200000)
    torch.cuda.synchronize()
    print(f"c3 forward search: {n} candidates", flush=True)
    assert torch.equal(y, p.forward(xd))
    ref = F.boxcar_search(y, m)
    for k in ("peak", "t"):
        assert torch.equal(stats[k], ref[k]), k
    pf = F.Plan(w.nf, w.nt, w.nd, w.f_min, w.f_max, in_dtype=torch.uint8, tuned=True, search_rows=1)
    assert pf.search_fused(m)
    yf, sf, cf, nf_ = pf.forward_search(xd, m, threshold=7.0, cap=200000)
    assert torch.equal(yf, y) and nf_ == n
    for k in ("peak", "t"):
        assert torch.equal(sf[k], stats[k]), k
    assert sorted(map(tuple, cf.cpu().numpy().tolist())) == sorted(map(tuple, cands.cpu().numpy().tolist()))
    del yf, sf, cf
    rows = sorted({dt for dt, _, _ in pulses} | {0, 1000, w.nd - 1})
    yr = y[rows].cpu().numpy()
    check_boxcar_float64({k: v[:, rows] for k, v in stats.items()}, yr, m)
    c = _cand_rows(cands)
    assert n == len(c)
    # The row statistics span the whole record, partial paths (t0 < dt) included,
    # whose sums on this uint8 data ramp up from far below the row mean: they
    # dominate the standard deviation, so a pulse's block is a candidate when
    # its S/N under those statistics (float64, the oracle's boxcar) reaches the
    # threshold; every such pulse must be in the list near its (dt, T).
    y64 = yr.astype(np.float64)
    detected = 0
    for dt, t_arr, amp in pulses:
        bw = boxcar(y64[rows.index(dt)], 1)
        blk = bw[(t_arr // BLOCK) * BLOCK:(t_arr // BLOCK + 1) * BLOCK]
        snr = (blk.max() - bw.mean()) / bw.std()
        hits = [x for x in c if abs(x[1] - dt) <= 2 and abs(x[3] - t_arr) <= 2]
        print(f"  pulse dt={dt} T={t_arr} amp={amp:.1f}: S/N {snr:.1f}, {len(hits)} candidates near it")
        if snr >= 7.0 * (1 + 1e-4):
            assert hits, f"pulse (dt={dt}, T={t_arr}, amp={amp:.1f}, S/N {snr:.1f}) not among the candidates"
            detected += 1
    assert detected >= 4
