"""GPU parity of the boxcar search (fdmt_boxcar_search) against the oracle.

Bar: against the float64 definition of every running sum (oracle `boxcar`),
each result lies within the rounding bound of a binary32 window sum of depth
log2(w) (tests/numerics.py, check_boxcar_float64): the peak within that bound,
its time at a value that is a maximum up to twice the bound (and the exact
argmax where only one index qualifies), mean, standard deviation and S/N by
error propagation. Additionally, the peaks and their times equal the oracle's
binary32 evaluation of the doubling tree bit for bit."""
import numpy as np
import pytest

import workloads as W
from numerics import check_boxcar_float64
from oracle import boxcar_search as oboxcar

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1411_5373_amd as F  # noqa: E402

DEV = torch.device("cuda", 0)


def _check(res, y, m):
    check_boxcar_float64(res, y, m)
    _check_tree(res, oboxcar(y, m, acc=np.float32))


def _check_tree(res, ref):
    peak = res["peak"].cpu().numpy()
    np.testing.assert_array_equal(peak, ref["peak"].astype(np.float32))
    np.testing.assert_array_equal(res["t"].cpu().numpy(), ref["t"])
    scale = np.maximum(ref["stdev"], np.abs(ref["mean"])) + 1e-30
    for k in ("mean", "stdev"):
        assert np.all(np.abs(res[k].cpu().numpy() - ref[k]) <= 1e-6 * scale), k
    np.testing.assert_allclose(res["snr"].cpu().numpy(), ref["snr"], rtol=1e-5, atol=1e-5)


@pytest.mark.parametrize("batch,nd,nt,m", [(1, 1, 1, 0), (2, 3, 37, 5), (1, 5, 4096, 3), (1, 7, 4097, 10),
                                           (1, 64, 10000, 8), (3, 2, 300, 10), (1, 4, 8191, 1)])
def test_boxcar_matches_oracle(batch, nd, nt, m):
    print(f"boxcar batch={batch} nd={nd} nt={nt} max_log2={m}", flush=True)
    y = W.random_input((batch, nd, nt), np.float32, seed=nd * 1000 + nt + m)
    res = F.boxcar_search(torch.from_numpy(y).to(DEV), m)
    _check(res, y, m)
    # a 2-D plane gives the same rows without the batch axis
    res2 = F.boxcar_search(torch.from_numpy(y[0]).to(DEV), m)
    np.testing.assert_array_equal(res2["t"].cpu().numpy(), res["t"].cpu().numpy()[0])


def test_boxcar_ties_and_constant_rows():
    """Equal maxima: the first time wins; a constant row has stdev 0 only at
    width 1 (later widths ramp up), and S/N 0 there."""
    y = np.zeros((3, 5000), dtype=np.float32)
    y[0, [100, 4500]] = 7.0          # two equal peaks in different tiles
    y[1, :] = 1.5
    y[2, [4095, 4096]] = 2.0         # a width-2 window across the tile border
    res = F.boxcar_search(torch.from_numpy(y).to(DEV), 4)
    _check(res, y, 4)
    assert int(res["t"][0, 0]) == 100 and float(res["snr"][0, 1]) == 0.0
    assert int(res["t"][1, 2]) == 4096 and float(res["peak"][1, 2]) == 4.0


def test_boxcar_finds_dispersed_pulse():
    """Pipeline: FDMT of a dispersed 8-sample pulse in noise, then the boxcar
    search: the widest S/N sits at the pulse's delay row and the width-8
    boxcar peaks at its end; the search equals the oracle on the same plane."""
    nf, nt, nd, band = 256, 6000, 256, (1.2, 1.6)
    rng = np.random.default_rng(77)
    x = rng.standard_normal((nf, nt)).astype(np.float32)
    dt, t_end = 150, 4000
    for i in range(8):
        W.inject_pulses(x, *band, [(dt, t_end - i, 1.5)])
    plan = F.Plan(nf, nt, nd, *band)
    y = plan.forward(torch.from_numpy(x).to(DEV))
    res = F.boxcar_search(y, 5)
    _check(res, y.cpu().numpy(), 5)
    snr = res["snr"].cpu().numpy()
    j, row = np.unravel_index(np.argmax(snr), snr.shape)
    assert abs(row - dt) <= 2 and (1 << j) in (4, 8, 16), (j, row)
    assert abs(int(res["t"][3, row]) - t_end) <= 2
    assert snr.max() > 10
