"""GPU parity over seeded random shapes and schedules: Nf (powers of two and
not), Nt (ragged tails, Nt < Nd), Nd, band, delay law, d_min and kernel forms
drawn from a fixed seed; every plan the library accepts must match the oracle
(int64 exact for uint8 input into int32, binary32 bit for bit for FP32),
forward and adjoint."""
import random

import numpy as np
import pytest

import workloads as W
from oracle import build_tables, fdmt as ofdmt, fdmt_adjoint as oadj

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1411_5373_amd as F  # noqa: E402

DEV = torch.device("cuda", 0)


def _case(seed):
    r = random.Random(seed)
    nf = r.choice([r.randint(1, 40), r.randint(40, 700), 2 ** r.randint(0, 9)])
    nd = r.randint(1, 600)
    nt = r.choice([r.randint(1, 300), r.randint(300, 3000)])
    kw = {}
    for key, lo, hi, prob in (("first_kernel", 0, 3, 0.5), ("later_kernel", 0, 3, 0.5), ("first_levels", 1, 4, 0.3),
                              ("later_levels", 1, 4, 0.3), ("gather_rows", 0, 4, 0.3), ("gather_vecs", 0, 2, 0.3),
                              ("adjoint_levels", 1, 4, 0.3), ("adjoint_last_levels", 1, 3, 0.3)):
        if r.random() < prob:
            v = r.randint(lo, hi)
            kw[key] = (1 << v) if key == "gather_rows" else (v if key != "gather_vecs" else (1, 2, 4)[v])
    if r.random() < 0.2:
        kw["d_min"] = r.randint(1, 1500)
    if r.random() < 0.2:
        kw["gamma"] = r.choice([-1.0, 1.0, -3.0])
    f0 = r.uniform(0.2, 2.0)
    return nf, nt, nd, (f0, f0 * r.uniform(1.1, 2.5)), kw


@pytest.mark.parametrize("seed", range(64))
def test_random_shape(seed):
    nf, nt, nd, band, kw = _case(seed)
    print(f"seed {seed}: nf={nf} nt={nt} nd={nd} band={band} {kw}", flush=True)
    gamma, d_min = kw.pop("gamma", -2.0), kw.pop("d_min", 0)
    try:
        pu = F.Plan(nf, nt, nd, *band, in_dtype=torch.uint8, acc_dtype=torch.int32, gamma=gamma, d_min=d_min, **kw)
        pf = F.Plan(nf, nt, nd, *band, gamma=gamma, d_min=d_min, **kw)
    except F.FDMTError as e:
        assert e.status == F.binding.FDMT_E_UNSUPPORTED
        pytest.skip(f"schedule refused: {e}")
    tab = build_tables(nf, nd, *band, gamma=gamma, d_min=d_min)
    xu = W.random_input((nf, nt), np.uint8, seed=seed)
    np.testing.assert_array_equal(pu.forward(torch.from_numpy(xu).to(DEV)).cpu().numpy().astype(np.int64),
                                  ofdmt(xu, *band, nd, tab))
    x = W.random_input((nf, nt), np.float32, seed=seed + 100)
    np.testing.assert_array_equal(pf.forward(torch.from_numpy(x).to(DEV)).cpu().numpy(),
                                  ofdmt(x, *band, nd, tab, acc=np.float32))
    g = W.random_input((nd, nt), np.float32, seed=seed + 200)
    np.testing.assert_array_equal(pf.adjoint(torch.from_numpy(g).to(DEV)).cpu().numpy(),
                                  oadj(g, *band, nf, tab, acc=np.float32))
