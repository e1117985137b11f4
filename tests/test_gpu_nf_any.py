"""GPU parity for Nf not a power of two (Sec. 4.2, the case Nf != 2^k):
every pass kernel, dtype, schedule and variant against the oracle's reading
of unequal sub-bands, through the C ABI.

Bar: bit-exact against the int64 oracle for integer input (and uint8 into
FP32), against the oracle's binary32 evaluation for FP32 input (a copy node
adds an exact zero on the GPU and copies in the oracle, so only the sign of a
zero may differ, which equality ignores)."""
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

SHAPES = [  # nf, nt, nd, band
    (5, 1000, 40, (1.2, 1.6)),
    (6, 300, 900, (0.4, 0.8)),        # Nd >> Nf: long partial-sum chains
    (336, 1030, 200, (0.4, 0.8)),
    (1000, 2000, 512, (1.2, 1.6)),
    (1025, 1500, 700, (1.2, 1.6)),    # one channel past a power of two
]

SCHEDULES = [
    dict(),
    dict(later_kernel=2, later_levels=3),                  # level-by-level LDS passes
    dict(later_kernel=1, later_levels=3, tile=256),        # staged passes
    dict(later_levels=4, gather_rows=4, gather_vecs=4),
    dict(gather_vecs=2, adjoint_levels=3, adjoint_last_levels=3, adjoint_last_rows=16,
         adjoint_tile_major=0xFFFF),
    dict(later_levels=2, gather_rows=16, adjoint_levels=1, adjoint_last_levels=1),
    dict(unfused=True),
    dict(first_kernel=1, later_kernel=1, tile=256),        # staged passes from the padded input
    dict(first_kernel=3, first_levels=3, later_levels=3, gather_rows=4, gather_vecs=4,
         adjoint_levels=3, adjoint_last_levels=3, adjoint_last_rows=8),  # input gathers, uint16 planes
    dict(first_kernel=3, first_levels=4, later_levels=4, gather_vecs=2),
]


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


_CASES = {}


def _case(nf, nt, nd, band):
    """Seeded inputs of one shape and the oracle's results (shared by the schedules)."""
    key = (nf, nt, nd, band)
    if key not in _CASES:
        tab = build_tables(nf, nd, *band)
        x = W.random_input((nf, nt), np.float32, seed=nf + 3 * nt)
        g = W.random_input((nd, nt), np.float32, seed=nd + 5 * nt)
        xu = W.random_input((nf, nt), np.uint8, seed=nf + 7 * nt)
        gi = W.random_input((nd, nt), np.int32, seed=nd + 9 * nt, lo=-1000, hi=1000)
        _CASES.clear()
        _CASES[key] = dict(x=x, g=g, xu=xu, gi=gi,
                           y=ofdmt(x, *band, nd, tab, acc=np.float32),
                           xb=oadj(g, *band, nf, tab, acc=np.float32),
                           yu=ofdmt(xu, *band, nd, tab),
                           xbi=oadj(gi.astype(np.int64), *band, nf, tab))
    return _CASES[key]


@pytest.mark.parametrize("sched", SCHEDULES)   # the schedules of one shape run back to back
@pytest.mark.parametrize("nf,nt,nd,band", SHAPES)
def test_forward_and_adjoint(sched, nf, nt, nd, band):
    print(f"nf={nf} nt={nt} nd={nd} {sched}", flush=True)
    c = _case(nf, nt, nd, band)
    p = F.Plan(nf, nt, nd, *band, **sched)
    np.testing.assert_array_equal(p.forward(_dev(c["x"])).cpu().numpy(), c["y"])
    np.testing.assert_array_equal(p.adjoint(_dev(c["g"])).cpu().numpy(), c["xb"])
    for acc in (torch.int32, torch.float32):
        pu = F.Plan(nf, nt, nd, *band, in_dtype=torch.uint8, acc_dtype=acc, **sched)
        np.testing.assert_array_equal(pu.forward(_dev(c["xu"])).cpu().numpy().astype(np.int64), c["yu"])
    pi = F.Plan(nf, nt, nd, *band, in_dtype=torch.int32, acc_dtype=torch.int32, **sched)
    np.testing.assert_array_equal(pi.adjoint(_dev(c["gi"])).cpu().numpy().astype(np.int64), c["xbi"])


@pytest.mark.parametrize("nf,nt,nd,band", SHAPES[:3])
def test_f16_input_and_batch(nf, nt, nd, band):
    """FP16 input, and a batch of three beams equal to three single calls."""
    x = W.random_input((3, nf, nt), np.float16, seed=nf + nd)
    p = F.Plan(nf, nt, nd, *band, in_dtype=torch.float16)
    y = p.forward(_dev(x)).cpu().numpy()
    for b in range(3):
        np.testing.assert_array_equal(y[b], ofdmt(x[b].astype(np.float32), *band, nd, acc=np.float32))


@pytest.mark.parametrize("nf,nt,nd,band,d_min,gamma", [(100, 2000, 128, (1.2, 1.6), 600, -2.0),
                                                       (336, 1030, 200, (0.4, 0.8), 0, 1.0),
                                                       (1000, 1500, 256, (1.2, 1.6), 900, -3.0)])
def test_dmin_and_power_law(nf, nt, nd, band, d_min, gamma):
    """The d_min pre-shift and another delay law together with Nf != 2^k."""
    tab = build_tables(nf, nd, *band, gamma=gamma, d_min=d_min)
    x = W.random_input((nf, nt), np.uint8, seed=nf + d_min)
    p = F.Plan(nf, nt, nd, *band, in_dtype=torch.uint8, acc_dtype=torch.int32, gamma=gamma, d_min=d_min)
    np.testing.assert_array_equal(p.forward(_dev(x)).cpu().numpy().astype(np.int64), ofdmt(x, *band, nd, tab))
    g = W.random_input((nd, nt), np.float32, seed=nd + d_min)
    pf = F.Plan(nf, nt, nd, *band, gamma=gamma, d_min=d_min)
    np.testing.assert_array_equal(pf.adjoint(_dev(g)).cpu().numpy(), oadj(g, *band, nf, tab, acc=np.float32))


def test_pulse_recovered_on_gpu():
    """A dispersed width-1 pulse over 1000 channels peaks at its (dt, T)."""
    nf, nt, nd, band = 1000, 3000, 512, (1.2, 1.6)
    img = np.zeros((nf, nt), dtype=np.uint8)
    W.inject_pulses(img, *band, [(300, 2000, 1.0)])
    y = F.Plan(nf, nt, nd, *band, in_dtype=torch.uint8, acc_dtype=torch.int32).forward(_dev(img)).cpu().numpy()
    i, j = np.unravel_index(np.argmax(y), y.shape)
    assert abs(i - 300) <= 2 and abs(j - 2000) <= 2 and y[i, j] >= 0.6 * nf
