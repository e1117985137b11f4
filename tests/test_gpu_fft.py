"""GPU parity of FFT-FDMT (Algorithm 2) against the oracle's complex128
evaluation of the same algorithm, through the C ABI.

Bar: the transforms round in FP32, so results are not bit-exact: the RMS
error is at most 1e-5 of the output RMS (the stated floating-point
tolerance) and no element is off by more than 1e-4 of it; the shift-based
transform of the same input agrees to the same bar."""
import numpy as np
import pytest

import workloads as W
from numerics import rms_ratio, rel_to_rms
from oracle import build_tables, fdmt_fft as offt

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1411_5373_amd as F  # noqa: E402

DEV = torch.device("cuda", 0)
RMS_TOL, MAX_TOL = 1e-5, 1e-4


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _check(y, ref, tag):
    r, m = rms_ratio(y, ref), rel_to_rms(y, ref)
    print(f"  {tag}: RMS(err)/RMS = {r:.2e}, max|err|/RMS = {m:.2e}", flush=True)
    assert r <= RMS_TOL and m <= MAX_TOL


@pytest.mark.parametrize("nf,nt,nd,band", [
    (1, 100, 7, (1.2, 1.6)), (8, 1000, 12, (1.2, 1.6)), (32, 50, 64, (0.4, 0.8)),
    (64, 1030, 100, (1.2, 1.6)), (256, 3001, 300, (1.2, 1.6)), (100, 2000, 128, (1.2, 1.6)),
    (1024, 4096, 1024, (0.4, 0.8))])
@pytest.mark.parametrize("in_dtype", [torch.float32, torch.uint8, torch.float16])
def test_fft_forward_matches_oracle(nf, nt, nd, band, in_dtype):
    print(f"fft nf={nf} nt={nt} nd={nd} {in_dtype}", flush=True)
    npdt = {torch.float32: np.float32, torch.uint8: np.uint8, torch.float16: np.float16}[in_dtype]
    x = W.random_input((nf, nt), npdt, seed=nf + nt + nd)
    p = F.Plan(nf, nt, nd, *band, in_dtype=in_dtype, fft=True)
    y = p.forward_fft(_dev(x)).cpu().numpy()
    ref = offt(x.astype(np.float64), *band, nd)
    _check(y, ref, "vs oracle")
    _check(y, p.forward(_dev(x)).cpu().numpy().astype(np.float64), "vs shift transform")


def test_fft_batch_and_variants():
    """A batch equals single calls bit for bit; d_min, another law and the
    two-C table rule follow the oracle built with them."""
    nf, nt, nd, band = 128, 2000, 200, (1.2, 1.6)
    x = W.random_input((3, nf, nt), np.float32, seed=5)
    p = F.Plan(nf, nt, nd, *band, fft=True)
    y = p.forward_fft(_dev(x))
    for b in range(3):
        assert torch.equal(y[b], p.forward_fft(_dev(x[b])))
    for kw in (dict(d_min=500), dict(gamma=1.0), dict(rule=1)):
        t = build_tables(nf, nd, *band, **kw)
        q = F.Plan(nf, nt, nd, *band, fft=True, **kw)
        _check(q.forward_fft(_dev(x[0])).cpu().numpy(), offt(x[0].astype(np.float64), *band, nd, t), str(kw))


def test_fft_needs_fft_plan():
    p = F.Plan(64, 1000, 64, 1.2, 1.6)
    with pytest.raises(F.FDMTError) as e:
        p.forward_fft(torch.zeros(64, 1000, device=DEV), ws=torch.empty(256, dtype=torch.uint8, device=DEV))
    assert e.value.status == F.binding.FDMT_E_INVALID
