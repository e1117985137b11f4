"""The schedule autotuner on the GPU: it times the candidates, stores the
fastest, the library's cache lookup (fdmt_tuned_options, behind
Plan(tuned=True)) returns it, and a plan built from the stored options
computes the oracle's bits."""
import numpy as np
import pytest

from oracle import fdmt as ofdmt, fdmt_adjoint as oadj

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("no GPU", allow_module_level=True)

import paper_1411_5373_amd as F  # noqa: E402
from paper_1411_5373_amd import autotune as A  # noqa: E402

DEV = torch.device("cuda", 0)


def _set(options):
    """Schedule fields a cache entry sets: zero is the library default, the
    same as leaving the field out."""
    return {k: v for k, v in options.items() if v != 0}


@pytest.mark.parametrize("in_dtype", [torch.uint8, torch.float32])
def test_tuned_schedule_round_trip(tmp_path, monkeypatch, in_dtype):
    monkeypatch.setenv("FDMT_TUNE_CACHE", str(tmp_path / "cache.json"))
    args = (256, 3000, 300, 1.2, 1.6, in_dtype, torch.float32)
    res = A.tune(*args, reps=1)
    assert res["forward_ms"] > 0 and res["adjoint_ms"] > 0
    assert len(res["tried"]) >= len(A.forward_candidates())
    A.store(*args, res)
    p = F.Plan(256, 2900, 300, 1.2, 1.6, in_dtype=in_dtype, tuned=True)  # same Nt bucket
    assert p.tuned == _set(res["options"])
    gen = torch.Generator(DEV).manual_seed(3)
    if in_dtype == torch.uint8:
        x = torch.randint(0, 256, (256, 2900), device=DEV, dtype=torch.uint8, generator=gen)
    else:
        x = torch.randn(256, 2900, device=DEV, generator=gen)
    xn = x.cpu().numpy()
    ref = ofdmt(xn.astype(np.int64), 1.2, 1.6, 300) if in_dtype == torch.uint8 else \
        ofdmt(xn, 1.2, 1.6, 300, acc=np.float32)
    np.testing.assert_array_equal(p.forward(x).cpu().numpy().astype(ref.dtype), ref)
    g = torch.randn(300, 2900, device=DEV, generator=gen)
    pa = F.Plan(256, 2900, 300, 1.2, 1.6, tuned=False, **{k: v for k, v in res["options"].items()})
    np.testing.assert_array_equal(pa.adjoint(g).cpu().numpy(), oadj(g.cpu().numpy(), 1.2, 1.6, 256, acc=np.float32))


def test_ragged_tuning(tmp_path, monkeypatch):
    """Tuning a ragged batch times RaggedPlan candidates (staged passes, which
    the ragged form refuses, are skipped) and stores under the longest beam."""
    monkeypatch.setenv("FDMT_TUNE_CACHE", str(tmp_path / "cache.json"))
    lengths = A.ragged_lengths(6, 200, 3000, 5)
    res = A.tune(64, 0, 64, 1.2, 1.6, reps=1, lengths=lengths)
    assert res["forward_ms"] > 0 and res["adjoint_ms"] > 0
    A.store(64, max(lengths), 64, 1.2, 1.6, torch.float32, torch.float32, res)
    p = F.Plan(64, max(lengths), 64, 1.2, 1.6, tuned=True)
    assert p.tuned == _set(res["options"])
    r = F.RaggedPlan(p, lengths)
    x = torch.randn(64 * sum(lengths), device=DEV, generator=torch.Generator(DEV).manual_seed(4))
    y = r.forward(x)
    for xb, yb in zip(r.unpack(x, 64), r.unpack(y, 64)):
        np.testing.assert_array_equal(yb.cpu().numpy(), ofdmt(xb.cpu().numpy(), 1.2, 1.6, 64, acc=np.float32))
