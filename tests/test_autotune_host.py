"""Host checks of the schedule autotuner's cache (no GPU): keys, Nt buckets,
store/lookup round trip, and that every candidate schedule is a valid plan."""
import pytest

torch = pytest.importorskip("torch")

import paper_1411_5373_amd as F  # noqa: E402
from paper_1411_5373_amd import autotune as A  # noqa: E402


def test_nt_bucket_and_key():
    assert [A.nt_bucket(n) for n in (1, 2, 3, 1024, 1025, 65536)] == [1, 2, 4, 1024, 2048, 65536]
    k = A.cache_key("gfx950", 4096, 65000, 2048, 1.2, 1.6, torch.uint8, torch.float32)
    assert k == "gfx950/nf4096/nd2048/band1.2-1.6/u8->f32/nt65536"
    assert k != A.cache_key("gfx950", 4096, 65000, 2048, 1.2, 1.6, torch.float16, torch.float32)


def test_store_lookup_round_trip(tmp_path, monkeypatch):
    monkeypatch.setenv("FDMT_TUNE_CACHE", str(tmp_path / "cache.json"))
    args = (1024, 3000, 512, 1.2, 1.6, torch.float32, torch.float32)
    assert A.lookup(*args, arch_name="gfx950") is None
    res = {"options": {"first_kernel": 3, "first_levels": 3, "gather_rows": 4}, "forward_ms": 1.0,
           "adjoint_ms": 2.0}
    A.store(*args, res, arch_name="gfx950")
    assert A.lookup(*args, arch_name="gfx950") == res["options"]
    # another Nt in the same power-of-two bucket finds it; another band does not
    assert A.lookup(1024, 4000, 512, 1.2, 1.6, torch.float32, torch.float32, arch_name="gfx950") == res["options"]
    assert A.lookup(1024, 3000, 512, 0.4, 0.8, torch.float32, torch.float32, arch_name="gfx950") is None


@pytest.mark.parametrize("nf,nd,band", [(4096, 2048, (1.2, 1.6)), (1024, 512, (1.2, 1.6)),
                                        (1024, 1024, (0.4, 0.8)), (64, 64, (1.2, 1.6))])
def test_candidates_build_host_plans(nf, nd, band):
    """Every candidate either builds or is refused as unsupported for the shape
    (the tuner skips those); the default-built ones cover both directions."""
    built = 0
    for rows in A.GATHER_ROWS:
        for cand in A.forward_candidates() + A.adjoint_candidates(rows):
            def make(**o):
                return F.Plan(nf, 8192, nd, *band, host_only=True, gather_rows=rows,
                              gather_vecs=A.GATHER_VECS[-1], **o)
            try:
                opts = A.resolve_order(cand, make)
                if opts is not None:
                    make(**opts)
                    built += 1
            except F.FDMTError as e:
                assert e.status == 2, str(e)
    assert built > 0


def test_tile_major_masks():
    """Work-order names map to masks over the adjoint passes in launch order."""
    assert [A.tile_major_mask(n, 4) for n in A.TILE_MAJOR_MASKS] == [0, 0b1001, 0b1111]
    assert A.tile_major_mask("ends", 1) == 1 and A.tile_major_mask("all", 0) == 0
    opts = A.resolve_order(dict(adjoint_levels=3, adjoint_last_levels=3, adjoint_tile_major="ends"),
                           lambda **o: F.Plan(4096, 8192, 2048, 1.2, 1.6, host_only=True, **o))
    assert opts["adjoint_tile_major"] == 0b1001  # 12 iterations in 4 passes of 3
