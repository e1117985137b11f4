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


def _parse_key(key):
    """(arch, nf, nd, f_min, f_max, gamma, in, acc, nt) of a cache key."""
    parts = key.split("/")
    arch, nf, nd = parts[0], int(parts[1][2:]), int(parts[2][2:])
    lo, hi = (float(v) for v in parts[3][4:].split("-"))
    gamma, rest = -2.0, parts[4:]
    if rest[0].startswith("gamma"):
        gamma, rest = float(rest[0][5:]), rest[1:]
    i, a = rest[0].split("->")
    return arch, nf, nd, lo, hi, gamma, A.DTYPES[i], A.DTYPES[a], int(rest[1][2:])


def test_c_abi_lookup_matches_every_shipped_entry():
    """fdmt_tuned_options (the C ABI's reader of the tuning cache, which
    Plan(tuned=True) goes through) returns, for every workload in the cache
    shipped beside the library, exactly the options the tuner stored; an Nt in
    the same power-of-two bucket finds the same entry."""
    cache = A.load_cache("gfx950")
    assert cache
    B = F.binding
    code = {v: k for k, v in B._CODE_TO_TORCH.items()}
    for key, entry in cache.items():
        arch, nf, nd, lo, hi, gamma, i, a, nt = _parse_key(key)
        assert A.cache_key(arch, nf, nt, nd, lo, hi, i, a, gamma) == key
        got = B.fdmt_tuned_options(nf, nt, nd, lo, hi, code[i], code[a], gamma=gamma, arch=arch)
        assert got == {k: v for k, v in entry["options"].items() if v != 0}, key
        assert B.fdmt_tuned_options(nf, nt // 2 + 1, nd, lo, hi, code[i], code[a], gamma=gamma, arch=arch) == got


def test_c_abi_lookup_rules(tmp_path, monkeypatch):
    """Explicit nonzero fields win over the cache; a missing file or another
    architecture finds nothing; a d_min plan keeps a gather from the input; a
    malformed cache or an unknown field is an invalid-argument error."""
    B = F.binding
    args = (1024, 3000, 512, 1.2, 1.6, B.FDMT_F32, B.FDMT_F32)
    path = tmp_path / "c.json"
    monkeypatch.setenv("FDMT_TUNE_CACHE", str(path))
    A.store(1024, 3000, 512, 1.2, 1.6, torch.float32, torch.float32,
            {"options": {"first_kernel": 2, "first_levels": 4, "gather_rows": 4}, "forward_ms": 1.0,
             "adjoint_ms": 1.0}, arch_name="gfx950")
    monkeypatch.delenv("FDMT_TUNE_CACHE")
    assert B.fdmt_tuned_options(*args, cache_path=str(path), arch="gfx950") == \
        {"first_kernel": 2, "first_levels": 4, "gather_rows": 4}
    assert B.fdmt_tuned_options(*args, cache_path=str(path), arch="gfx950", gather_rows=16)["gather_rows"] == 16
    assert B.fdmt_tuned_options(*args, cache_path=str(path), arch="gfx950", d_min=100)["first_kernel"] == 3
    assert B.fdmt_tuned_options(*args, cache_path=str(path), arch="gfx942") is None
    assert B.fdmt_tuned_options(*args, cache_path=str(tmp_path / "none.json"), arch="gfx950") is None
    bad = tmp_path / "bad.json"
    bad.write_text('{"gfx950/nf1024": {"options": {"first_kernel": 2,}}}')
    with pytest.raises(F.FDMTError) as e:
        B.fdmt_tuned_options(*args, cache_path=str(bad), arch="gfx950")
    assert e.value.status == B.FDMT_E_INVALID
    key = A.cache_key("gfx950", 1024, 3000, 512, 1.2, 1.6, torch.float32, torch.float32)
    bad.write_text('{"%s": {"options": {"warp_size": 32}}}' % key)
    with pytest.raises(F.FDMTError) as e:
        B.fdmt_tuned_options(*args, cache_path=str(bad), arch="gfx950")
    assert "warp_size" in str(e.value)
