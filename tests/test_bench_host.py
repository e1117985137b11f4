"""Host checks of the benchmark's command line (no GPU)."""
import os
import subprocess
import sys

from conftest import ROOT


def test_more_than_one_gpu_is_refused():
    """bench.py measures one GPU; --gpus N > 1 exits with status 2 and says so
    before touching a device."""
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_accuracy_leg_flags_exact_and_planted_errors():
    """The benchmark's accuracy check: a forward slice equal to the oracle's
    int64 transform is exact; a binary32 adjoint slice is close but not exact;
    one wrong element shows up in the largest error."""
    import numpy as np

    import bench
    import workloads as W
    from oracle import build_tables, fdmt, fdmt_adjoint
    w = W.WORKLOADS["c1"]
    x = W.random_input((w.nf, 300), np.uint8, seed=3)
    tab = build_tables(w.nf, w.nd, w.f_min, w.f_max)
    y = fdmt(x.astype(np.int64), w.f_min, w.f_max, w.nd, tab).astype(np.float32)
    g = W.random_input((w.nd, 300), np.float32, seed=4)
    xb = fdmt_adjoint(g, w.f_min, w.f_max, w.nf, tab, acc=np.float32)
    res = bench.accuracy_leg({"f": ("fwd", x, y), "a": ("adj", g, xb)}, w)
    assert res["f"]["exact"] and res["f"]["max_err_rel_rms"] == 0.0
    assert not res["a"]["exact"] and 0 < res["a"]["rms_rel_err"] < 1e-6
    y[3, 7] += 1
    bad = bench.accuracy_leg({"f": ("fwd", x, y)}, w)["f"]
    assert not bad["exact"] and bad["max_err_rel_rms"] > 0
