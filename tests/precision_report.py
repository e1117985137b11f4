"""Accuracy and speed of each precision form at full size (Nf=4096,
Nt=65536, Nd=2048, 1.2-1.6 GHz), written to profiles/precision_c3.txt.

Run on a GPU from the repository root:
    python tests/precision_report.py

Each form runs the whole record on the GPU with the tuned schedule; its
accuracy is measured against the oracle on a 4096-sample slice: the first
samples for the forward (an output depends only on earlier input), the last
for the adjoint (a gradient depends only on later output gradients), so the
slice results equal the full-record ones. Integer-valued forms are compared
exactly with the int64 oracle, floating forms with the float64 oracle. Every
schedule adds the same terms in the same tree, so the accuracy does not depend
on the schedule; the times do.
"""
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
sys.path.insert(0, os.path.join(ROOT, "tests"))

import paper_1411_5373_amd as F  # noqa: E402
import workloads as W  # noqa: E402
from numerics import rel_to_rms, rms_ratio  # noqa: E402
from oracle import build_tables, fdmt, fdmt_adjoint  # noqa: E402

SLICE = 4096
OUT = os.path.join(ROOT, "profiles", "precision_c3.txt")


def timed(fn, reps=10):
    fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def main():
    w = W.WORKLOADS["c3"]
    tab = build_tables(w.nf, w.nd, w.f_min, w.f_max)
    u8, f16, _ = W.make_c3()
    f32 = f16.astype(np.float32)
    forms = [("f32_in_f32_acc", f32, torch.float32, torch.float32),
             ("f16_in_f32_acc", f16, torch.float16, torch.float32),
             ("u8_in_f32_acc", u8, torch.uint8, torch.float32),
             ("u8_in_i32_acc", u8, torch.uint8, torch.int32),
             ("i32_in_i32_acc", u8.astype(np.int32), torch.int32, torch.int32)]
    lines = []
    ref_ms = None
    for name, x, ind, acc in forms:
        print(name, flush=True)
        p = F.Plan(w.nf, w.nt, w.nd, w.f_min, w.f_max, in_dtype=ind, acc_dtype=acc, tuned=True)
        xd = torch.from_numpy(np.ascontiguousarray(x)).cuda()
        y = torch.empty(w.nd, w.nt, device="cuda", dtype=acc)
        ws = p.workspace(1)
        ms = timed(lambda: p.forward(xd, out=y, ws=ws))
        got = y[:, :SLICE].cpu().numpy()
        if np.dtype(x.dtype).kind in "iu":
            ref = fdmt(x[:, :SLICE].astype(np.int64), w.f_min, w.f_max, w.nd, tab)
            exact = bool(np.array_equal(got.astype(np.int64), ref))
            rms, mx = (0.0, 0.0) if exact else (rms_ratio(got, ref), rel_to_rms(got, ref))
        else:
            ref = fdmt(x[:, :SLICE].astype(np.float64), w.f_min, w.f_max, w.nd, tab)
            exact = bool(np.array_equal(got.astype(np.float64), ref))
            rms, mx = rms_ratio(got, ref), rel_to_rms(got, ref)
        if name == "f32_in_f32_acc":
            ref_ms = ms
        lines.append((name, ms, exact, rms, mx))
        del p, xd, y, ws
    # adjoint, FP32 gradients
    print("adjoint", flush=True)
    p = F.Plan(w.nf, w.nt, w.nd, w.f_min, w.f_max, tuned=True)
    g = np.random.default_rng(W.SEED_BASE + 102).standard_normal((w.nd, w.nt), dtype=np.float32)
    gd = torch.from_numpy(g).cuda()
    xb = torch.empty(w.nf, w.nt, device="cuda")
    ws = p.workspace(1)
    adj_ms = timed(lambda: p.adjoint(gd, out=xb, ws=ws))
    got = xb[:, w.nt - SLICE:].cpu().numpy()
    ref = fdmt_adjoint(g[:, w.nt - SLICE:].astype(np.float64), w.f_min, w.f_max, w.nf, tab)
    adj = ("adjoint_f32", adj_ms, bool(np.array_equal(got.astype(np.float64), ref)), rms_ratio(got, ref),
           rel_to_rms(got, ref))
    with open(OUT, "w") as f:
        f.write("# Precision forms of the FDMT at Nf=4096 (1.2-1.6 GHz), Nt=65536, Nd=2048 on one MI355X,\n")
        f.write("# tuned schedules; time per forward (adjoint) over the whole record, accuracy against\n")
        f.write(f"# the oracle on a {SLICE}-sample slice (int64 for integer-valued input, float64 otherwise).\n")
        f.write("# Input: the c3 workload (uint8 = clip(rint(64 + 8x)), FP16 = x, FP32 = the FP16 values).\n")
        f.write("# command (from the repository root): python tests/precision_report.py\n")
        f.write(f"# written {time.strftime('%Y-%m-%d')}\n#\n")
        f.write("# form             ms      speedup_vs_f32  exact  rms_err/rms  max_err/rms\n")
        for name, ms, exact, rms, mx in lines:
            f.write(f"{name:16s} {ms:8.4f} {ref_ms / ms:10.3f}      {int(exact)}  {rms:11.3e}  {mx:11.3e}\n")
        name, ms, exact, rms, mx = adj
        f.write(f"{name:16s} {ms:8.4f} {'-':>10s}      {int(exact)}  {rms:11.3e}  {mx:11.3e}\n")
    print(open(OUT).read())


if __name__ == "__main__":
    main()
