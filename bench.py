#!/usr/bin/env python3
"""FDMT benchmark on one MI355X.

One step = the whole hot path over one beam of the Nf=4096 workload
(Nf=4096 channels over 1.2-1.6 GHz, Nt=65536 samples, Nd=2048 delay trials):
the forward transform of a uint8 intensity matrix with FP32 accumulation,
followed by the hand-written adjoint of an FP32 gradient of the same shape.
Inputs are synthetic and resident in HBM before timing starts.

Prints one JSON line. `value` is DM-trial x samples per second of the whole
step (Nd * Nt / step time); forward-only and adjoint-only rates, achieved HBM
bandwidth, the adjoint/forward time ratio and the other precision forms (with
their speedup over the FP32 form) are reported beside it, and so are the
ragged 256-beam workload and the batch-16 differentiable workload, and the
forward transform with the boxcar search and candidate list fused into its
last pass. `roofline` describes the step's longest kernel: its algorithmic bytes (every
element it must read and write, once) over its average duration measured
with HIP events on the launch stream, against the HBM peak, against the
library's own streaming copy measured in the same run, and against the
library's read/write-mix stream moving that kernel's own read and written
bytes (HBM writes are slower than reads, so a kernel that writes more than it
reads has a lower ceiling than the copy); every step kernel gets the same
three fractions.

The CPU leg (skipped with --cpu-sample 0) runs the oracle: it times it on a
bounded slice of the workload (`cpu_baseline`; the ragged and differentiable
workloads on a pool of host cores, `cpu_baselines`), and it checks this run's
GPU outputs against it on causal slices (`accuracy_vs_oracle`): the first
samples of each forward output, which depend only on the first input
samples, and the last samples of the adjoint output, which depend only on
the last gradient samples.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_c3.txt")
# Files whose change invalidates the committed counter traffic: kernels,
# schedule builder and the tuned schedule choice.
KERNEL_SOURCES = ("paper_1411_5373_amd/csrc/fdmt_kernels.hip",
                  "paper_1411_5373_amd/csrc/fdmt_gather.hip",
                  "paper_1411_5373_amd/csrc/fdmt_narrow.hip",
                  "paper_1411_5373_amd/csrc/fdmt_adjoint.hip",
                  "paper_1411_5373_amd/csrc/fdmt_device.h",
                  "paper_1411_5373_amd/csrc/fdmt_launch.h",
                  "paper_1411_5373_amd/csrc/fdmt_schedule.cpp",
                  "paper_1411_5373_amd/tuning/gfx950.json")
ACCURACY_SAMPLES = 4096  # length of the causal slices checked against the oracle
MAX_POOL = 16            # worker processes of the CPU leg (one GPU's share of host cores)


def source_hash():
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def read_traffic(kernel_key):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    counter summary, or None if absent or taken on different kernel sources."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    vals = {}
    for line in open(TRAFFIC_FILE):
        line = line.strip()
        if line and not line.startswith("#") and "=" in line:
            k, v = line.split("=", 1)
            vals[k.strip()] = v.strip()
    if vals.get("source_hash") != source_hash() or vals.get("kernel") != kernel_key:
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def time_steps(plan, tensors, steps, warmup, torch):
    """Runs warmup + timed steps; returns (wall ms per step, per-kernel mean ms,
    step descriptions). Every kernel is bracketed by HIP events recorded on the
    stream the kernels are launched on (torch's current stream)."""
    x, y, g, xb, ws = tensors
    fwd = plan.steps(False)
    adj = plan.steps(True)
    kernels = [(False, i) for i in range(len(fwd))] + [(True, i) for i in range(len(adj))]

    def run(events=None):
        for j, (is_adj, i) in enumerate(kernels):
            if is_adj:
                plan.run_step(True, i, g, xb, ws)
            else:
                plan.run_step(False, i, x, y, ws)
            if events is not None:
                events[j + 1].record()

    for _ in range(warmup):
        run()
    torch.cuda.synchronize()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(len(kernels) + 1)] for _ in range(steps)]
    t0 = time.perf_counter()
    for k in range(steps):
        ev[k][0].record()
        run(ev[k])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    per = [sum(ev[k][j].elapsed_time(ev[k][j + 1]) for k in range(steps)) / steps
           for j in range(len(kernels))]
    infos = [("adjoint" if a else "forward", (adj if a else fwd)[i]) for a, i in kernels]
    return (t1 - t0) * 1000.0 / steps, per, infos


# ------------------------------------------------------------------ CPU leg

def host_cores():
    return len(os.sched_getaffinity(0))


def cpu_baseline(nt_sample, min_seconds=10.0, max_reps=4):
    """Oracle forward (int64) + adjoint (float64) on the first nt_sample samples,
    repeated until at least min_seconds of CPU work (at most max_reps times)."""
    import numpy as np

    import workloads as W
    from oracle import build_tables, fdmt, fdmt_adjoint
    w = W.WORKLOADS["c3"]
    u8, _, _ = W.make_c3(nt=nt_sample)
    g = np.random.default_rng(7).standard_normal((w.nd, nt_sample))
    reps = 0
    t0 = time.perf_counter()
    while reps < max_reps and (reps == 0 or time.perf_counter() - t0 < min_seconds):
        tab = build_tables(w.nf, w.nd, w.f_min, w.f_max)
        fdmt(u8, w.f_min, w.f_max, w.nd, tab)
        fdmt_adjoint(g, w.f_min, w.f_max, w.nf, tab)
        reps += 1
    dt = (time.perf_counter() - t0) / reps
    n = host_cores()
    return {"value": w.nd * nt_sample / dt, "unit": "DM-trial*samples/s", "cores": 1, "host_cores": n,
            "kind": "oracle",
            "sample": f"one step (forward uint8 -> int64, adjoint float64) of Nf=4096, Nd=2048 on the "
                      f"first {nt_sample} of 65536 samples, {reps} repetition(s), {dt:.2f} s each; "
                      f"NumPy, single thread: 1 of {n} host cores"}


def _oracle_c4_beam(b, nt):
    """Oracle forward (float64) of beam b of the ragged workload (a pool worker)."""
    import numpy as np

    import workloads as W
    from oracle import fdmt
    w = W.WORKLOADS["c4"]
    img, _ = W.make_c4_beam(b, nt)
    fdmt(img.astype(np.float64), w.f_min, w.f_max, w.nd)
    return w.nd * int(nt)


def _oracle_c5_beam(b):
    """Oracle forward and adjoint (float64) of beam b of the differentiable
    workload, the adjoint applied to the loss gradient softmax(A x) (a pool
    worker)."""
    import numpy as np

    import workloads as W
    from oracle import build_tables, fdmt, fdmt_adjoint
    w = W.WORKLOADS["c5"]
    x = W.make_c5()[b].astype(np.float64)
    tab = build_tables(w.nf, w.nd, w.f_min, w.f_max)
    y = fdmt(x, w.f_min, w.f_max, w.nd, tab)
    p = np.exp(y - y.max())
    fdmt_adjoint(p / p.sum(), w.f_min, w.f_max, w.nf, tab)
    return w.nd * w.nt


def cpu_baselines_pooled(beams_c4=48):
    """The ragged and differentiable workloads' oracle on a process pool over
    beams (spawned interpreters that import only NumPy and the oracle)."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor

    import workloads as W
    n = host_cores()
    workers = min(MAX_POOL, n)
    out = {}
    lengths = [int(v) for v in W.c4_lengths()][:beams_c4]
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as pool:
        list(pool.map(_oracle_c4_beam, [0] * workers, [2048] * workers))  # start the workers
        t0 = time.perf_counter()
        cells = sum(pool.map(_oracle_c4_beam, range(len(lengths)), lengths))
        dt = time.perf_counter() - t0
        out["ragged_forward"] = {
            "value": cells / dt, "unit": "DM-trial*samples/s", "cores": workers, "host_cores": n,
            "kind": "oracle",
            "sample": f"forward (float64) of beams 0-{len(lengths) - 1} of the 256-beam workload "
                      f"({sum(lengths)} samples), one beam per worker, {workers} of {n} host cores, "
                      f"{dt:.1f} s"}
        w = W.WORKLOADS["c5"]
        t0 = time.perf_counter()
        cells = sum(pool.map(_oracle_c5_beam, range(w.batch)))
        dt = time.perf_counter() - t0
        out["differentiable"] = {
            "value": cells / dt, "unit": "DM-trial*samples/s", "cores": workers, "host_cores": n,
            "kind": "oracle",
            "sample": f"the whole batch-16 workload: forward + adjoint of softmax (float64) per beam, "
                      f"one beam per worker, {workers} of {n} host cores, {dt:.1f} s"}
    return out


def accuracy(got, ref, integer):
    """Error of a GPU result against the oracle: bit-exact flag, RMS error and
    largest error, both relative to the oracle output's RMS."""
    import numpy as np
    ref64 = np.asarray(ref, dtype=np.float64)
    err = np.asarray(got, dtype=np.float64) - ref64
    rms = float(np.sqrt(np.mean(ref64 * ref64))) or 1.0
    if integer:
        exact = bool(np.array_equal(np.asarray(got).astype(np.int64), np.asarray(ref).astype(np.int64)))
    else:
        exact = bool(np.all(err == 0))
    return {"exact": exact, "rms_rel_err": float(np.sqrt(np.mean(err * err))) / rms,
            "max_err_rel_rms": float(np.max(np.abs(err))) / rms}


def accuracy_leg(checks, w):
    """Compares this run's GPU outputs with the oracle on their slices.
    checks: {name: (kind, input slice, GPU output slice)}; kind 'fwd' (first
    samples of a forward) or 'adj' (last samples of an adjoint)."""
    import numpy as np

    from oracle import build_tables, fdmt, fdmt_adjoint
    tab = build_tables(w.nf, w.nd, w.f_min, w.f_max)
    out = {}
    for name, (kind, x, y) in checks.items():
        integer = x.dtype.kind in "iu"
        xin = x.astype(np.int64) if integer else x.astype(np.float64)
        if kind == "fwd":
            ref = fdmt(xin, w.f_min, w.f_max, w.nd, tab)
        else:
            ref = fdmt_adjoint(xin, w.f_min, w.f_max, w.nf, tab)
        res = accuracy(y, ref, integer and y.dtype.kind in "iuf")
        n = x.shape[-1]
        res["sample"] = (f"first {n} of {w.nt} samples of every output row" if kind == "fwd"
                         else f"last {n} of {w.nt} samples of every channel")
        out[name] = res
    return out


# ------------------------------------------------------------------ GPU legs

def copy_ceiling(F, torch, nbytes=1 << 30, reps=10):
    """Read + write bandwidth of the library's streaming copy kernel on this
    GPU (the practical ceiling of a kernel that moves every byte once)."""
    a = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1)
    F.copy_bytes(b, a)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        F.copy_bytes(b, a)
    ev1.record()
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1) / reps
    ok = bool(torch.equal(a, b))
    del a, b
    return {"bytes_copied": nbytes, "ms": round(ms, 4), "gb_s": round(2 * nbytes / ms / 1e6, 1), "verified": ok}


def mix_ceilings(F, torch, infos, reps=10):
    """Per step kernel: bandwidth of the library's read/write-mix stream
    moving the kernel's own algorithmic bytes (read once, written once). HBM
    serves writes more slowly than reads, so a kernel that writes more than
    it reads has a lower ceiling than the 1:1 copy."""
    pairs = [(i["bytes_read"] // 16 * 16, i["bytes_written"] // 16 * 16) for _, i in infos]
    src = torch.empty(max(r for r, _ in pairs), dtype=torch.uint8, device="cuda")
    dst = torch.empty(max(wr for _, wr in pairs), dtype=torch.uint8, device="cuda")
    src.fill_(1)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    out = []
    for r, wr in pairs:
        if not (r and wr and r <= 2 * wr and wr <= 2 * r):
            out.append(None)
            continue
        a, b = src[:r], dst[:wr]
        F.stream_mix(b, a)
        torch.cuda.synchronize()
        ev0.record()
        for _ in range(reps):
            F.stream_mix(b, a)
        ev1.record()
        torch.cuda.synchronize()
        out.append(round((r + wr) / (ev0.elapsed_time(ev1) / reps) / 1e6, 1))
    del src, dst
    return out


def differentiable_c5(F, torch, W, reps=3):
    """The differentiable form: batch 16, Nf=1024, 0.4-0.8 GHz, Nt=16384,
    Nd=1024, FP32; loss = logsumexp over each beam's DM-time plane, backward
    through the hand-written adjoint (torch.autograd)."""
    w = W.WORKLOADS["c5"]
    plan = F.Plan(w.nf, w.nt, w.nd, w.f_min, w.f_max, tuned=True)
    x = W.torch_noise((w.batch, w.nf, w.nt), W.SEED_BASE + 50, "cuda").requires_grad_(True)

    def step():
        x.grad = None
        y = F.fdmt(x, plan)
        # logsumexp over each beam's Nd*Nt plane, in two stages (over time,
        # then over delay) so torch spreads the reduction over the GPU; the
        # value is the same up to rounding
        lse = torch.logsumexp(torch.logsumexp(y.reshape(w.batch, w.nd, -1), dim=2), dim=1)
        lse.sum().backward()

    step()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        step()
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    return {"workload": f"batch {w.batch}, Nf={w.nf} 0.4-0.8 GHz, Nt={w.nt}, Nd={w.nd}, FP32; "
                        "loss = logsumexp per beam; forward + autograd backward (hand-written adjoint)",
            "ms_per_step": round(ms, 4),
            "dm_trial_samples_per_s": w.batch * w.nd * w.nt / (ms / 1000.0),
            "schedule": plan.options}


def boxcar_on_output(F, torch, y, max_log2=8, reps=10):
    """Boxcar search (widths 1..2^max_log2) over the step's FP32 forward output
    ([Nd][Nt]); its algorithmic bytes are one read of the plane."""
    nd, nt = y.shape
    ws = torch.empty(F.fdmt_boxcar_workspace_bytes(1, nd, nt, max_log2), dtype=torch.uint8, device=y.device)
    F.boxcar_search(y, max_log2, ws=ws)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        F.boxcar_search(y, max_log2, ws=ws)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    return {"widths": f"1..{1 << max_log2}", "plane": f"[{nd}][{nt}] FP32 forward output", "ms": round(ms, 4),
            "alg_gb_s": round(nd * nt * 4 / ms / 1e6, 1)}


def forward_search_leg(F, torch, plan, x, y, max_log2=8, threshold=7.0, reps=10):
    """The forward transform with the boxcar search (widths 1..2^max_log2) and
    its candidate list (fdmt_forward_search), against the forward followed
    by the standalone search over its output, and with the search run inside
    the last forward pass (search_rows = 1)."""
    import ctypes
    nd, nt = y.shape
    stats = torch.empty((1, max_log2 + 1, nd, 5), dtype=torch.int32, device=y.device)
    cap = 1 << 16
    cands = torch.empty((cap, 6), dtype=torch.int32, device=y.device)
    count = torch.zeros(1, dtype=torch.int32, device=y.device)
    vp = ctypes.c_void_p
    stream = F.binding._stream_handle(y.device)

    def search_call(p):
        ws = p.search_workspace(1, max_log2)
        return lambda: F.fdmt_forward_search(p.handle, vp(x.data_ptr()), vp(y.data_ptr()), 1, max_log2, threshold,
                                             vp(stats.data_ptr()), vp(cands.data_ptr()), cap, vp(count.data_ptr()),
                                             vp(ws.data_ptr()), ws.numel(), stream)

    fws = plan.workspace(1)
    bws = torch.empty(F.fdmt_boxcar_workspace_bytes(1, nd, nt, max_log2), dtype=torch.uint8, device=y.device)

    def separate():
        plan.forward(x, out=y, ws=fws)
        F.boxcar_search(y, max_log2, ws=bws)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    ms = timed(search_call(plan))
    n = int(count.item())
    sep = timed(separate)
    in_pass = F.Plan(plan.nf, plan.nt, plan.nd, plan.f_min, plan.f_max, in_dtype=plan.in_dtype,
                     acc_dtype=plan.acc_dtype, search_rows=1, **plan.options)
    in_pass_ms = timed(search_call(in_pass)) if in_pass.search_fused(max_log2) else None
    return {"widths": f"1..{1 << max_log2}", "threshold_snr": threshold, "candidates": n,
            "ms": round(ms, 4), "forward_then_search_ms": round(sep, 4),
            "search_in_last_pass_ms": None if in_pass_ms is None else round(in_pass_ms, 4),
            "dm_trial_samples_per_s": nd * nt / (ms / 1000.0)}


def forward_only(F, torch, w, in_dtype, acc_dtype, reps=10):
    """Tuned forward of one precision form on a fresh input; returns its timing
    and the (input, output) slices the accuracy check compares."""
    plan = F.Plan(w.nf, w.nt, w.nd, w.f_min, w.f_max, in_dtype=in_dtype, acc_dtype=acc_dtype, tuned=True)
    gen = torch.Generator(device="cuda").manual_seed(11)
    if in_dtype == torch.uint8:
        x = torch.randint(0, 256, (w.nf, w.nt), device="cuda", dtype=torch.uint8, generator=gen)
    elif in_dtype == torch.int32:
        x = torch.randint(0, 256, (w.nf, w.nt), device="cuda", dtype=torch.int32, generator=gen)
    else:
        x = torch.randn(w.nf, w.nt, device="cuda", generator=gen).to(in_dtype)
    y = torch.empty(w.nd, w.nt, device="cuda", dtype=acc_dtype)
    ws = plan.workspace(1)
    plan.forward(x, out=y, ws=ws)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        plan.forward(x, out=y, ws=ws)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    k = ACCURACY_SAMPLES
    sl = ("fwd", x[:, :k].cpu().numpy(), y[:, :k].cpu().numpy())
    return {"ms": round(ms, 4), "dm_trial_samples_per_s": w.nd * w.nt / (ms / 1000.0)}, sl


def fft_fdmt(F, torch, w, shift_ms, reps=5):
    """FFT-FDMT (Algorithm 2) forward of the FP32-input form: time per call
    against the shift-based forward of the same input."""
    plan = F.Plan(w.nf, w.nt, w.nd, w.f_min, w.f_max, fft=True)
    x = torch.randn(w.nf, w.nt, device="cuda", generator=torch.Generator(device="cuda").manual_seed(12))
    y = torch.empty(w.nd, w.nt, device="cuda")
    ws = plan.fft_workspace()
    plan.forward_fft(x, out=y, ws=ws)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        plan.forward_fft(x, out=y, ws=ws)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    return {"ms": round(ms, 4), "dm_trial_samples_per_s": w.nd * w.nt / (ms / 1000.0),
            "shift_forward_ms": shift_ms, "slowdown_vs_shift": round(ms / shift_ms, 2),
            "workspace_gb": round(ws.numel() / 1e9, 2)}


def ragged_c4(F, torch, W, reps=5):
    """The ragged workload: 256 beams, Nf=1024, Nd=512, Nt log-uniform in
    [2048, 32768], FP32 in and out. Times the ragged forward and adjoint (one
    launch per step for all beams), the forward replayed from a captured HIP
    graph, and, for comparison, a loop of per-beam calls."""
    w = W.WORKLOADS["c4"]
    lengths = [int(n) for n in W.c4_lengths()]
    tot = sum(lengths)
    plan = F.Plan(w.nf, max(lengths), w.nd, w.f_min, w.f_max, tuned=True)
    r = F.RaggedPlan(plan, lengths)
    x = W.torch_noise((w.nf * tot,), W.SEED_BASE + 40, "cuda")
    g = W.torch_noise((w.nd * tot,), W.SEED_BASE + 41, "cuda")
    y = torch.empty(w.nd * tot, device="cuda")
    xb = torch.empty(w.nf * tot, device="cuda")
    ws = r.workspace()

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            fn()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    fwd_ms = timed(lambda: r.forward(x, out=y, ws=ws))
    adj_ms = timed(lambda: r.adjoint(g, out=xb, ws=ws))
    # one launch per pass: the passes' own times against the whole call (the
    # difference is launch gaps), and the call split into two half batches
    # (t1 + t2 - t = what one call costs beyond its work: launches plus each
    # pass's fill and drain, the most a single persistent kernel could save)
    fwd_kernels = [timed(lambda: r.run_step(False, i, x, y, ws)) for i in range(len(plan.steps(False)))]
    half = len(lengths) // 2
    halves = []
    for sel in (lengths[:half], lengths[half:]):
        rp = F.RaggedPlan(plan, sel)
        n = sum(sel)
        wsp = rp.workspace()
        halves.append(timed(lambda: rp.forward(x[:w.nf * n], out=y[:w.nd * n], ws=wsp)))
        del rp, wsp
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, stream=s):
        r.forward(x, out=y, ws=ws)
    graph_ms = timed(graph.replay)
    plans = [F.Plan(w.nf, n, w.nd, w.f_min, w.f_max, **plan.options) for n in lengths]
    xs, ys = r.unpack(x, w.nf), r.unpack(y, w.nd)

    def loop():
        for p, xi, yi in zip(plans, xs, ys):
            p.forward(xi, out=yi, ws=ws)
    loop_ms = timed(loop)
    rate = w.nd * tot / (fwd_ms / 1000.0)
    return {"workload": f"{len(lengths)} beams, Nf={w.nf} 1.2-1.6 GHz, Nd={w.nd}, Nt log-uniform "
                        f"2048-32768 (total {tot} samples), FP32",
            "launches_forward_plus_adjoint": r.info()[2],
            "forward_ms": round(fwd_ms, 4), "forward_graph_ms": round(graph_ms, 4),
            "adjoint_ms": round(adj_ms, 4), "per_beam_loop_forward_ms": round(loop_ms, 4),
            "forward_kernels_ms": [round(m, 4) for m in fwd_kernels],
            "forward_launch_gaps_ms": round(fwd_ms - sum(fwd_kernels), 4),
            "half_batches_forward_ms": [round(m, 4) for m in halves],
            "per_call_fixed_ms": round(sum(halves) - fwd_ms, 4),
            "forward_dm_trial_samples_per_s": rate, "schedule": plan.options}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--cpu-sample", type=int, default=32768,
                    help="samples of the workload the CPU oracle baseline processes (0: skip the CPU leg, "
                         "including the accuracy checks)")
    ap.add_argument("--no-forms", action="store_true", help="skip the other precision forms")
    ap.add_argument("--no-ragged", action="store_true",
                    help="skip the ragged-batch and differentiable workloads")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="BYTES",
                    help="only run one streaming copy of BYTES (HBM counter calibration)")
    ap.add_argument("--only", choices=("ragged", "differentiable"),
                    help="only run this workload's leg and print its result (for profiling it alone)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(beams and time ranges shard across GPUs without exchange, see the design notes)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_1411_5373_amd as F
    import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_probe:
        a = torch.empty(args.copy_probe, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        a.fill_(1)
        torch.cuda.synchronize()
        F.copy_bytes(b, a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": args.copy_probe}), flush=True)
        return
    if args.only:
        leg = ragged_c4 if args.only == "ragged" else differentiable_c5
        print(json.dumps({args.only: leg(F, torch, W)}), flush=True)
        return

    copy = copy_ceiling(F, torch)
    w = W.WORKLOADS["c3"]
    plan = F.Plan(w.nf, w.nt, w.nd, w.f_min, w.f_max, in_dtype=torch.uint8, acc_dtype=torch.float32,
                  tuned=True)
    x = W.torch_noise((w.nf, w.nt), W.SEED_BASE + 2, "cuda", kind="u8")
    g = W.torch_noise((w.nd, w.nt), W.SEED_BASE + 102, "cuda")
    y = torch.empty(w.nd, w.nt, device="cuda", dtype=torch.float32)
    xb = torch.empty(w.nf, w.nt, device="cuda", dtype=torch.float32)
    ws = plan.workspace(1)
    torch.cuda.synchronize()

    ms_step, per, infos = time_steps(plan, (x, y, g, xb, ws), args.steps, args.warmup, torch)
    k = ACCURACY_SAMPLES
    checks = {"step_forward_u8_f32": ("fwd", x[:, :k].cpu().numpy(), y[:, :k].cpu().numpy()),
              "step_adjoint_f32": ("adj", g[:, -k:].cpu().numpy(), xb[:, -k:].cpu().numpy())}
    fwd_ms = sum(m for m, (d, _) in zip(per, infos) if d == "forward")
    adj_ms = sum(m for m, (d, _) in zip(per, infos) if d == "adjoint")
    fwd_bytes = sum(i["bytes_read"] + i["bytes_written"] for d, i in infos if d == "forward")
    adj_bytes = sum(i["bytes_read"] + i["bytes_written"] for d, i in infos if d == "adjoint")
    j = max(range(len(per)), key=lambda q: per[q])
    dom_dir, dom = infos[j]
    key = f"{dom_dir}:{dom['kind']}:{dom['level_first']}-{dom['level_last']}"
    alg = dom["bytes_read"] + dom["bytes_written"]
    achieved = alg / (per[j] / 1000.0) / 1e9
    traffic = read_traffic(key)
    # Byte models of the transform: compulsory = the
    # input read and the output written once; unfused = every plane of the
    # level-by-level recursion written once and read once (uint8 input, FP32
    # planes); schedule = what this plan's kernels consume and produce.
    _, plane_rows = plan.info()
    compulsory = {"forward": w.nf * w.nt * 1 + w.nd * w.nt * 4, "adjoint": (w.nd + w.nf) * w.nt * 4}
    planes = sum(plane_rows) * w.nt * 4 + sum(plane_rows[:-1]) * w.nt * 4
    unfused = {"forward": w.nf * w.nt * 1 + planes, "adjoint": w.nf * w.nt * 4 + planes}
    models = {d: {"compulsory_gb": round(compulsory[d] / 1e9, 3), "unfused_gb": round(unfused[d] / 1e9, 3),
                  "schedule_gb": round(b / 1e9, 3), "compulsory_gb_s": round(compulsory[d] / ms / 1e6, 1)}
              for d, b, ms in (("forward", fwd_bytes, fwd_ms), ("adjoint", adj_bytes, adj_ms))}
    mixes = mix_ceilings(F, torch, infos)
    kernels = [{"direction": d, "kind": i["kind"], "levels": [i["level_first"], i["level_last"]],
                "ms": round(m, 4), "alg_gb_s": round((i["bytes_read"] + i["bytes_written"]) / m / 1e6, 1),
                "frac_of_peak": round((i["bytes_read"] + i["bytes_written"]) / m / 1e6 / HBM_PEAK_GBS, 3),
                "frac_of_copy": round((i["bytes_read"] + i["bytes_written"]) / m / 1e6 / copy["gb_s"], 3),
                "mix_ceiling_gb_s": mx,
                "frac_of_mix": round((i["bytes_read"] + i["bytes_written"]) / m / 1e6 / mx, 3) if mx else None}
               for m, (d, i), mx in zip(per, infos, mixes)]

    out = {
        "metric": "DM-trial*samples/sec (forward + adjoint step), Nf=4096",
        "value": w.nd * w.nt / (ms_step / 1000.0),
        "unit": "DM-trial*samples/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "Nf=4096 channels 1.2-1.6 GHz, Nt=65536, Nd=2048; uint8 input "
                               "clip(rint(64 + 8 N(0,1))), FP32 accumulation; step = forward + adjoint",
                   "nf": w.nf, "nt": w.nt, "nd": w.nd, "batch": 1, "parallelism": "single GPU",
                   "schedule": plan.options},
        "forward": {"ms": round(fwd_ms, 4), "dm_trial_samples_per_s": w.nd * w.nt / (fwd_ms / 1000.0),
                    "alg_hbm_gb_s": round(fwd_bytes / fwd_ms / 1e6, 1), "bytes": models["forward"]},
        "adjoint": {"ms": round(adj_ms, 4), "alg_hbm_gb_s": round(adj_bytes / adj_ms / 1e6, 1),
                    "bytes": models["adjoint"]},
        "adjoint_forward_ratio": round(adj_ms / fwd_ms, 3),
        "kernels": kernels,
        "roofline": {"bound": "hbm", "kernel": key, "achieved": round(achieved, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic, "algorithmic_bytes": alg, "launch_ms": round(per[j], 4),
                     "copy_ceiling_gb_s": copy["gb_s"], "frac_of_copy": round(achieved / copy["gb_s"], 4),
                     "mix_ceiling_gb_s": mixes[j],
                     "frac_of_mix": round(achieved / mixes[j], 4) if mixes[j] else None},
        "copy_ceiling": copy,
    }
    if not args.no_forms:
        names = {"u8_in_f32_acc": (torch.uint8, torch.float32), "f16_in_f32_acc": (torch.float16, torch.float32),
                 "f32_in_f32_acc": (torch.float32, torch.float32), "u8_in_i32_acc": (torch.uint8, torch.int32),
                 "i32_in_i32_acc": (torch.int32, torch.int32)}
        forms = {}
        for name, (i, a) in names.items():
            forms[name], checks[name] = forward_only(F, torch, w, i, a)
            torch.cuda.empty_cache()
        for form in forms.values():
            form["speedup_vs_f32"] = round(forms["f32_in_f32_acc"]["ms"] / form["ms"], 3)
        out["precision_forms"] = forms
        out["fft_fdmt"] = fft_fdmt(F, torch, w, forms["f32_in_f32_acc"]["ms"])
        torch.cuda.empty_cache()
    out["boxcar"] = boxcar_on_output(F, torch, y)
    out["search"] = forward_search_leg(F, torch, plan, x, y)
    del x, g, y, xb, ws, plan
    if not args.no_ragged:
        torch.cuda.empty_cache()
        out["ragged"] = ragged_c4(F, torch, W)
        torch.cuda.empty_cache()
        out["differentiable"] = differentiable_c5(F, torch, W)
        torch.cuda.empty_cache()
    if args.cpu_sample > 0:
        acc = accuracy_leg(checks, w)
        out["forward"]["accuracy_vs_oracle"] = acc.pop("step_forward_u8_f32")
        out["adjoint"]["accuracy_vs_oracle"] = acc.pop("step_adjoint_f32")
        for name, res in acc.items():
            out["precision_forms"][name]["accuracy_vs_oracle"] = res
        out["cpu_baseline"] = cpu_baseline(args.cpu_sample)
        if not args.no_ragged:
            out["cpu_baselines"] = cpu_baselines_pooled()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
