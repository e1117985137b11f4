"""Schedule autotuner: times candidate plan options on the GPU and keeps the
fastest per workload in a JSON cache that `Plan(..., tuned=True)` consults.

Every candidate is a set of `fdmt_options_t` schedule fields (kernel form and
iterations of each pass, tile width, LDS budget, rows, threads and samples per
gather workgroup, adjoint pass depths). Schedule fields never change results,
only speed, so the tuner compares times alone. Forward and adjoint are tuned
separately: the forward's pass structure first, at one workgroup shape, then
the workgroup shapes of its first and later passes; the adjoint's depths,
last-pass shape and work order for each row count. The one field they share
(samples per lane) is chosen to minimise their sum.

Cache key: GPU architecture, Nf, Nd, band, the delay law's power when it is
not -2, input and accumulation dtypes and Nt rounded up to a power of two.
The cache shipped with the package (tuning/<arch>.json) holds the entries its
benchmark workloads use; FDMT_TUNE_CACHE names another file to read and
update instead.

Command line (on a GPU):
  python -m paper_1411_5373_amd.autotune --nf 4096 --nt 65536 --nd 2048 \
      --band 1.2 1.6 --in-dtype u8 --acc-dtype f32 [--write]
"""
from __future__ import annotations

import argparse
import json
import os
import time

import torch

from . import binding as B

DTYPES = {"f32": torch.float32, "f16": torch.float16, "u8": torch.uint8, "i32": torch.int32}
_NAMES = {v: k for k, v in DTYPES.items()}

PKG_DIR = os.path.dirname(os.path.abspath(__file__))

GATHER_ROWS = (4, 8)
GATHER_VECS = (1, 2, 4)
GATHER_THREADS = (512, 1024)
# (first_rows, first_threads) of a first pass that gathers from the input;
# (0, 0) = the later passes' shape
FIRST_SHAPES = ((0, 0), (2, 512), (4, 512))
GATHER_ROWS_DEFAULT = 8  # the library's gather_rows when the option is 0

# Fields that shape only the forward or only the adjoint schedule.
FORWARD_FIELDS = ("first_kernel", "first_levels", "later_kernel", "later_levels", "tile", "lds_kib",
                  "max_block_rows", "stream_tiles", "gather_rows", "gather_threads", "first_rows",
                  "first_threads")
ADJOINT_FIELDS = ("adjoint_levels", "adjoint_last_levels", "adjoint_last_rows", "adjoint_tile_major",
                  "adjoint_last_threads", "adjoint_rows")
SHARED_FIELDS = ("gather_vecs",)


def forward_shapes():
    """Workgroup shapes of the forward gathers: rows and threads of the later
    passes, rows and threads of a first pass from the input (0: the same)."""
    out = []
    for rows in GATHER_ROWS:
        for threads in GATHER_THREADS:
            if 64 * rows > threads:
                continue
            for first_rows, first_threads in FIRST_SHAPES:
                shape = dict(gather_rows=rows, gather_threads=threads)
                if first_rows:
                    shape.update(first_rows=first_rows, first_threads=first_threads)
                out.append(shape)
    return out


def forward_candidates():
    """Forward schedules worth timing: level-by-level LDS first pass, or a
    gather straight from the input, followed by cache gathers or staged
    gathers."""
    out = []
    for later in (2, 3):
        out.append(dict(first_kernel=2, first_levels=4, later_levels=later))
        out.append(dict(first_kernel=2, first_levels=4, later_levels=later, stream_tiles=1))
        for first in (2, 3, 4):
            out.append(dict(first_kernel=3, first_levels=first, later_levels=later))
        # later passes as staged gathers (each workgroup's term rows in LDS)
        out.append(dict(first_kernel=3, first_levels=3, later_levels=later, later_kernel=1))
    return out


# Adjoint passes that run each row group's tiles back to back: none, the
# first and last (leaves at the largest shifts; one sub-band per workgroup),
# or all.
TILE_MAJOR_MASKS = ("none", "ends", "all")


def adjoint_candidates(rows=GATHER_ROWS_DEFAULT):
    """Adjoint pass depths, channels per workgroup of the last pass (the
    `rows` of the adjoint gathers into planes, or a whole sub-band per
    workgroup), the last pass's workgroup size (1024 threads, or 256 with at
    most 4 channels) and work order."""
    last_rows = [0] + [r for r in (8, 16) if r > rows]
    small = [r for r in ([0] if rows <= 4 else []) + [2, 4] if r != rows]
    shapes = [(r, 0) for r in last_rows] + [(r, 256) for r in small]
    out = []
    for a in (1, 2, 3):
        for b in (1, 2, 3):
            for r, th in shapes:
                for m in TILE_MAJOR_MASKS:
                    c = dict(adjoint_levels=a, adjoint_last_levels=b, adjoint_last_rows=r, adjoint_tile_major=m)
                    if th:
                        c["adjoint_last_threads"] = th
                    out.append(c)
    return out


def tile_major_mask(name, passes):
    """Bitmask over `passes` adjoint passes for a TILE_MAJOR_MASKS name."""
    if name == "none" or passes == 0:
        return 0
    if name == "all":
        return (1 << passes) - 1
    return 1 | (1 << (passes - 1))


def adjoint_gather_passes(plan):
    """Number of adjoint gather passes of a plan."""
    return sum(1 for s in plan.steps(adjoint=True) if s["kind"] == B.STEP_KINDS[8])


def resolve_order(cand, make_plan):
    """Replaces a candidate's work-order name by its bitmask. `make_plan(**opts)`
    builds a plan from schedule options; returns the options, or None when the
    name selects no pass."""
    cand = dict(cand)
    order = cand.pop("adjoint_tile_major", "none")
    if order != "none":
        mask = tile_major_mask(order, adjoint_gather_passes(make_plan(**cand)))
        if mask == 0:
            return None
        cand["adjoint_tile_major"] = mask
    return cand


def arch():
    name = torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName
    return name.split(":")[0]


def nt_bucket(nt):
    b = 1
    while b < nt:
        b *= 2
    return b


def cache_key(arch_name, nf, nt, nd, f_min, f_max, in_dtype, acc_dtype, gamma=-2.0, rule=0):
    law = "" if float(gamma) == -2.0 else f"/gamma{float(gamma):.6g}"
    law += "/twoC" if rule == 1 else ""
    return (f"{arch_name}/nf{nf}/nd{nd}/band{float(f_min):.6g}-{float(f_max):.6g}{law}/"
            f"{_NAMES[in_dtype]}->{_NAMES[acc_dtype]}/nt{nt_bucket(nt)}")


def cache_path(arch_name):
    return os.environ.get("FDMT_TUNE_CACHE") or os.path.join(PKG_DIR, "tuning", f"{arch_name}.json")


def load_cache(arch_name):
    path = cache_path(arch_name)
    if not os.path.exists(path):
        return {}
    with open(path) as f:
        return json.load(f)


def lookup(nf, nt, nd, f_min, f_max, in_dtype, acc_dtype, arch_name=None, gamma=-2.0):
    """Tuned schedule options for this workload, or None."""
    a = arch_name or arch()
    entry = load_cache(a).get(cache_key(a, nf, nt, nd, f_min, f_max, in_dtype, acc_dtype, gamma))
    return None if entry is None else dict(entry["options"])


def _time(fn, reps):
    fn()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        fn()
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps


def ragged_lengths(beams, lo, hi, seed):
    """Beam lengths log-uniform in [lo, hi] (a survey's mix of record lengths)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    return [int(n) for n in np.rint(np.exp(rng.uniform(np.log(lo), np.log(hi), size=beams)))]


def tune(nf, nt, nd, f_min, f_max, in_dtype=torch.float32, acc_dtype=torch.float32, reps=5,
         verbose=False, gamma=-2.0, lengths=None):
    """Times every candidate; returns {"options", "forward_ms", "adjoint_ms", "tried"}.
    With `lengths`, candidates are timed as a ragged batch of beams of those
    lengths (RaggedPlan; nt is then the longest beam)."""
    dev = torch.device("cuda", torch.cuda.current_device())
    gen = torch.Generator(device=dev).manual_seed(1)
    if lengths is not None:
        nt = max(lengths)
    shape_in, shape_out = ((nf * sum(lengths),), (nd * sum(lengths),)) if lengths else ((nf, nt), (nd, nt))
    if in_dtype in (torch.uint8, torch.int32):
        x = torch.randint(0, 256, shape_in, device=dev, dtype=torch.int32, generator=gen).to(in_dtype)
    else:
        x = torch.randn(shape_in, device=dev, generator=gen).to(in_dtype)
    if acc_dtype == torch.int32:
        g = torch.randint(-8, 8, shape_out, device=dev, dtype=torch.int32, generator=gen)
    else:
        g = torch.randn(shape_out, device=dev, generator=gen)
    y = torch.empty(shape_out, device=dev, dtype=acc_dtype)
    xb = torch.empty(shape_in, device=dev, dtype=acc_dtype)

    def runner(p, adjoint):
        if lengths:
            r = B.RaggedPlan(p, lengths)
            ws = r.workspace()
            return (lambda: r.adjoint(g, out=xb, ws=ws)) if adjoint else (lambda: r.forward(x, out=y, ws=ws))
        ws = p.workspace(1)
        return (lambda: p.adjoint(g, out=xb, ws=ws)) if adjoint else (lambda: p.forward(x, out=y, ws=ws))

    tried = []
    best = {}

    def timed(direction, opts, make):
        try:
            p = make(**opts)
            fn = runner(p, direction == "adjoint")
        except B.FDMTError:
            return None  # this schedule does not fit the shape (or the ragged form)
        ms = _time(fn, reps)
        tried.append({"direction": direction, "options": opts, "ms": round(ms, 4)})
        if verbose:
            print(f"{direction} {opts}: {ms:.4f} ms", flush=True)
        return ms

    def make_fwd(**o):
        return B.Plan(nf, nt, nd, f_min, f_max, in_dtype=in_dtype, acc_dtype=acc_dtype, gamma=gamma, **o)

    def make_adj(**o):
        return B.Plan(nf, nt, nd, f_min, f_max, in_dtype=acc_dtype, acc_dtype=acc_dtype, gamma=gamma, **o)

    for vecs in GATHER_VECS:
        # forward: the pass structure at one workgroup shape, then the shapes
        fwd_best, adj_best = None, None
        for cand in forward_candidates():
            opts = dict(cand, gather_vecs=vecs, gather_rows=GATHER_ROWS[0])
            ms = timed("forward", opts, make_fwd)
            if ms is not None and (fwd_best is None or ms < fwd_best[0]):
                fwd_best = (ms, opts)
        if fwd_best is not None:
            structure = {k: v for k, v in fwd_best[1].items() if k not in ("gather_rows", "gather_threads")}
            for shape in forward_shapes():
                opts = dict(structure, **shape)
                if opts == fwd_best[1]:
                    continue
                ms = timed("forward", opts, make_fwd)
                if ms is not None and ms < fwd_best[0]:
                    fwd_best = (ms, opts)
        # adjoint: depths, last-pass shape and work order per row count
        for rows in GATHER_ROWS:
            for cand in adjoint_candidates(rows):
                if lengths and cand["adjoint_tile_major"] != "none":
                    continue  # ragged launches take their work order from the tile maps
                shared = dict(gather_vecs=vecs, adjoint_rows=rows)
                try:
                    c = resolve_order(cand, lambda **o: make_adj(**o, **shared))
                except B.FDMTError:
                    continue
                if c is None:
                    continue
                opts = dict(c, **shared)
                ms = timed("adjoint", opts, make_adj)
                if ms is not None and (adj_best is None or ms < adj_best[0]):
                    adj_best = (ms, opts)
        if fwd_best is None or adj_best is None:
            continue
        total = fwd_best[0] + adj_best[0]
        if not best or total < best["forward_ms"] + best["adjoint_ms"]:
            best = {"options": dict(fwd_best[1], **adj_best[1]),
                    "forward_ms": round(fwd_best[0], 4), "adjoint_ms": round(adj_best[0], 4)}
    if not best:
        raise RuntimeError("no candidate schedule fits this workload")
    best["tried"] = tried
    return best


def store(nf, nt, nd, f_min, f_max, in_dtype, acc_dtype, result, arch_name=None, gamma=-2.0):
    a = arch_name or arch()
    path = cache_path(a)
    cache = load_cache(a)
    cache[cache_key(a, nf, nt, nd, f_min, f_max, in_dtype, acc_dtype, gamma)] = {
        "options": result["options"], "forward_ms": result["forward_ms"],
        "adjoint_ms": result["adjoint_ms"], "tuned_at_nt": int(nt),
        "date": time.strftime("%Y-%m-%d")}
    os.makedirs(os.path.dirname(path), exist_ok=True)
    with open(path, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
        f.write("\n")
    return path


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--nf", type=int, required=True)
    ap.add_argument("--nt", type=int, default=0, help="samples (not used with --ragged)")
    ap.add_argument("--nd", type=int, required=True)
    ap.add_argument("--band", type=float, nargs=2, required=True)
    ap.add_argument("--in-dtype", choices=sorted(DTYPES), default="f32")
    ap.add_argument("--acc-dtype", choices=sorted(DTYPES), default="f32")
    ap.add_argument("--gamma", type=float, default=-2.0, help="delay law dt ~ f^gamma")
    ap.add_argument("--ragged", type=int, nargs=4, metavar=("BEAMS", "LO", "HI", "SEED"),
                    help="time a ragged batch of BEAMS beams, lengths log-uniform in [LO, HI] "
                         "(the entry is stored under Nt = the longest beam)")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--write", action="store_true", help="store the result in the cache")
    ap.add_argument("--out", help="also write the full result (every candidate's time) to this JSON file")
    args = ap.parse_args()
    ind, acc = DTYPES[args.in_dtype], DTYPES[args.acc_dtype]
    lengths = ragged_lengths(*args.ragged) if args.ragged else None
    nt = max(lengths) if lengths else args.nt
    res = tune(args.nf, nt, args.nd, *args.band, ind, acc, reps=args.reps, verbose=True, gamma=args.gamma,
               lengths=lengths)
    print(json.dumps({k: v for k, v in res.items() if k != "tried"}), flush=True)
    if args.out:
        with open(args.out, "w") as f:
            json.dump(dict(res, workload=vars(args)), f, indent=1)
    if args.write:
        print("stored in", store(args.nf, nt, args.nd, *args.band, ind, acc, res, gamma=args.gamma),
              flush=True)


if __name__ == "__main__":
    main()
