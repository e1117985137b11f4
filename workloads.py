"""Seeded synthetic inputs for the FDMT workloads.

This module is shared by the tests, the benchmark and the CPU oracle's
callers. It only draws random numbers and places dispersed pulses on the
time-frequency plane; it contains none of the transform's arithmetic (no
merge coefficients, no delay tables, no sums along curves).

Conventions (Zackay & Ofek, Sec. 1 and Sec. 4):
  * the input is I[f][t] with the time axis contiguous;
  * channel k covers [e_k, e_k + df), e_k = f_min + k*df, df = (f_max-f_min)/Nf,
    channel 0 is the lowest frequency;
  * a pulse with total band delay `dt` samples that reaches the lowest
    frequency at sample T reaches frequency f at T - dt*phi(f), where
    phi(f) = (f_min^-2 - f^-2) / (f_min^-2 - f_max^-2) is the dispersion law
    of Eq. (DtD) normalised to the band (higher frequencies arrive earlier).

Each workload below is the synthetic stand-in for one measured
configuration: the paper's data are not public, so noise + injected pulses
of the stated shapes and distributions are used instead.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

SEED_BASE = 14115373


@dataclass(frozen=True)
class Workload:
    name: str
    nf: int
    nt: int            # samples per beam (0 for the ragged workload)
    nd: int            # delay trials = output rows
    f_min: float       # GHz
    f_max: float       # GHz
    batch: int = 1
    description: str = ""
    extra: dict = field(default_factory=dict)


WORKLOADS = {
    "c1": Workload("c1", 64, 1024, 64, 1.2, 1.6, 1,
                   "FP32, Nf=64, Nt=1024, Nd=64, 1 pulse of 5 sigma sweeping 40 samples"),
    "c2": Workload("c2", 1024, 8192, 1024, 1.2, 1.6, 1,
                   "FP32, Nf=1024, Nt=8192, Nd=1024, 8 pulses of 3-10 sigma"),
    "c3": Workload("c3", 4096, 65536, 2048, 1.2, 1.6, 1,
                   "precision form, Nf=4096, Nt=65536, Nd=2048; uint8 N(64,8) and FP16 N(0,1); 16 pulses"),
    "c4": Workload("c4", 1024, 0, 512, 1.2, 1.6, 256,
                   "ragged batch: 256 beams, Nf=1024, Nd=512, Nt log-uniform in [2048, 32768]"),
    "c5": Workload("c5", 1024, 16384, 1024, 0.4, 0.8, 16,
                   "differentiable form: batch 16, Nf=1024, Nt=16384, Nd=1024, 0.4-0.8 GHz"),
}


def band_fraction(f, f_min, f_max, gamma=-2.0):
    """Fraction of the full-band delay reached at frequency f, for the delay law
    dt ~ f^gamma (-2: cold-plasma dispersion)."""
    f = np.asarray(f, dtype=np.float64)
    return (f_min ** gamma - f ** gamma) / (f_min ** gamma - f_max ** gamma)


def channel_centres(nf, f_min, f_max):
    df = (f_max - f_min) / nf
    return f_min + (np.arange(nf, dtype=np.float64) + 0.5) * df


def pulse_samples(nf, f_min, f_max, dt, t_arr, gamma=-2.0):
    """Per-channel sample index of a width-1 pulse: round(T - dt*phi(centre_k))."""
    frac = band_fraction(channel_centres(nf, f_min, f_max), f_min, f_max, gamma)
    return np.rint(t_arr - dt * frac).astype(np.int64)


def inject_pulses(img, f_min, f_max, pulses, scale=1.0, gamma=-2.0):
    """Add each pulse (dt, T, amp) to img[nf][nt] in place (amp*scale per channel)."""
    nf, nt = img.shape
    rows = np.arange(nf)
    for dt, t_arr, amp in pulses:
        ts = pulse_samples(nf, f_min, f_max, dt, t_arr, gamma)
        ok = (ts >= 0) & (ts < nt)
        np.add.at(img, (rows[ok], ts[ok]), img.dtype.type(amp * scale))
    return img


def draw_pulses(rng, count, nd, nt, amp_lo=3.0, amp_hi=10.0, dt=None, amp=None):
    """Pulse parameters: dt ~ U{0..nd-1} (or fixed), T ~ U{nd..nt-1} so the whole
    sweep lies inside the record, amp ~ U(amp_lo, amp_hi) (or fixed)."""
    out = []
    for _ in range(count):
        d = int(rng.integers(0, nd)) if dt is None else int(dt)
        t_arr = int(rng.integers(nd, nt))
        a = float(rng.uniform(amp_lo, amp_hi)) if amp is None else float(amp)
        out.append((d, t_arr, a))
    return out


def random_input(shape, dtype, seed, lo=0, hi=255):
    """Generic seeded input for parity tests: integers in [lo, hi] for integer
    dtypes, N(0,1) otherwise."""
    rng = np.random.default_rng(seed)
    dtype = np.dtype(dtype)
    if dtype.kind in "iu":
        return rng.integers(lo, hi + 1, size=shape).astype(dtype)
    return rng.standard_normal(shape, dtype=np.float32).astype(dtype)


def make_c1(seed=SEED_BASE + 0):
    w = WORKLOADS["c1"]
    rng = np.random.default_rng(seed)
    img = rng.standard_normal((w.nf, w.nt), dtype=np.float32)
    pulses = draw_pulses(rng, 1, w.nd, w.nt, dt=40, amp=5.0)
    inject_pulses(img, w.f_min, w.f_max, pulses)
    return img, pulses


def make_c2(seed=SEED_BASE + 1):
    w = WORKLOADS["c2"]
    rng = np.random.default_rng(seed)
    img = rng.standard_normal((w.nf, w.nt), dtype=np.float32)
    pulses = draw_pulses(rng, 8, w.nd, w.nt)
    inject_pulses(img, w.f_min, w.f_max, pulses)
    return img, pulses


def make_c3(seed=SEED_BASE + 2, nt=None):
    """Returns (u8 image, f16 image, pulses). Both images carry the same noise
    and pulses: u8 = clip(rint(64 + 8*x), 0, 255), f16 = x as float16."""
    w = WORKLOADS["c3"]
    nt = w.nt if nt is None else nt
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((w.nf, nt), dtype=np.float32)
    pulses = draw_pulses(rng, 16, w.nd, nt)
    inject_pulses(x, w.f_min, w.f_max, pulses)
    u8 = np.clip(np.rint(64.0 + 8.0 * x), 0, 255).astype(np.uint8)
    f16 = x.astype(np.float16)
    return u8, f16, pulses


def make_c3_f32(seed=SEED_BASE + 2, nt=None):
    """The FP32 form of the Nf=4096 workload: the same N(0,1) noise and pulses
    as make_c3, before quantisation."""
    w = WORKLOADS["c3"]
    nt = w.nt if nt is None else nt
    rng = np.random.default_rng(seed)
    x = rng.standard_normal((w.nf, nt), dtype=np.float32)
    pulses = draw_pulses(rng, 16, w.nd, nt)
    inject_pulses(x, w.f_min, w.f_max, pulses)
    return x


def c4_lengths(seed=SEED_BASE + 3, beams=256, lo=2048, hi=32768):
    rng = np.random.default_rng(seed)
    return np.rint(np.exp(rng.uniform(math.log(lo), math.log(hi), size=beams))).astype(np.int64)


def make_c4_beam(b, nt, seed=SEED_BASE + 3):
    """Beam b of the ragged workload: N(0,1) FP32 plus U{0,1,2} pulses."""
    w = WORKLOADS["c4"]
    rng = np.random.default_rng([seed, b])
    img = rng.standard_normal((w.nf, int(nt)), dtype=np.float32)
    pulses = draw_pulses(rng, int(rng.integers(0, 3)), w.nd, int(nt))
    inject_pulses(img, w.f_min, w.f_max, pulses)
    return img, pulses


def make_c5(seed=SEED_BASE + 4, batch=None, nf=None, nt=None):
    w = WORKLOADS["c5"]
    rng = np.random.default_rng(seed)
    shape = (w.batch if batch is None else batch, w.nf if nf is None else nf,
             w.nt if nt is None else nt)
    return rng.standard_normal(shape, dtype=np.float32)


def torch_noise(shape, seed, device, kind="normal"):
    """Device-side generator for full-size benchmark inputs (same distributions,
    torch's Philox stream instead of numpy's PCG64)."""
    import torch
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    if kind == "normal":
        return torch.randn(shape, generator=g, device=device, dtype=torch.float32)
    if kind == "u8":
        x = torch.randn(shape, generator=g, device=device, dtype=torch.float32)
        return torch.clamp(torch.round(64.0 + 8.0 * x), 0, 255).to(torch.uint8)
    raise ValueError(kind)
