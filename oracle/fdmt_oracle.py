"""CPU oracle for the Fast Dispersion Measure Transform and its adjoint.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or
execute this module; only the tests, the smoke check and the benchmark's
CPU-baseline leg use it. It shares no code, headers, tables or constants
with the HIP library.

It follows Zackay & Ofek, "An accurate and efficient algorithm for detection
of radio bursts with an unknown dispersion measure" (arXiv:1411.5373),
Sec. 4 ("The FDMT Algorithm") and Algorithm 1, step by step, in plain NumPy:
one vector add per (iteration, sub-band, delay) row, as in the paper's
vectorised form (caption of Fig. 2). Integer inputs are summed in int64,
floating inputs in float64 after an exact upcast. An explicit `acc=np.float32`
evaluates the same recursion in IEEE binary32 (one rounding per addition, in
the order written here); the paper does not fix a precision, and every
output's sum is a fixed tree of single additions, so this mode is the exact
reference for a binary32 implementation of the same recursion.

Notation. I[f][t]: input, channel 0 = lowest frequency, t contiguous.
A_{f0}^{f2}(t0, dt): sum along the dispersion curve that enters the
sub-band [f0, f2) at time t0 (its lowest frequency) and leaves it dt samples
earlier (Eq. parametrization). All planes are indexed [dt][t0].

Readings where the paper is silent, garbled or inconsistent (each one is
listed with its justification in the design notes):
  R-f1   f1 in the addition rule is the border frequency between the two
         sub-bands, i.e. the midpoint of [f0, f2] (Sec. 4.2, "Dealing with the
         case Nf != 2^k", names it the border frequency; "(f2-f0)/2" is a typo).
  R-t2   the upper half is A_{f1}^{f2}(t1, t1 - t2) (the second statement of the
         rule repeats it as t1 - t0, a typo).
  R-init the Option-1 partial sums run backwards in time,
         A_f^{f+df}(t, dt) = sum_{i=0}^{dt} I(f, t - i): a curve leaves a
         channel earlier at its upper edge, as t1 < t0 in the addition rule.
  R-copy the alternative (copy) rule for t1 < 0 equals treating I as zero at
         negative times; outputs with t0 < dt are partial paths.
  R-round t0 - t1 = C*dt is rounded half up in float64: d_lo = floor(dt*C + 0.5);
         the upper sub-band's delay is dt - d_lo and its shift is d_lo, so the
         two halves meet at one shared sample time t1 = t0 - d_lo.
  R-rows row counts are derived top-down from the Nd output rows, child rows
         = largest index the parent reads + 1 (the paper's dt_max formula is
         its continuous estimate of the same quantity).
  R-fp   1/f^2 is evaluated as 1.0/(f*f); C = (1/f1^2 - 1/f0^2)/(1/f2^2 - 1/f0^2)
         in that order, IEEE float64, no fused multiply-add.
  R-law  another delay law dt ~ f^gamma (Sec. 4.2, other functional forms)
         replaces the power -2 of Eq. (Cf2f0) by gamma and nothing else;
         f^gamma is the C library's pow (gamma = -2 keeps 1.0/(f*f)).
  R-dmin a known smallest delay d_min (Sec. 4.2, different range of
         dispersions) is applied as the frequency-dependent input shift the
         paper names: channel k is delayed by pre_k = round_half_up(d_min *
         phi(c_k)) samples (zero history), phi(f) = (f_min^g - f^g) /
         (f_min^g - f_max^g) at the channel's centre c_k = (e_k + e_k+1)/2, so
         the run a row adds in a channel is centred on the curve's passage
         through it; row dt then follows total delay d_min + dt. The delay
         tables themselves are unchanged.
  R-fft  Algorithm 2 (FFT-FDMT) prints its initialisation with I(f, t + i);
         it is read as Algorithm 1's (reading R-init), since both algorithms
         compute the same transform. Its time axis is zero-padded to
         Nt + Nd - 1 samples, the least padding after which no path wraps.
  R-twoC the two versions of C (Sec. 4.2, rounding and binning), a table rule
         of its own (rule=1): a channel is the point of its label (lower
         edge) e_k and a sub-band's delay runs from its first channel's label
         to its last's. Merging [k0..km-1] and [km..k1]: the lower half's delay
         is d_lo = round_half_up(dt * C_lo), C_lo = C with f1 = e_{km-1} (the
         end frequency of the lower sub-band) and f2 = e_{k1}; the upper half
         starts s = round_half_up(dt * C_hi) back, C_hi = C with f1 = e_{km}
         (the start frequency of the upper sub-band), and spans d_hi = dt - s.
         The curve's travel between the two labels is then the gap s - d_lo.
         A channel alone spans no delay, so each needs only row 0 (its
         samples, the Option-1 sum with no chain) and every output adds one
         sample per channel. Copy nodes and channel-free sub-bands as in
         R-nf. Parity unpinned against the authors' code, which is absent.
  R-nf   Nf need not be a power of two (Sec. 4.2, the case Nf != 2^k): the
         iterations still pair sub-bands 2j and 2j+1, sub-band j of iteration
         l holding channels j*2^l .. min((j+1)*2^l, Nf) - 1, so there are
         ceil(log2 Nf) iterations. A sub-band with no channels has no rows; a
         sub-band whose upper half has no channels is its lower half as it is
         (a copy node); every other merge is between sub-bands of possibly
         unequal width, split at the border frequency f1 between them, with
         f2 the upper edge of the sub-band's last channel.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np


# ----------------------------------------------------------------------------
# Frequency grid and merge coefficient (Sec. 1 Eq. DtD, Sec. 4 Eq. Cf2f0)
# ----------------------------------------------------------------------------

def channel_edges(nf, f_min, f_max):
    """Edges e_k = f_min + k*delta_f, delta_f = (f_max - f_min)/N_f (Sec. 4,
    definition of delta_f under the simple initialization), k = 0..N_f."""
    delta_f = (f_max - f_min) / nf
    return [f_min + k * delta_f for k in range(nf + 1)]


def _inv_sq(f):
    return 1.0 / (f * f)


def _law(f, gamma):
    """f^gamma (reading R-law); the cold-plasma f^-2 as 1.0/(f*f)."""
    return _inv_sq(f) if gamma == -2.0 else math.pow(f, gamma)


def merge_coefficient(f0, f1, f2, gamma=-2.0):
    """Eq. (Cf2f0): C_{f2,f0} = (f1^-2 - f0^-2) / (f2^-2 - f0^-2), the fraction of
    the sub-band delay spent between f0 and the border frequency f1; for the law
    dt ~ f^gamma the power -2 becomes gamma (Sec. 4.2)."""
    return (_law(f1, gamma) - _law(f0, gamma)) / (_law(f2, gamma) - _law(f0, gamma))


def round_half_up(x):
    """Reading R-round: nearest integer, ties upward."""
    return int(math.floor(x + 0.5))


# ----------------------------------------------------------------------------
# Delay tables (Sec. 4: t1 = t0 - C*dt; dt_max decided before the computation)
# ----------------------------------------------------------------------------

@dataclass
class Tables:
    nf: int
    nd: int
    f_min: float
    f_max: float
    levels: int                 # ceil(log2(nf))
    rows: list                  # rows[l][j]: number of dt rows of sub-band j at iteration l
                                # (2^(levels-l) sub-bands; 0 rows for one with no channels)
    split: list                 # split[l][j][dt] = (d_lo, s, d_hi) for l >= 1; d_hi is None
                                # in a copy node (reading R-nf)
    gamma: float = -2.0         # delay law dt ~ f^gamma
    pre: list = None            # per channel: the d_min pre-shift (reading R-dmin)
    rule: int = 0               # 0: one C at the border (R-round); 1: two C's (R-twoC)

    @property
    def leaf_rows(self):
        return self.rows[0]


def build_tables(nf, nd, f_min, f_max, gamma=-2.0, d_min=0, rule=0):
    """Per iteration l = 1..log2(Nf) and sub-band j (channels j*2^l .. (j+1)*2^l - 1,
    f0 = e[j*2^l], f1 = e[(2j+1)*2^(l-1)], f2 = e[(j+1)*2^l]):
        for each dt: t0 - t1 = d_lo = round(C_{f2,f0} * dt)   (lower half's delay)
                     s = d_lo                                  (upper half's start shift)
                     t1 - t2 = d_hi = dt - d_lo                (upper half's delay)
    Row counts run top-down from Nd at the last iteration (reading R-rows).
    gamma: the delay law dt ~ f^gamma (reading R-law). d_min: the smallest
    delay searched (reading R-dmin), which sets the per-channel pre-shift.
    Any Nf >= 1 (reading R-nf): sub-band j of iteration l holds channels
    j*2^l .. min((j+1)*2^l, Nf) - 1; f2 is the upper edge of its last channel.
    rule=1 (reading R-twoC): two coefficients per merge, from the lower
    sub-band's last label and the upper sub-band's first, over the band's
    label span; the lower half's delay and the upper half's shift then
    differ."""
    if nf < 1:
        raise ValueError("Nf must be >= 1")
    if nd < 1:
        raise ValueError("Nd must be >= 1")
    if not (0.0 < f_min < f_max):
        raise ValueError("need 0 < f_min < f_max")
    if not math.isfinite(gamma) or gamma == 0.0:
        raise ValueError("gamma must be finite and nonzero")
    if d_min < 0:
        raise ValueError("d_min must be >= 0")
    if rule not in (0, 1):
        raise ValueError("rule must be 0 (one C) or 1 (two C's)")
    levels = (nf - 1).bit_length()
    e = channel_edges(nf, f_min, f_max)

    def channels(l, j):
        return max(0, min((j + 1) << l, nf) - (j << l))

    rows = [None] * (levels + 1)
    split = [None] * (levels + 1)
    rows[levels] = [nd]
    for l in range(levels, 0, -1):
        nsub = 1 << (levels - l)
        rows[l - 1] = [0] * (2 * nsub)
        split[l] = []
        for j in range(nsub):
            if channels(l, j) == 0:
                split[l].append([])       # no channels, no rows
                continue
            if channels(l - 1, 2 * j + 1) == 0:
                # copy node: the sub-band is its lower half (reading R-nf)
                split[l].append([(dt, 0, None) for dt in range(rows[l][j])])
                rows[l - 1][2 * j] = rows[l][j]
                continue
            triples = []
            if rule == 0:
                f0 = e[j << l]
                f1 = e[(2 * j + 1) << (l - 1)]
                f2 = e[min((j + 1) << l, nf)]
                c = merge_coefficient(f0, f1, f2, gamma)
                for dt in range(rows[l][j]):
                    d_lo = round_half_up(dt * c)
                    triples.append((d_lo, d_lo, dt - d_lo))
            else:
                mid = (2 * j + 1) << (l - 1)            # first channel of the upper half
                first, last = e[j << l], e[min((j + 1) << l, nf) - 1]
                c_lo = merge_coefficient(first, e[mid - 1], last, gamma)
                c_hi = merge_coefficient(first, e[mid], last, gamma)
                for dt in range(rows[l][j]):
                    d_lo = round_half_up(dt * c_lo)
                    s = round_half_up(dt * c_hi)
                    triples.append((d_lo, s, dt - s))
            split[l].append(triples)
            last = triples[-1]
            rows[l - 1][2 * j] = last[0] + 1
            rows[l - 1][2 * j + 1] = last[2] + 1
    pre = [0] * nf
    if d_min > 0:
        den = _law(f_min, gamma) - _law(f_max, gamma)
        for k in range(nf):
            centre = 0.5 * (e[k] + e[k + 1])
            phi = (_law(f_min, gamma) - _law(centre, gamma)) / den
            pre[k] = round_half_up(float(d_min) * phi)
    return Tables(nf, nd, f_min, f_max, levels, rows, split, float(gamma), pre, rule)


# ----------------------------------------------------------------------------
# Forward transform (Algorithm 1)
# ----------------------------------------------------------------------------

def _acc_dtype(x, acc=None):
    """int64 for integer input, float64 for floating input, unless `acc` names
    the accumulation type explicitly (np.float32: the same recursion evaluated
    in IEEE binary32, one rounding per addition, in the order written here)."""
    if acc is not None:
        return np.dtype(acc).type
    return np.int64 if np.asarray(x).dtype.kind in "iub" else np.float64


def initialize(img, tables, acc=None):
    """Option 1 (Sec. 4): A_f^{f+df}(t, dt) = sum_{i=0}^{dt} I(f, t - i) for
    dt = 0..rows[0][k]-1, with I = 0 before the record starts (readings R-init,
    R-copy). Built as the chain A(t, dt) = A(t, dt-1) + I(f, t - dt)."""
    img = np.asarray(img)
    nf, nt = img.shape
    acc = _acc_dtype(img, acc)
    x = img.astype(acc)
    if any(tables.pre):
        # reading R-dmin: channel k's input delayed by pre_k samples
        xs = np.zeros_like(x)
        for k, sh in enumerate(tables.pre):
            if sh < nt:
                xs[k, sh:] = x[k, : nt - sh]
        x = xs
    planes = []
    for k in range(len(tables.rows[0])):
        if k >= nf:
            planes.append(np.zeros((0, nt), dtype=acc))  # no channel here (reading R-nf)
            continue
        n = tables.rows[0][k]
        a = np.zeros((n, nt), dtype=acc)
        a[0] = x[k]
        for dt in range(1, n):
            a[dt] = a[dt - 1]
            if dt < nt:
                a[dt, dt:] += x[k, : nt - dt]
        planes.append(a)
    return planes


def iterate(planes, tables, nt):
    """The iterations of Algorithm 1: for i = 1..log2(Nf), for each sub-band pair,
    for each dt, for each t0:
        A_{f0}^{f2}(t0, dt) = A_{f0}^{f1}(t0, d_lo) + A_{f1}^{f2}(t0 - s, d_hi)   (t0 >= s)
        A_{f0}^{f2}(t0, dt) = A_{f0}^{f1}(t0, d_lo)                             (t0 <  s)
    where the second line is the alternative (copy) rule for t1 = t0 - s < 0.
    A copy node (reading R-nf) is its lower half: A_{f0}^{f2}(t0, dt) = A_{f0}^{f1}(t0, dt)."""
    for l in range(1, tables.levels + 1):
        merged = []
        for j in range(len(planes) // 2):
            lower, upper = planes[2 * j], planes[2 * j + 1]
            out = np.empty((tables.rows[l][j], nt), dtype=lower.dtype)
            for dt, (d_lo, s, d_hi) in enumerate(tables.split[l][j]):
                if d_hi is None:
                    out[dt] = lower[d_lo]
                elif s < nt:
                    out[dt, s:] = lower[d_lo, s:] + upper[d_hi, : nt - s]
                    out[dt, :s] = lower[d_lo, :s]
                else:
                    out[dt] = lower[d_lo]
            merged.append(out)
        planes = merged
    return planes[0]


def fdmt(img, f_min, f_max, nd, tables=None, acc=None):
    """A_{f_min}^{f_max}(t0, dt) for dt = 0..nd-1, t0 = 0..nt-1; shape [nd][nt]."""
    img = np.asarray(img)
    nf, nt = img.shape
    if tables is None:
        tables = build_tables(nf, nd, f_min, f_max)
    return iterate(initialize(img, tables, acc), tables, nt)


def fdmt_batch(imgs, f_min, f_max, nd, acc=None):
    tables = build_tables(imgs.shape[-2], nd, f_min, f_max)
    return np.stack([fdmt(x, f_min, f_max, nd, tables, acc) for x in imgs])


# ----------------------------------------------------------------------------
# Adjoint (transpose of the linear map above, term by term)
# ----------------------------------------------------------------------------

def fdmt_adjoint(grad, f_min, f_max, nf, tables=None, acc=None):
    """Transpose of fdmt(): grad [nd][nt] -> [nf][nt].

    Each forward term out[dt][t0] += lower[d_lo][t0] becomes
    lower_bar[d_lo][t0] += out_bar[dt][t0]; each out[dt][t0] += upper[d_hi][t0 - s]
    (t0 >= s) becomes upper_bar[d_hi][t] += out_bar[dt][t + s] (t + s < nt); each
    init term A(t, dt) += I(f, t - i) becomes I_bar(f, t) += A_bar(t + i, dt).
    Iterations run from the last to the first; within a sub-band, dt ascends."""
    grad = np.asarray(grad)
    nd, nt = grad.shape
    if tables is None:
        tables = build_tables(nf, nd, f_min, f_max)
    acc = _acc_dtype(grad, acc)
    planes = [grad.astype(acc)]
    for l in range(tables.levels, 0, -1):
        split_planes = []
        for j, g in enumerate(planes):
            lo_bar = np.zeros((tables.rows[l - 1][2 * j], nt), dtype=acc)
            hi_bar = np.zeros((tables.rows[l - 1][2 * j + 1], nt), dtype=acc)
            for dt, (d_lo, s, d_hi) in enumerate(tables.split[l][j]):
                lo_bar[d_lo] += g[dt]
                if d_hi is not None and s < nt:
                    hi_bar[d_hi, : nt - s] += g[dt, s:]
            split_planes += [lo_bar, hi_bar]
        planes = split_planes
    out = np.zeros((nf, nt), dtype=acc)
    for k in range(nf):
        a_bar = planes[k]
        sh = tables.pre[k]    # transpose of the R-dmin input delay
        for dt in range(tables.rows[0][k]):
            for i in range(dt + 1):
                if sh + i < nt:
                    out[k, : nt - sh - i] += a_bar[dt, sh + i:]
    return out


# ----------------------------------------------------------------------------
# Path walk: which samples each output adds (used by brute-force checks)
# ----------------------------------------------------------------------------

def path(tables, dt):
    """Descend the tables from output row dt to the channels. Returns per channel
    k the pair (sigma_k, delta_k): channel k contributes I[k][t0 - sigma_k - i]
    for i = 0..delta_k (sigma_k includes the channel's d_min pre-shift)."""
    nodes = [(0, dt)]
    for l in range(tables.levels, 0, -1):
        nxt = []
        for j, node in enumerate(nodes):
            if node is None:              # no channels below (reading R-nf)
                nxt += [None, None]
                continue
            sigma, d = node
            d_lo, s, d_hi = tables.split[l][j][d]
            nxt.append((sigma, d_lo))
            nxt.append(None if d_hi is None else (sigma + s, d_hi))
        nodes = nxt
    assert all(n is not None for n in nodes[:tables.nf]) and all(n is None for n in nodes[tables.nf:])
    return [(sigma + pre, d) for (sigma, d), pre in zip(nodes[:tables.nf], tables.pre)]


def brute_point(img, tables, dt, t0):
    """One output by explicit summation along its path (plain loops)."""
    img = np.asarray(img)
    nt = img.shape[1]
    total = 0 if img.dtype.kind in "iub" else 0.0
    for k, (sigma, delta) in enumerate(path(tables, dt)):
        for i in range(delta + 1):
            t = t0 - sigma - i
            if 0 <= t < nt:
                total += int(img[k, t]) if img.dtype.kind in "iub" else float(img[k, t])
    return total


def brute_row(img, tables, dt):
    """One whole output row by explicit summation along its path, vectorised over t0."""
    img = np.asarray(img)
    nf, nt = img.shape
    acc = _acc_dtype(img)
    out = np.zeros(nt, dtype=acc)
    for k, (sigma, delta) in enumerate(path(tables, dt)):
        for i in range(delta + 1):
            sh = sigma + i
            if sh < nt:
                out[sh:] += img[k, : nt - sh].astype(acc)
    return out


def brute_ideal(img, f_min, f_max, nd, gamma=-2.0):
    """Brute-force dedispersion along the exact law (prior-art comparator, Sec. 3):
    each channel contributes I[k][t0 - round(dt * phi(centre_k))]."""
    img = np.asarray(img)
    nf, nt = img.shape
    e = channel_edges(nf, f_min, f_max)
    acc = _acc_dtype(img)
    out = np.zeros((nd, nt), dtype=acc)
    den = _law(f_min, gamma) - _law(f_max, gamma)
    for k in range(nf):
        centre = 0.5 * (e[k] + e[k + 1])
        phi = (_law(f_min, gamma) - _law(centre, gamma)) / den
        for dt in range(nd):
            sh = round_half_up(dt * phi)
            if sh < nt:
                out[dt, sh:] += img[k, : nt - sh].astype(acc)
    return out


# ----------------------------------------------------------------------------
# FFT-FDMT (Algorithm 2): the same iterations with the time axis Fourier
# transformed, where a shift by s becomes a product with the shift vector
# V(w, s), the transform of a unit impulse at s.
# ----------------------------------------------------------------------------

def fft_length(nt, nd):
    """Zero padding (Algorithm 2 comments): shifts become cyclic, so the time
    axis is padded with at least Nd - 1 zeros; a path's samples lie in
    [t0 - dt, t0] with dt <= Nd - 1, so nothing wraps onto the record."""
    return nt + nd - 1


def shift_vector(n, s):
    """V(w, s) = F(delta_s)(w) for w = 0..n//2 (real-input half spectrum)."""
    w = np.arange(n // 2 + 1)
    return np.exp(-2j * np.pi * ((w * s) % n) / n)


def fdmt_fft(img, f_min, f_max, nd, tables=None, n=None):
    """Algorithm 2 in complex128: the Option-1 rows of every channel (reading
    R-init, and R-dmin's pre-shift), zero-padded to n samples and Fourier
    transformed along time; every iteration adds B_lo(w, d_lo) + B_hi(w, d_hi) *
    V(w, s) (a copy node, reading R-nf, keeps B_lo); the last plane is
    transformed back and cut to the record. With n >= fft_length(nt, nd) it
    equals fdmt() up to rounding; a shorter n wraps the tail of the record
    onto its start."""
    img = np.asarray(img)
    nf, nt = img.shape
    if tables is None:
        tables = build_tables(nf, nd, f_min, f_max)
    n = fft_length(nt, nd) if n is None else n
    planes = []
    for a in initialize(img.astype(np.float64), tables):
        padded = np.zeros((a.shape[0], n))
        padded[:, :nt] = a
        planes.append(np.fft.rfft(padded, axis=1))
    for l in range(1, tables.levels + 1):
        merged = []
        for j in range(len(planes) // 2):
            lower, upper = planes[2 * j], planes[2 * j + 1]
            out = np.empty((tables.rows[l][j], n // 2 + 1), dtype=np.complex128)
            for dt, (d_lo, s, d_hi) in enumerate(tables.split[l][j]):
                out[dt] = lower[d_lo] if d_hi is None else lower[d_lo] + upper[d_hi] * shift_vector(n, s)
            merged.append(out)
        planes = merged
    return np.fft.irfft(planes[0], n=n, axis=1)[:, :nt]


# ----------------------------------------------------------------------------
# Boxcar search on the output (Sec. 4.2, pulse profile: a profile common to all
# frequencies commutes with the transform, so several widths share one FDMT)
# ----------------------------------------------------------------------------

def boxcar(plane, w):
    """b_w[t] = y[t] + y[t-1] + ... + y[t-w+1] over the last axis, with y = 0
    before t = 0: the causal boxcar of width w by its definition, in float64."""
    y = np.asarray(plane, dtype=np.float64)
    nt = y.shape[-1]
    b = np.zeros_like(y)
    for i in range(min(w, nt)):
        b[..., i:] += y[..., : nt - i]
    return b


def boxcar_search(plane, max_log2, acc=None):
    """For every row of plane[..., nd, nt] and width w = 2^j, j = 0..max_log2:
    b_w[t] = y[t] + y[t-1] + ... + y[t-w+1] (y = 0 before t = 0), its largest
    value and the first t where it occurs, its mean and population standard
    deviation over t = 0..nt-1, and snr = (peak - mean) / stdev (0 if stdev is 0).

    Default: b_w by that definition in float64. acc=np.float32: b_w in binary32
    as the doubling tree b_2w[t] = b_w[t] + b_w[t-w] from b_1 = y, the exact
    reference for a binary32 implementation of that tree. The statistics are
    float64 in both modes. Returns a dict of arrays [..., max_log2 + 1, nd]."""
    y = np.asarray(plane)
    nt = y.shape[-1]
    widths = [1 << j for j in range(max_log2 + 1)]
    sums = []
    if acc is None:
        sums = [boxcar(y, w) for w in widths]
    else:
        b = y.astype(acc)
        sums.append(b.copy())
        for w in widths[:-1]:
            nb = b.copy()
            if w < nt:
                nb[..., w:] = (b[..., w:] + b[..., : nt - w]).astype(acc)
            b = nb
            sums.append(b.copy())
    out = {"peak": [], "t": [], "mean": [], "stdev": [], "snr": []}
    for b in sums:
        b64 = b.astype(np.float64)
        t = np.argmax(b64, axis=-1)          # first maximum
        peak = np.take_along_axis(b64, t[..., None], axis=-1)[..., 0]
        mean = b64.sum(axis=-1) / nt
        sd = np.sqrt(((b64 - mean[..., None]) ** 2).sum(axis=-1) / nt)
        snr = np.where(sd > 0, (peak - mean) / np.where(sd > 0, sd, 1.0), 0.0)
        for k, v in zip(("peak", "t", "mean", "stdev", "snr"), (peak, t, mean, sd, snr)):
            out[k].append(v)
    return {k: np.stack(v, axis=-2) for k, v in out.items()}


def boxcar_candidates(plane, max_log2, threshold, block=2048):
    """Candidate events of the boxcar search (Sec. 1: a detection is a
    statistic above a threshold; Sec. 4.2, pulse profile: one transform serves
    every width). For every beam b, row dt, width w = 2^j and block of
    `block` samples [k*block, (k+1)*block) of the record: the block's largest
    b_w (its first time t), and its S/N = (peak - mean) / stdev with the row's
    mean and stdev of b_w over the whole record (0 if stdev is 0); a block
    whose S/N is at least `threshold` is one candidate. Float64, b_w by its
    definition. Returns a list of (b, dt, j, t, peak, snr), in that order of
    loops (b, j, dt, k)."""
    y = np.asarray(plane, dtype=np.float64)
    if y.ndim == 2:
        y = y[None]
    nb, nd, nt = y.shape
    out = []
    for b in range(nb):
        for j in range(max_log2 + 1):
            bw = boxcar(y[b], 1 << j)
            mean = bw.mean(axis=1)
            sd = bw.std(axis=1)
            for dt in range(nd):
                for k in range(0, nt, block):
                    seg = bw[dt, k: k + block]
                    i = int(np.argmax(seg))
                    peak = float(seg[i])
                    snr = (peak - mean[dt]) / sd[dt] if sd[dt] > 0 else 0.0
                    if snr >= threshold:
                        out.append((b, dt, j, k + i, peak, snr))
    return out

