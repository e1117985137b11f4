"""Pins for the CPU oracle: each test ties it to something other than itself
(a hand-worked example, a closed form, a bound from the dispersion law, an
invariant of the transform, brute force on tiny inputs, or a textbook
reduction). Together they are chosen so that a dropped term, a wrong sign or
index, or a swapped operand in the oracle fails at least one of them."""
import math

import numpy as np
import pytest

from conftest import read_golden
from oracle import (boxcar_search, brute_ideal, brute_point, brute_row, build_tables, channel_edges, fdmt,
                    fdmt_adjoint, fdmt_fft, fft_length, path)
import workloads as W

BANDS = [(1.2, 1.6), (0.4, 0.8), (1.0, 2.0)]


def _rng(seed):
    return np.random.default_rng(seed)


# ---------------------------------------------------------------- worked examples

@pytest.mark.parametrize("name", ["tiny_nf2_nd3.txt", "tiny_nf4_nd4.txt", "tiny_nf3_nd4.txt"])
def test_hand_derived_examples(name):
    """Hand-derived outputs of one and two iterations (fixtures cite the
    addition rule, Eq. Cf2f0 and Option-1 init); pins direction of shifts,
    which half is shifted, and the per-sub-band f0/f1/f2."""
    f_min, f_max, nd, img, expect = read_golden(name)
    np.testing.assert_array_equal(fdmt(img, f_min, f_max, nd), expect)


# ---------------------------------------------------------------- delay tables

@pytest.mark.parametrize("nf,nd", [(2, 3), (8, 8), (64, 64), (256, 100), (1024, 1024), (4096, 2048),
                                   (3, 4), (6, 20), (100, 90), (1000, 1024)])
@pytest.mark.parametrize("band", BANDS)
def test_table_invariants(nf, nd, band):
    """Each split is a partition of the delay (d_lo + d_hi = dt, s = d_lo), the
    maps are monotone with unit steps, and every child row exists. With Nf not
    a power of two (Sec. 4.2), sub-band j of iteration l has rows exactly when
    it holds a channel, and one whose upper half holds none passes its rows
    straight down."""
    t = build_tables(nf, nd, *band)
    assert t.rows[t.levels] == [nd] and t.levels == math.ceil(math.log2(nf))
    for l in range(1, t.levels + 1):
        for j, trip in enumerate(t.split[l]):
            assert len(trip) == t.rows[l][j]
            assert (t.rows[l][j] > 0) == (j << l < nf)
            if trip and trip[0][2] is None:  # upper half without channels
                assert (2 * j + 1) << (l - 1) >= nf and t.rows[l - 1][2 * j + 1] == 0
                assert [x[0] for x in trip] == list(range(len(trip))) and t.rows[l - 1][2 * j] == len(trip)
                continue
            if not trip:
                continue
            assert (2 * j + 1) << (l - 1) < nf
            prev = None
            for dt, (d_lo, s, d_hi) in enumerate(trip):
                assert 0 <= d_lo <= dt and s == d_lo and d_lo + d_hi == dt
                assert d_lo < t.rows[l - 1][2 * j] and d_hi < t.rows[l - 1][2 * j + 1]
                if prev is not None:
                    assert d_lo - prev[0] in (0, 1) and d_hi - prev[2] in (0, 1)
                prev = (d_lo, s, d_hi)
            assert trip[-1][0] + 1 == t.rows[l - 1][2 * j]
            assert trip[-1][2] + 1 == t.rows[l - 1][2 * j + 1]


@pytest.mark.parametrize("nf,nd", [(16, 40), (64, 64), (1024, 1024), (4096, 2048), (12, 40), (1000, 1024),
                                   (336, 500)])
@pytest.mark.parametrize("band", BANDS)
def test_path_follows_dispersion_law(nf, nd, band):
    """Closed-form bound from Eq. (DtD): along every output path the start shift
    of channel k deviates from the exact law dt*phi(e_k) by at most
    log2(Nf)/2 samples (each iteration rounds once, by <= 1/2, and carries a
    convex combination of its parent's errors). The runs of consecutive
    channels tile [t0 - dt, t0], sharing one sample per channel border."""
    f_min, f_max = band
    t = build_tables(nf, nd, f_min, f_max)
    e = np.array([f_min + k * (f_max - f_min) / nf for k in range(nf)])
    phi = (f_min ** -2 - e ** -2) / (f_min ** -2 - f_max ** -2)
    bound = 0.5 * t.levels + 1e-9
    step = max(1, nd // 97)
    for dt in list(range(0, nd, step)) + [nd - 1]:
        p = np.array(path(t, dt))
        sig, dlt = p[:, 0], p[:, 1]
        assert sig[0] == 0
        np.testing.assert_array_equal(sig[1:], sig[:-1] + dlt[:-1])
        assert sig[-1] + dlt[-1] == dt
        assert np.max(np.abs(sig - dt * phi)) <= bound


@pytest.mark.parametrize("gamma", [-1.0, 1.0, 2.0, -3.5])
@pytest.mark.parametrize("nf,nd", [(16, 40), (256, 300), (1024, 1024), (100, 300)])
@pytest.mark.parametrize("band", BANDS)
def test_path_follows_power_law(gamma, nf, nd, band):
    """Another delay law dt ~ f^gamma (Sec. 4.2, other functional forms): the
    tables built with gamma keep every path within log2(Nf)/2 samples of
    dt*phi_gamma(e_k), phi_gamma(f) = (f_min^g - f^g)/(f_min^g - f_max^g), and
    the runs still tile [t0 - dt, t0]; the -2 law's phi misses them."""
    f_min, f_max = band
    t = build_tables(nf, nd, f_min, f_max, gamma=gamma)
    e = np.array([f_min + k * (f_max - f_min) / nf for k in range(nf)])
    phi = (f_min ** gamma - e ** gamma) / (f_min ** gamma - f_max ** gamma)
    phi2 = (f_min ** -2 - e ** -2) / (f_min ** -2 - f_max ** -2)
    bound = 0.5 * t.levels + 1e-9
    worst2 = 0.0
    for dt in list(range(0, nd, max(1, nd // 53))) + [nd - 1]:
        p = np.array(path(t, dt))
        sig, dlt = p[:, 0], p[:, 1]
        assert sig[0] == 0
        np.testing.assert_array_equal(sig[1:], sig[:-1] + dlt[:-1])
        assert sig[-1] + dlt[-1] == dt
        assert np.max(np.abs(sig - dt * phi)) <= bound
        worst2 = max(worst2, np.max(np.abs(sig - dt * phi2)))
    if nd >= 300:
        assert worst2 > bound


@pytest.mark.parametrize("nf,nd", [(8, 50), (512, 700)])
def test_linear_law_splits_in_half(nf, nd):
    """dt ~ f (gamma = 1): equal sub-bands take equal delays, so every merge
    coefficient is 1/2 and d_lo is dt/2 rounded (either way at odd dt, where
    dt*C sits within rounding of a half)."""
    t = build_tables(nf, nd, 1.2, 1.6, gamma=1.0)
    for l in range(1, t.levels + 1):
        for trip in t.split[l]:
            for dt, (d_lo, s, d_hi) in enumerate(trip):
                assert d_lo in (dt // 2, (dt + 1) // 2) and s == d_lo and d_lo + d_hi == dt
                if dt % 2 == 0:
                    assert d_lo == dt // 2


@pytest.mark.parametrize("gamma", [-1.0, 2.0])
def test_power_law_pulses_recovered(gamma):
    """Width-1 pulses placed along dt ~ f^gamma peak at their (dt, T) in the
    transform built for that law and sum to Nf there by brute force along it."""
    nf, nd, band = 256, 256, (1.2, 1.6)
    rng = _rng(int(10 * gamma) + 99)
    nt = nd + 200
    tab = build_tables(nf, nd, *band, gamma=gamma)
    for dt in [0, nd // 3, nd - 1]:
        t_arr = int(rng.integers(nd, nt))
        img = np.zeros((nf, nt), dtype=np.int64)
        W.inject_pulses(img, band[0], band[1], [(dt, t_arr, 1.0)], gamma=gamma)
        out = fdmt(img, band[0], band[1], nd, tab)
        i, j = np.unravel_index(np.argmax(out), out.shape)
        assert abs(i - dt) <= 2 and abs(j - t_arr) <= 2, (dt, t_arr, i, j)
        assert out[i, j] >= 0.6 * nf
        assert brute_ideal(img, band[0], band[1], nd, gamma=gamma)[dt, t_arr] == nf


def test_work_below_paper_bound():
    """Sec. 4.1: additions <= 2*Nf*Nt + Nt*Nd*log2(Nf) (per unit Nt)."""
    for nf, nd in [(64, 64), (1024, 1024), (4096, 2048), (1024, 512)]:
        t = build_tables(nf, nd, 1.2, 1.6)
        adds = sum(sum(r) for r in t.rows[1:]) + sum(n - 1 for n in t.rows[0])
        assert adds <= 2 * nf + nd * t.levels


# ---------------------------------------------------------------- recursion

@pytest.mark.parametrize("nf,nt,nd", [(1, 20, 7), (2, 16, 5), (8, 40, 12), (16, 64, 30), (32, 50, 64),
                                      (3, 20, 9), (7, 30, 20), (20, 50, 40)])
@pytest.mark.parametrize("band", BANDS)
def test_recursion_equals_path_brute_force(nf, nt, nd, band):
    """Bottom-up recursion == top-down path summation, exact in int64, including
    partial paths (t0 < dt: copy rule) and Nt < Nd."""
    img = _rng(nf * 1000 + nt).integers(-50, 200, size=(nf, nt))
    t = build_tables(nf, nd, *band)
    out = fdmt(img, band[0], band[1], nd, t)
    for dt in range(nd):
        np.testing.assert_array_equal(out[dt], brute_row(img, t, dt))
    for dt, t0 in [(0, 0), (nd - 1, nt - 1), (nd // 2, nt // 3), (nd - 1, 0)]:
        assert out[dt, t0] == brute_point(img, t, dt, t0)


@pytest.mark.parametrize("nf,nd", [(8, 8), (64, 64), (256, 300), (5, 9), (100, 64)])
def test_zero_delay_row_is_channel_sum(nf, nd):
    """At dt = 0 the curve is vertical: row 0 = sum over frequencies of I[f][t0]."""
    img = _rng(nf).integers(0, 256, size=(nf, 300))
    np.testing.assert_array_equal(fdmt(img, 1.2, 1.6, nd)[0], img.sum(axis=0))


@pytest.mark.parametrize("nf,nd", [(4, 9), (64, 64), (128, 200), (3, 7), (100, 120), (257, 64)])
def test_all_ones_closed_form(nf, nd):
    """A complete path (t0 >= dt) through all-ones data adds Nf + dt samples
    (Nf channel runs whose lengths add to dt + Nf); no term is dropped or doubled."""
    nt = nd + 40
    out = fdmt(np.ones((nf, nt), dtype=np.int64), 1.2, 1.6, nd)
    for dt in range(nd):
        np.testing.assert_array_equal(out[dt, dt:], nf + dt)


def test_single_channel_is_running_box_sum():
    """Nf = 1 (no iterations): A(t0, dt) = sum_{i=0}^{dt} I(t0 - i), i.e. a
    difference of cumulative sums (textbook moving sum)."""
    x = _rng(5).integers(-9, 10, size=(1, 64))
    out = fdmt(x, 1.2, 1.6, 20)
    c = np.concatenate([[0], np.cumsum(x[0])])
    for dt in range(20):
        t0 = np.arange(64)
        expect = c[t0 + 1] - c[np.maximum(t0 - dt, 0)]
        np.testing.assert_array_equal(out[dt], expect)


def test_linearity_exact():
    a = _rng(1).integers(-100, 100, size=(32, 80))
    b = _rng(2).integers(-100, 100, size=(32, 80))
    fa, fb = fdmt(a, 1.2, 1.6, 40), fdmt(b, 1.2, 1.6, 40)
    np.testing.assert_array_equal(fdmt(3 * a - 2 * b, 1.2, 1.6, 40), 3 * fa - 2 * fb)


def test_time_shift_equivariance():
    """Delaying every channel by tau (zero fill) delays every output row by tau."""
    x = _rng(3).integers(0, 50, size=(16, 100))
    tau = 13
    xs = np.zeros_like(x)
    xs[:, tau:] = x[:, :-tau]
    a, b = fdmt(x, 1.2, 1.6, 24), fdmt(xs, 1.2, 1.6, 24)
    np.testing.assert_array_equal(b[:, tau:], a[:, :-tau])
    np.testing.assert_array_equal(b[:, :tau], 0)


def test_causal_window():
    """Output (dt, t0) reads only input times in [t0 - dt, t0]."""
    nf, nt, nd = 16, 90, 30
    x = _rng(4).integers(0, 50, size=(nf, nt))
    base = fdmt(x, 1.2, 1.6, nd)
    tp = 40
    y = x.copy()
    y[:, tp] += 1000
    diff = fdmt(y, 1.2, 1.6, nd) - base
    for dt in range(nd):
        assert np.all(diff[dt, :tp] == 0)
        assert np.all(diff[dt, tp + dt + 1:] == 0)
        assert diff[dt, tp] != 0  # channel 0 is always read at t0


def test_commutes_with_causal_time_filter():
    """Sec. 4.2 (pulse profile): convolving every channel's time series with the
    same profile commutes with the transform (exact in integers)."""
    x = _rng(6).integers(-20, 20, size=(32, 120))
    h = np.array([3, -1, 2, 5])

    def filt(a):
        out = np.zeros_like(a)
        for i, hi in enumerate(h):
            out[..., i:] += hi * a[..., : a.shape[-1] - i]
        return out

    np.testing.assert_array_equal(fdmt(filt(x), 1.2, 1.6, 48), filt(fdmt(x, 1.2, 1.6, 48)))


def test_blocked_streaming_equals_one_shot():
    """Processing time in blocks with Nd-1 samples of history per channel
    reproduces the one-shot transform exactly (outputs only look back dt)."""
    nf, nt, nd = 32, 400, 50
    x = _rng(7).integers(0, 255, size=(nf, nt))
    full = fdmt(x, 1.2, 1.6, nd)
    for t_start, t_end in [(0, 130), (130, 131), (131, 290), (290, 400)]:
        h = max(0, t_start - (nd - 1))
        blk = fdmt(x[:, h:t_end], 1.2, 1.6, nd)
        np.testing.assert_array_equal(blk[:, t_start - h:], full[:, t_start:t_end])


def test_init_rows_are_partial_sums():
    """Option-1 init (with the backward-in-time reading) is what a single-channel
    sub-band holds: with Nf = 1 the output equals the partial sums directly."""
    x = np.array([[1, 2, 4, 8, 16]])
    out = fdmt(x, 1.0, 2.0, 3)
    np.testing.assert_array_equal(out, [[1, 2, 4, 8, 16], [1, 3, 6, 12, 24], [1, 3, 7, 14, 28]])


# ---------------------------------------------------------------- pulse recovery

def test_c1_pulse_recovered():
    """A dispersed pulse (Eq. DtD) peaks at its (dt, T) in the transform."""
    img, pulses = W.make_c1()
    w = W.WORKLOADS["c1"]
    out = fdmt(img, w.f_min, w.f_max, w.nd)
    dt, t_arr, amp = pulses[0]
    i, j = np.unravel_index(np.argmax(out), out.shape)
    assert abs(i - dt) <= 2 and abs(j - t_arr) <= 2
    assert out[i, j] >= 0.6 * w.nf * amp


@pytest.mark.parametrize("nf,nd,band", [(256, 256, (1.2, 1.6)), (256, 512, (0.4, 0.8)), (1024, 300, (1.2, 1.6)),
                                        (1000, 512, (1.2, 1.6)), (336, 300, (0.4, 0.8))])
def test_noiseless_pulses_recovered(nf, nd, band):
    """Noiseless width-1 pulses at several delays: the transform's peak sits within
    2 samples of the truth in both axes (2*Nd/Nf in delay when Nd > Nf, where each
    channel spans several delay samples and neighbouring delays tie) and captures
    >= 60% of the pulse; the brute-force law integration (Sec. 3) captures all of
    it at the truth."""
    rng = _rng(nf + nd)
    nt = nd + 200
    tol_dt = 2 * max(1, nd // nf)
    for dt in [0, nd // 5, nd // 2, nd - 1]:
        t_arr = int(rng.integers(nd, nt))
        img = np.zeros((nf, nt), dtype=np.int64)
        W.inject_pulses(img, band[0], band[1], [(dt, t_arr, 1.0)])
        out = fdmt(img, band[0], band[1], nd)
        i, j = np.unravel_index(np.argmax(out), out.shape)
        assert abs(i - dt) <= tol_dt and abs(j - t_arr) <= 2, (dt, t_arr, i, j)
        assert out[i, j] >= 0.6 * nf
    ideal = brute_ideal(img, band[0], band[1], nd)
    assert ideal[dt, t_arr] == nf


# ---------------------------------------------------------------- adjoint

@pytest.mark.parametrize("nf,nt,nd", [(1, 30, 9), (8, 40, 16), (32, 64, 64), (64, 50, 90), (3, 30, 9), (12, 40, 30),
                                      (100, 50, 64)])
@pytest.mark.parametrize("band", [(1.2, 1.6), (0.4, 0.8)])
def test_adjoint_dot_product_exact(nf, nt, nd, band):
    """<A x, y> = <x, A^T y>, exact in int64."""
    rng = _rng(nf * 7 + nt)
    x = rng.integers(-30, 30, size=(nf, nt))
    y = rng.integers(-30, 30, size=(nd, nt))
    ax = fdmt(x, band[0], band[1], nd)
    aty = fdmt_adjoint(y, band[0], band[1], nf)
    assert int(np.sum(ax * y)) == int(np.sum(x * aty))


def test_adjoint_matches_explicit_matrix():
    """A^T from the adjoint equals the transpose of the matrix assembled column by
    column from forward transforms of unit impulses."""
    nf, nt, nd = 8, 12, 10
    cols = []
    for k in range(nf):
        for t in range(nt):
            e = np.zeros((nf, nt), dtype=np.int64)
            e[k, t] = 1
            cols.append(fdmt(e, 1.2, 1.6, nd).ravel())
    a = np.stack(cols, axis=1)
    for r in range(nd * nt):
        y = np.zeros(nd * nt, dtype=np.int64)
        y[r] = 1
        np.testing.assert_array_equal(fdmt_adjoint(y.reshape(nd, nt), 1.2, 1.6, nf).ravel(), a[r])


def _lse(z):
    m = z.max()
    return m + math.log(np.exp(z - m).sum())


def test_adjoint_finite_differences_fp64():
    """Loss = logsumexp over the DM-time plane on the Nf=32, Nt=256, Nd=32 slice of
    the 0.4-0.8 GHz workload; gradient A^T softmax(Ax) vs central differences."""
    nf, nt, nd, band = 32, 256, 32, (0.4, 0.8)
    x = W.make_c5(batch=1, nf=nf, nt=nt)[0].astype(np.float64)
    ax = fdmt(x, *band, nd)
    p = np.exp(ax - ax.max())
    p /= p.sum()
    grad = fdmt_adjoint(p, *band, nf)
    rng = _rng(11)
    h = 1e-5
    for _ in range(8):
        v = rng.standard_normal((nf, nt))
        fd = (_lse(fdmt(x + h * v, *band, nd)) - _lse(fdmt(x - h * v, *band, nd))) / (2 * h)
        an = float(np.sum(grad * v))
        assert abs(fd - an) <= 1e-7 * max(1.0, abs(an))
    gmax = np.abs(grad).max()
    for _ in range(64):
        k, t = int(rng.integers(nf)), int(rng.integers(nt))
        e = np.zeros((nf, nt))
        e[k, t] = 1.0
        fd = (_lse(fdmt(x + h * e, *band, nd)) - _lse(fdmt(x - h * e, *band, nd))) / (2 * h)
        assert abs(fd - grad[k, t]) <= 1e-6 * gmax


# ---------------------------------------------------------------- binary32 mode

def test_binary32_mode_exact_on_representable_data():
    """With small integers every partial sum is exactly representable in binary32,
    so the binary32 recursion must reproduce the int64 result exactly."""
    x = _rng(21).integers(-100, 100, size=(64, 300))
    ref = fdmt(x, 1.2, 1.6, 64)
    got = fdmt(x.astype(np.float32), 1.2, 1.6, 64, acc=np.float32)
    assert got.dtype == np.float32
    np.testing.assert_array_equal(got.astype(np.int64), ref)
    g = _rng(22).integers(-100, 100, size=(64, 300))
    np.testing.assert_array_equal(
        fdmt_adjoint(g.astype(np.float32), 1.2, 1.6, 64, acc=np.float32).astype(np.int64),
        fdmt_adjoint(g, 1.2, 1.6, 64))


def test_binary32_mode_within_rounding_bound():
    """binary32 results stay inside the first-order tree-summation bound of the
    float64 result, and are not identical to it (so rounding really happens)."""
    from numerics import adjoint_bound, forward_bound
    x = W.random_input((128, 700), np.float32, seed=23)
    x[:, 300] += 40.0
    ref = fdmt(x.astype(np.float64), 0.4, 0.8, 200)
    got = fdmt(x, 0.4, 0.8, 200, acc=np.float32)
    assert np.all(np.abs(got - ref) <= forward_bound(x, 0.4, 0.8, 200))
    assert np.any(got != ref)
    g = W.random_input((200, 700), np.float32, seed=24)
    ref_a = fdmt_adjoint(g.astype(np.float64), 0.4, 0.8, 128)
    got_a = fdmt_adjoint(g, 0.4, 0.8, 128, acc=np.float32)
    assert np.all(np.abs(got_a - ref_a) <= adjoint_bound(g, 0.4, 0.8, 128))


# ---------------------------------------------------------------- boxcar search

def test_boxcar_impulse_closed_form():
    """One impulse A at (row r, t0) of a zero plane: b_w is A on
    [t0, t0 + w - 1] and 0 elsewhere, so the peak is A first at t0, the mean
    A*n/Nt and the variance A^2*n/Nt - mean^2, n = min(w, Nt - t0); other rows
    are all zero (stdev 0, snr 0)."""
    nd, nt, t0, amp, m = 3, 50, 40, 3.0, 5
    y = np.zeros((nd, nt))
    y[1, t0] = amp
    res = boxcar_search(y, m)
    for j in range(m + 1):
        n = min(1 << j, nt - t0)
        mean = amp * n / nt
        assert res["peak"][j, 1] == amp and res["t"][j, 1] == t0
        assert math.isclose(res["mean"][j, 1], mean, rel_tol=1e-12)
        assert math.isclose(res["stdev"][j, 1], math.sqrt(amp * amp * n / nt - mean * mean), rel_tol=1e-12)
        assert res["peak"][j, 0] == 0 and res["t"][j, 0] == 0 and res["stdev"][j, 0] == 0 and res["snr"][j, 0] == 0


def test_boxcar_constant_row_closed_form():
    """A constant c: b_w[t] = c * min(t + 1, w), so the peak c*min(w, Nt) first
    reached at t = min(w, Nt) - 1, and the mean c/Nt * sum_t min(t + 1, w)."""
    c, nt, m = 2.0, 37, 6
    res = boxcar_search(np.full((1, nt), c), m)
    for j in range(m + 1):
        w = 1 << j
        assert res["peak"][j, 0] == c * min(w, nt) and res["t"][j, 0] == min(w, nt) - 1
        ramp = [c * min(t + 1, w) for t in range(nt)]
        assert math.isclose(res["mean"][j, 0], sum(ramp) / nt, rel_tol=1e-12)


def test_boxcar_commutes_with_transform():
    """Sec. 4.2: a pulse profile shared by all frequencies commutes with the
    FDMT. The oracle's width-w boxcar of the transform equals the transform of
    the input boxcar-filtered per channel (causal, zero history), exactly on
    integers; and the binary32 tree equals it on small integers."""
    nf, nt, nd, band, m = 16, 300, 24, (1.2, 1.6), 4
    x = _rng(5).integers(0, 20, size=(nf, nt)).astype(np.int64)
    y = fdmt(x, *band, nd)
    res = boxcar_search(y, m)
    res32 = boxcar_search(y.astype(np.float32), m, acc=np.float32)
    for j in range(m + 1):
        w = 1 << j
        xw = np.zeros_like(x)
        for i in range(w):
            xw[:, i:] += x[:, : nt - i]
        yw = fdmt(xw, *band, nd)
        np.testing.assert_array_equal(res["peak"][j], yw.max(axis=1))
        np.testing.assert_array_equal(res["t"][j], yw.argmax(axis=1))
        np.testing.assert_allclose(res["mean"][j], yw.mean(axis=1), rtol=1e-12)
        np.testing.assert_allclose(res["stdev"][j], yw.std(axis=1), rtol=1e-12)
        for k in ("peak", "t"):
            np.testing.assert_array_equal(res32[k][j], res[k][j])


def test_boxcar_binary32_tree_within_rounding():
    """On Gaussian data the binary32 tree's b_w differs from the float64
    definition by at most j rounding steps of its magnitude (the tree adds
    each window in j levels), so the peaks agree to ~j * 2^-24 relative."""
    y = _rng(6).standard_normal((4, 500)).astype(np.float32)
    m = 6
    r64 = boxcar_search(y, m)
    r32 = boxcar_search(y, m, acc=np.float32)
    for j in range(m + 1):
        bound = (j + 1) * 2.0 ** -24 * (1 << j) * np.abs(y).max()
        assert np.all(np.abs(r32["peak"][j] - r64["peak"][j]) <= bound)


# ---------------------------------------------------------------- d_min pre-shift

@pytest.mark.parametrize("nf,nd,d_min", [(16, 40, 100), (256, 128, 700), (1024, 256, 3000), (100, 64, 300)])
@pytest.mark.parametrize("band", [(1.2, 1.6), (0.4, 0.8)])
def test_dmin_path_follows_law_from_dmin(nf, nd, d_min, band):
    """Sec. 4.2 (different range of dispersions): with the pre-shift, row dt
    follows total delay d_min + dt. The run channel k adds, [sigma_k,
    sigma_k + delta_k], is centred within (log2(Nf) + 1)/2 samples (+ the
    law's curvature over half a channel) of where the curve of delay
    d_min + dt crosses the channel, (d_min + dt) * (phi(e_k) + phi(e_k+1))/2:
    the path's own bound plus the pre-shift's rounding."""
    f_min, f_max = band
    t = build_tables(nf, nd, f_min, f_max, d_min=d_min)
    e = np.array([f_min + k * (f_max - f_min) / nf for k in range(nf + 1)])
    phi = (f_min ** -2 - e ** -2) / (f_min ** -2 - f_max ** -2)
    mid = 0.5 * (phi[:-1] + phi[1:])
    phic = (f_min ** -2 - (0.5 * (e[:-1] + e[1:])) ** -2) / (f_min ** -2 - f_max ** -2)
    assert 0 <= min(t.pre) and max(t.pre) <= d_min
    curv = d_min * np.max(np.abs(phic - mid))
    bound = 0.5 * (t.levels + 1) + curv + 1e-9
    for dt in list(range(0, nd, max(1, nd // 31))) + [nd - 1]:
        p = np.array(path(t, dt))
        centre = p[:, 0] + 0.5 * p[:, 1]
        assert np.max(np.abs(centre - (d_min + dt) * mid)) <= bound


def test_dmin_zero_is_the_plain_transform():
    x = _rng(8).integers(0, 50, size=(32, 200)).astype(np.int64)
    t0 = build_tables(32, 40, 1.2, 1.6)
    t1 = build_tables(32, 40, 1.2, 1.6, d_min=0)
    assert t1.pre == [0] * 32
    np.testing.assert_array_equal(fdmt(x, 1.2, 1.6, 40, t0), fdmt(x, 1.2, 1.6, 40, t1))


@pytest.mark.parametrize("d_min", [57, 400])
def test_dmin_recursion_matches_path_and_adjoint(d_min):
    """With a pre-shift the recursion still equals brute-force summation
    along each row's (shifted) path, and the adjoint is its exact transpose
    (<A x, g> = <x, A^T g> on integers)."""
    nf, nt, nd, band = 64, 500, 50, (1.2, 1.6)
    rng = _rng(d_min)
    t = build_tables(nf, nd, *band, d_min=d_min)
    x = rng.integers(0, 30, size=(nf, nt)).astype(np.int64)
    y = fdmt(x, *band, nd, t)
    for dt in [0, 17, nd - 1]:
        np.testing.assert_array_equal(y[dt], brute_row(x, t, dt))
    g = rng.integers(-5, 6, size=(nd, nt)).astype(np.int64)
    assert int((y * g).sum()) == int((x * fdmt_adjoint(g, *band, nf, t)).sum())


def test_dmin_pulse_recovered_at_offset_row():
    """A width-1 pulse of total delay D = d_min + dt0 peaks at row dt0 of the
    pre-shifted transform (within 2 samples, >= 60% of the pulse)."""
    nf, nd, band, d_min = 256, 128, (1.2, 1.6), 900
    nt = d_min + nd + 300
    t = build_tables(nf, nd, *band, d_min=d_min)
    for dt0 in [0, 40, nd - 1]:
        t_arr = nt - 100
        img = np.zeros((nf, nt), dtype=np.int64)
        W.inject_pulses(img, band[0], band[1], [(d_min + dt0, t_arr, 1.0)])
        out = fdmt(img, *band, nd, t)
        i, j = np.unravel_index(np.argmax(out), out.shape)
        assert abs(i - dt0) <= 2 and abs(j - t_arr) <= 2, (dt0, i, j)
        assert out[i, j] >= 0.6 * nf


# ---------------------------------------------------------------- FFT-FDMT (Algorithm 2)

@pytest.mark.parametrize("nf,nt,nd,band,kw", [
    (1, 40, 9, (1.2, 1.6), {}), (8, 100, 12, (1.2, 1.6), {}), (32, 50, 64, (0.4, 0.8), {}),
    (64, 300, 100, (1.2, 1.6), {}), (12, 200, 40, (1.0, 2.0), {}), (100, 256, 90, (1.2, 1.6), {}),
    (64, 300, 64, (1.2, 1.6), dict(d_min=150)), (64, 300, 64, (0.4, 0.8), dict(gamma=1.0))])
def test_fft_fdmt_equals_shift_fdmt(nf, nt, nd, band, kw):
    """Algorithm 2 computes the transform of Algorithm 1: on integer data its
    complex128 result rounds to the exact int64 result (errors far below 1/2),
    including partial paths, Nf != 2^k, the d_min pre-shift and other laws."""
    x = _rng(nf + nt).integers(0, 256, size=(nf, nt))
    t = build_tables(nf, nd, *band, **kw)
    y = fdmt_fft(x, *band, nd, t)
    ref = fdmt(x, *band, nd, t)
    assert np.max(np.abs(y - ref)) < 1e-6 * max(1, np.max(np.abs(ref)))
    np.testing.assert_array_equal(np.rint(y).astype(np.int64), ref)


def test_fft_fdmt_without_padding_wraps():
    """Zero padding (Algorithm 2 comments): the shifts are cyclic, so with no
    padding an output reads the end of the record in place of the zeros before
    it; the result is then the path sums with time taken modulo Nt (the
    Option-1 runs themselves start at t = 0)."""
    nf, nt, nd, band = 16, 64, 40, (1.2, 1.6)
    x = _rng(3).integers(0, 100, size=(nf, nt))
    t = build_tables(nf, nd, *band)
    y = np.rint(fdmt_fft(x, *band, nd, t, n=nt)).astype(np.int64)
    assert not np.array_equal(y, fdmt(x, *band, nd, t))
    for dt in (0, 7, nd - 1):
        for t0 in (0, 5, 30, nt - 1):
            total = 0
            for k, (sigma, delta) in enumerate(path(t, dt)):
                tc = (t0 - sigma) % nt
                total += sum(int(x[k, tc - i]) for i in range(delta + 1) if tc - i >= 0)
            assert y[dt, t0] == total, (dt, t0)
    np.testing.assert_array_equal(np.rint(fdmt_fft(x, *band, nd, t, n=fft_length(nt, nd))).astype(np.int64),
                                  fdmt(x, *band, nd, t))


def test_boxcar_float64_checker_accepts_tree_and_rejects_planted_errors():
    """The GPU boxcar's parity check (float64 definition with rounding bounds)
    accepts a binary32 evaluation of the doubling tree (here the oracle's own),
    including ties and rows shorter than the widest boxcar, and rejects
    results with a wrong time, a wrong peak, stdev of another width or a
    shifted mean."""
    import copy

    from numerics import check_boxcar_float64
    m = 6
    y = _rng(9).standard_normal((2, 3, 700)).astype(np.float32)
    y[0, 1, 300] = 40.0                      # a unique maximum at every width
    y[1, 2, :] = 0.0
    y[1, 2, [10, 600]] = 5.0                 # equal maxima
    good = boxcar_search(y, m, acc=np.float32)
    check_boxcar_float64(good, y, m)
    check_boxcar_float64(boxcar_search(y[..., :20], m, acc=np.float32), y[..., :20], m)
    planted = []
    bad = copy.deepcopy(good)
    bad["t"][0, 3, 1] += 1                   # unique maximum, time off by one
    planted.append(bad)
    bad = copy.deepcopy(good)
    bad["peak"][0, 2, 0] *= 1 + 1e-4         # peak beyond the rounding bound
    planted.append(bad)
    bad = copy.deepcopy(good)
    bad["stdev"][:, 4] = good["stdev"][:, 5]  # statistics of another width
    planted.append(bad)
    bad = copy.deepcopy(good)
    bad["mean"][1, 1, 0] += 1e-3
    planted.append(bad)
    for b in planted:
        with pytest.raises(AssertionError):
            check_boxcar_float64(b, y, m)


# ---------------------------------------------------------------- two-C rule (reading R-twoC)

def test_two_c_hand_derived_example():
    """The two-C rule on the hand-derived Nf=4 example: lower half's delay from
    C at the lower sub-band's end label, upper half's shift from C at the upper
    sub-band's start label (tests/golden/tiny_twoc_nf4_nd4.txt)."""
    f_min, f_max, nd, img, expect = read_golden("tiny_twoc_nf4_nd4.txt")
    np.testing.assert_array_equal(fdmt(img, f_min, f_max, nd, build_tables(4, nd, f_min, f_max, rule=1)), expect)


def test_two_c_two_channels_closed_form():
    """Nf = 2: C_lo = 0 and C_hi = 1 exactly, so row dt is I[0][t] + I[1][t - dt]
    (one sample per channel, the upper channel dt samples earlier)."""
    x = _rng(21).integers(0, 100, size=(2, 40)).astype(np.int64)
    y = fdmt(x, 0.4, 0.8, 25, build_tables(2, 25, 0.4, 0.8, rule=1))
    for dt in range(25):
        ref = x[0].copy()
        ref[dt:] += x[1, : 40 - dt]
        np.testing.assert_array_equal(y[dt], ref)


def _label_law(t):
    """Per channel, the fraction of the label-to-label delay reached at its label."""
    e = channel_edges(t.nf, t.f_min, t.f_max)
    g = t.gamma
    law = (lambda f: 1.0 / (f * f)) if g == -2.0 else (lambda f: f ** g)
    if t.nf == 1:
        return [0.0]
    return [(law(e[k]) - law(e[0])) / (law(e[t.nf - 1]) - law(e[0])) for k in range(t.nf)]


@pytest.mark.parametrize("nf,nd,band,gamma", [(8, 30, (1.2, 1.6), -2.0), (64, 64, (1.2, 1.6), -2.0),
                                              (1024, 1024, (0.4, 0.8), -2.0), (100, 90, (1.2, 1.6), -2.0),
                                              (256, 300, (1.0, 3.0), 2.0), (7, 50, (1.0, 2.0), -2.0)])
def test_two_c_paths(nf, nd, band, gamma):
    """Under the two-C rule every channel adds exactly one sample (row 0), the
    first channel at t0 and the last at t0 - dt exactly, and every channel's
    shift is within log2(Nf)/2 samples of dt times the label law (each
    iteration rounds once, by at most 1/2, a convex combination of its
    parent's errors). Channel rows are all 1; every inverse table entry is
    used."""
    t = build_tables(nf, nd, *band, gamma=gamma, rule=1)
    assert all(r == 1 for r in t.rows[0][:nf])
    bound = t.levels / 2 + 1e-9
    phi = _label_law(t)
    for dt in range(nd):
        p = path(t, dt)
        assert all(delta == 0 for _, delta in p)
        assert p[0][0] == 0 and p[-1][0] == (dt if nf > 1 else 0)
        for k, (sigma, _) in enumerate(p):
            assert abs(sigma - dt * phi[k]) <= bound, (dt, k, sigma)
        assert all(p[k][0] <= p[k + 1][0] for k in range(nf - 1))


@pytest.mark.parametrize("nf,nt,nd,band", [(16, 200, 40, (1.2, 1.6)), (5, 100, 30, (1.0, 2.0)),
                                           (64, 300, 64, (0.4, 0.8))])
def test_two_c_recursion_equals_path_sums(nf, nt, nd, band):
    """The recursion under the two-C tables equals explicit summation of one
    sample per channel along each row's path (integers, exact); row 0 is the
    channel sum; all-ones data give Nf wherever t0 >= dt; the adjoint is the
    exact transpose."""
    t = build_tables(nf, nd, *band, rule=1)
    x = _rng(nf + nd).integers(0, 50, size=(nf, nt)).astype(np.int64)
    y = fdmt(x, *band, nd, t)
    for dt in range(0, nd, 3):
        np.testing.assert_array_equal(y[dt], brute_row(x, t, dt))
    np.testing.assert_array_equal(y[0], x.sum(axis=0))
    ones = fdmt(np.ones((nf, nt), dtype=np.int64), *band, nd, t)
    for dt in range(nd):
        assert np.all(ones[dt, dt:] == nf)
    g = _rng(nt).integers(-20, 20, size=(nd, nt)).astype(np.int64)
    assert int((y * g).sum()) == int((x * fdmt_adjoint(g, *band, nf, t)).sum())


def test_two_c_recovers_pulse_at_labels():
    """A width-1 pulse that crosses each channel at its label time (the point
    the rule samples) is found within 2 samples of its (dt, T), with at least
    0.6 Nf of its amplitude, the criterion of the one-C pulse pin (the path
    sits up to log2(Nf)/2 samples off the exact curve, so a width-1 pulse
    loses some channels)."""
    nf, nt, nd, band = 256, 2000, 400, (1.2, 1.6)
    t = build_tables(nf, nd, *band, rule=1)
    phi = _label_law(t)
    x = np.zeros((nf, nt))
    for dt, T, amp in ((333, 1500, 5.0), (57, 900, 3.0)):
        for k in range(nf):
            x[k, int(round(T - dt * phi[k]))] += amp
        y = fdmt(x, *band, nd, t)
        i, j = np.unravel_index(np.argmax(y), y.shape)
        assert abs(i - dt) <= 2 and abs(j - T) <= 2, (i, j)
        assert y[i, j] >= 0.6 * amp * nf, y[i, j] / (amp * nf)
        x[:] = 0


def test_boxcar_candidates_closed_form_and_pulses():
    """Candidates (one per row, width and 2048-sample block whose peak S/N is
    at least the threshold). A zero row with impulses A at t1 < t2 in
    different blocks: for width w, b_w is A on [t_i, t_i + w - 1], mean
    2wA/Nt and stdev sqrt(2wA^2/Nt - mean^2); each impulse's block is a
    candidate at t_i with that S/N, no other block is. And pulses planted in
    noise are found at their row, width and end time."""
    from oracle import boxcar_candidates
    nt, a, t1, t2 = 10000, 4.0, 100, 6000
    y = np.zeros((2, nt))
    y[1, [t1, t2]] = a
    m = 3
    c = boxcar_candidates(y, m, 5.0)
    for j in range(m + 1):
        w = 1 << j
        mean = 2 * w * a / nt
        sd = math.sqrt(2 * w * a * a / nt - mean * mean)
        got = [x for x in c if x[2] == j]
        assert [(x[1], x[3]) for x in got] == [(1, t1), (1, t2)]
        for x in got:
            assert x[4] == a and math.isclose(x[5], (a - mean) / sd, rel_tol=1e-12)
    assert boxcar_candidates(y, m, 1e9) == []
    rng = _rng(17)
    z = rng.standard_normal((8, 12000))
    z[3, 5000:5008] += 4.0           # an 8-sample pulse ending at 5007 (S/N about 11 at width 8)
    c = boxcar_candidates(z, 5, 7.0)
    assert c and all(x[1] == 3 for x in c)
    best = max(c, key=lambda x: x[5])
    assert best[2] == 3 and abs(best[3] - 5007) <= 1

