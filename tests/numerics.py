"""Error bounds for binary32 evaluation of the recursion (test helpers).

Every output of the forward transform is a sum evaluated by a fixed tree of
additions whose depth (the most roundings any one term goes through) is at most
D = log2(Nf) + (longest Option-1 chain - 1). The standard bound for a sum
evaluated by such a tree gives, per element,
    |computed - exact| <= gamma_D * sum|terms|,  gamma_D = D*u/(1 - D*u), u = 2^-24,
and sum|terms| is the transform of |I|. The adjoint sums at most c_max parent
rows per child per iteration (c_max - 1 roundings each) and the Option-1
transpose adds n(n+1)/2 terms in one chain."""
import numpy as np

from oracle import build_tables, fdmt, fdmt_adjoint

U32 = 2.0 ** -24


def _gamma(d):
    return d * U32 / (1.0 - d * U32)


def forward_bound(img, f_min, f_max, nd):
    img = np.asarray(img, dtype=np.float64)
    t = build_tables(img.shape[0], nd, f_min, f_max)
    depth = t.levels + max(t.rows[0]) - 1
    return _gamma(depth) * fdmt(np.abs(img), f_min, f_max, nd, t)


def adjoint_bound(grad, f_min, f_max, nf):
    grad = np.asarray(grad, dtype=np.float64)
    t = build_tables(nf, grad.shape[0], f_min, f_max)
    cmax = 1
    for l in range(1, t.levels + 1):
        for trip in t.split[l]:
            for col in (0, 2):
                vals = [x[col] for x in trip if x[col] is not None]  # a copy row has no upper half
                if vals:
                    cmax = max(cmax, max(vals.count(v) for v in set(vals)))
    nmax = max(t.rows[0])
    depth = t.levels * (cmax - 1) + nmax * (nmax + 1) // 2
    return _gamma(depth) * fdmt_adjoint(np.abs(grad), f_min, f_max, nf, t)


def rel_to_rms(got, ref):
    ref = np.asarray(ref, dtype=np.float64)
    rms = float(np.sqrt(np.mean(ref * ref))) or 1.0
    return float(np.max(np.abs(np.asarray(got, dtype=np.float64) - ref))) / rms


def rms_ratio(got, ref):
    ref = np.asarray(ref, dtype=np.float64)
    err = np.asarray(got, dtype=np.float64) - ref
    return float(np.sqrt(np.mean(err * err)) / (np.sqrt(np.mean(ref * ref)) or 1.0))


def check_boxcar_float64(res, y, max_log2):
    """Checks a binary32 boxcar search result against the float64 definition.

    The search sums each window of w = 2^j samples in binary32 through a tree
    of depth j, so every running sum satisfies |b_gpu - b| <= gamma_j * B,
    with b the float64 boxcar of y and B that of |y| (bound E = max over the
    row). Then |peak_gpu - max b| <= E, and the reported time t must hold a
    value b[t] >= max b - 2E (any such t is a correct answer up to rounding);
    where that leaves one index, it must be the exact argmax. The mean and
    standard deviation are FP64 statistics of the binary32 sums, stored as
    binary32: within the mean (RMS) of the per-element bound plus FP64
    summation and output rounding. The S/N follows by error propagation.
    res: dict of arrays [..., max_log2 + 1, nd]; y: [..., nd, nt] float32."""
    from oracle import boxcar
    y = np.asarray(y, dtype=np.float64)
    nt = y.shape[-1]
    get = {k: np.asarray(v.cpu().numpy() if hasattr(v, "cpu") else v) for k, v in res.items()}
    u64 = 2.0 ** -53
    for j in range(max_log2 + 1):
        w = 1 << j
        b = boxcar(y, w)
        bound = _gamma(j) * boxcar(np.abs(y), w)
        e = bound.max(axis=-1)
        p = b.max(axis=-1)
        peak = get["peak"][..., j, :].astype(np.float64)
        t = get["t"][..., j, :].astype(np.int64)
        assert np.all(np.abs(peak - p) <= e * (1 + 1e-12) + 1e-300), f"peak, width {w}"
        assert np.all((t >= 0) & (t < nt)), f"t range, width {w}"
        bt = np.take_along_axis(b, t[..., None], axis=-1)[..., 0]
        assert np.all(bt >= p - 2 * e * (1 + 1e-12)), f"t not a maximum within rounding, width {w}"
        near = (b >= (p - 2 * e)[..., None]).sum(axis=-1)
        exact_t = np.argmax(b, axis=-1)
        assert np.all(t[near == 1] == exact_t[near == 1]), f"unique maximum missed, width {w}"
        mean = b.mean(axis=-1)
        sd = b.std(axis=-1)
        fp64 = nt * u64 * (np.abs(b).max(axis=-1) + bound.max(axis=-1))
        dm = bound.mean(axis=-1) + fp64
        ds = np.sqrt((bound ** 2).mean(axis=-1)) + nt * u64 * (mean ** 2 + sd ** 2 + 1.0) / np.maximum(sd, 1e-300)
        ds = np.where(sd > 0, ds, np.sqrt((bound ** 2).mean(axis=-1)))
        gm = get["mean"][..., j, :].astype(np.float64)
        gs = get["stdev"][..., j, :].astype(np.float64)
        assert np.all(np.abs(gm - mean) <= dm + U32 * np.abs(mean) + 1e-300), f"mean, width {w}"
        assert np.all(np.abs(gs - sd) <= ds + U32 * sd + 1e-300), f"stdev, width {w}"
        snr = np.where(sd > 0, (p - mean) / np.where(sd > 0, sd, 1.0), 0.0)
        gsnr = get["snr"][..., j, :].astype(np.float64)
        ok = sd > 2 * ds
        tol = (e + dm + np.abs(snr) * ds) / np.where(ok, sd - ds, 1.0) + 2 * U32 * np.abs(snr)
        assert np.all(np.abs(gsnr - snr)[ok] <= tol[ok] * (1 + 1e-9)), f"snr, width {w}"
        flat = sd == 0
        assert np.all(gsnr[flat] == 0.0), f"snr of a constant window sum, width {w}"
