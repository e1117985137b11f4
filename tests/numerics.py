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
