"""Pins of the oracle's reverse mode: central finite differences of the FP64
oracle forward, and the exact linearity of Gamma in each source's rate."""
import math

import numpy as np
import pytest

import oracle
from workloads import gaussian_field, lognormal_density

ALPHA = 4.3e24


def _case(N=14, nsrc=3, seed=31, R=5.5):
    rng = np.random.default_rng(seed)
    nH = lognormal_density(gaussian_field(N, rng))
    xHI = np.where(rng.random((N,) * 3) < 0.5, 1e-3, 1.0).astype(np.float64)
    ijk = rng.integers(0, N, size=(nsrc, 3)).astype(np.int32)
    Q = 10 ** rng.uniform(52, 55, nsrc)
    Rv = np.full(nsrc, R)
    w = rng.standard_normal((N,) * 3)
    return N, nH.astype(np.float64), xHI, ijk, Q, Rv, w


def _dloss(gp, gm, w):
    """L(+) - L(-) for L = sum w log10(Gamma + 1e-20), summed cell by cell so
    that the difference is not lost in the rounding of the full sum."""
    return float(np.sum(w * (np.log10(gp + 1e-20) - np.log10(gm + 1e-20))))


def _gbar(g, w):
    return w / ((g + 1e-20) * math.log(10))


@pytest.mark.parametrize("tau_w,reading", [(0.6, 0), (math.inf, 0), (0.6, 1)])
def test_reverse_mode_matches_central_differences(tau_w, reading):
    tb = oracle.blackbody_table()
    N, nH, xHI, ijk, Q, R, w = _case()
    fwd = lambda a, b, q: oracle.raytrace(N, ALPHA, tb, a, b, ijk, q, R, tau_w=tau_w, reading=reading)
    g = fwd(nH, xHI, Q)
    dnH, dxHI, dQ = oracle.raytrace_grad(N, ALPHA, tb, nH, xHI, ijk, Q, R, _gbar(g, w),
                                         tau_w=tau_w, reading=reading)
    rng = np.random.default_rng(2)
    covered = np.argwhere(g > 0)
    picks = covered[rng.choice(len(covered), 12, replace=False)]
    # include the source cells themselves (half-path rule, reading A / B)
    picks = np.concatenate([picks, ijk[:2]])
    for p in map(tuple, picks):
        for field, grad in ((nH, dnH), (xHI, dxHI)):
            h = 1e-4 * field[p]
            fp, fm = field.copy(), field.copy()
            fp[p] += h
            fm[p] -= h
            args_p = (fp, xHI) if field is nH else (nH, fp)
            args_m = (fm, xHI) if field is nH else (nH, fm)
            fd = _dloss(fwd(*args_p, Q), fwd(*args_m, Q), w) / (2 * h)
            scale = max(abs(fd), 1e-6 * np.abs(grad).max())
            assert abs(grad[p] - fd) <= 1e-5 * scale, (p, grad[p], fd)
    for s in range(len(Q)):
        h = 1e-4 * Q[s]
        qp, qm = Q.copy(), Q.copy()
        qp[s] += h
        qm[s] -= h
        fd = _dloss(fwd(nH, xHI, qp), fwd(nH, xHI, qm), w) / (2 * h)
        assert dQ[s] == pytest.approx(fd, rel=1e-6)


def test_rate_gradient_is_linear_response():
    """Gamma is linear in each Q_s, so dL/dQ_s = sum_p gbar_p Gamma^s_p / Q_s
    exactly, with Gamma^s the field of source s alone."""
    tb = oracle.blackbody_table()
    N, nH, xHI, ijk, Q, R, w = _case(seed=32)
    g = oracle.raytrace(N, ALPHA, tb, nH, xHI, ijk, Q, R)
    gb = _gbar(g, w)
    _, _, dQ = oracle.raytrace_grad(N, ALPHA, tb, nH, xHI, ijk, Q, R, gb)
    for s in range(len(Q)):
        gs = oracle.raytrace(N, ALPHA, tb, nH, xHI, ijk[s:s + 1], Q[s:s + 1], R[s:s + 1])
        assert dQ[s] == pytest.approx(float(np.sum(gb * gs)) / Q[s], rel=1e-12)
