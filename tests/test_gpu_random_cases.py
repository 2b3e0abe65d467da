"""Seeded random small cases across the options at once, GPU against the
oracle: grid size (odd and even, 9 to 40 cells), source count and positions,
radii up to beyond half the box, the optical-depth weights (tau_w 0.6, 2 or
geometric), the source-cell reading (directional or scalar half path), the
sweep of large pieces (layers, layers with the table through the caches,
shells), batched or one launch per source, and the scheduling radii; the
forward's Gamma at 1e-5 (G19 floor) and the adjoint's dL/dn_H, dL/dx_HI and
dL/dQ at 1e-5 in both rate forms.  Each case is drawn from its own seed, so
a failure names a reproducible case."""
import math

import numpy as np
import pytest
import torch

import oracle
from tests.parity import assert_grad_parity, assert_parity
from workloads import make_workload

pytestmark = pytest.mark.gpu
TOL = 1e-5
CASES = list(range(24))


@pytest.fixture(scope="module")
def asora():
    import paper_2311_01492_amd as m
    return m


@pytest.fixture(scope="module")
def bb():
    return oracle.blackbody_table()


def _draw(seed):
    rng = np.random.default_rng(7000 + seed)
    N = int(rng.integers(9, 41))
    n_src = int(rng.integers(1, 9))
    w = make_workload("c2", N=N, n_src=n_src, R=(0.5, 1.0), seed=7100 + seed)
    w.src.ijk[:] = rng.integers(0, N, size=(n_src, 3)).astype(np.int32)
    w.src.R[:] = rng.uniform(0.0, 0.75 * N, size=n_src).astype(np.float32)
    opt = dict(tau_w=[0.6, 2.0, math.inf][int(rng.integers(0, 3))],
               scalar=bool(rng.integers(0, 2)),
               sweep=[3, -3, 2][int(rng.integers(0, 3))],
               plain=bool(rng.integers(0, 2)),
               R_whole=float(rng.choice([3.0, 4.0, 6.0])),
               R_oct=float(rng.choice([6.0, 8.0, 12.0])),
               adj_rate=int(rng.integers(1, 3)),
               adj_waves=int(rng.choice([2, 4, 12, 16])))
    return w, opt


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


@pytest.mark.parametrize("seed", CASES)
def test_random_case_forward_and_adjoint(asora, bb, seed):
    w, o = _draw(seed)
    print(f"case random seed={seed} N={w.N} n_src={len(w.src)} R_max={float(w.src.R.max()):.2f} {o}",
          flush=True)
    reading = 1 if o["scalar"] else 0
    ctx = asora.Asora(w.N, w.cell_cm, bb.P, bb.dP, bb.lg_lo, bb.lg_hi, tau_w=o["tau_w"],
                      halfpath_scalar=o["scalar"])
    ctx.set_tuning(R_whole=o["R_whole"], R_oct=o["R_oct"], pyramid_sweep=abs(o["sweep"]),
                   table_place=2 if o["sweep"] < 0 else 1, adj_rate=o["adj_rate"], adj_waves=o["adj_waves"])
    nH, xH, ijk, Q, R = _t(w.n_H), _t(w.x_HI), _t(w.src.ijk), _t(w.src.Q), _t(w.src.R)
    g = ctx.raytrace(nH, xH, ijk, Q, R, plain=o["plain"])
    ctx.check()
    og = oracle.raytrace(w.N, w.cell_cm, bb, w.n_H, w.x_HI, w.src.ijk, w.src.Q, w.src.R, tau_w=o["tau_w"],
                         reading=reading)
    assert_parity(g.cpu().numpy().astype(np.float64), og, TOL, what=f"Gamma seed={seed}")
    wt = np.random.default_rng(7200 + seed).standard_normal(og.shape)
    gbar = wt / ((og + 1e-20) * math.log(10))
    on, ox, oq = oracle.raytrace_grad(w.N, w.cell_cm, bb, w.n_H, w.x_HI, w.src.ijk, w.src.Q, w.src.R, gbar,
                                      tau_w=o["tau_w"], reading=reading)
    dn, dx, dq = ctx.backward(nH, xH, ijk, Q, R, _t(gbar))
    ctx.check()
    assert_grad_parity(dn.cpu().numpy().astype(np.float64), on, TOL, what=f"dL/dn_H seed={seed}")
    assert_grad_parity(dx.cpu().numpy().astype(np.float64), ox, TOL, what=f"dL/dx_HI seed={seed}")
    np.testing.assert_allclose(dq.cpu().numpy(), oq, rtol=TOL, atol=1e-12 * np.abs(oq).max(),
                               err_msg=f"dL/dQ seed={seed}")
    ctx.close()
