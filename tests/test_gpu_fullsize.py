"""Full-size checks in the benchmark's launch configuration: the scheduling
parameters are the autotuner's (asora_autotune on the same workload, its
result taken from the library's tuning cache when the workload was tuned
before), on the 128^3 workload (1000 sources, R = 30), the 250^3 one (1e5
sources, R up to 50) and the million-source one (R up to 40).

- Forward: all 1000 sources of the 128^3 workload in one call against the
  oracle cell by cell.
- Adjoint at the radii of the 250^3 workloads, unclipped by the periodic
  extent: a few sources with R in [40, 50] on the 1e5-source workload's fields
  and with R in [30, 40] on the million-source workload's fields, with the
  columns recomputed (both forms of the rate terms) and kept by the forward,
  against the oracle's reverse mode cell by cell.
- Adjoint of whole workloads in one call: dL/dQ_s depends only on source s
  and on dL/dGamma (Gamma is a sum over sources, each linear in its Q), so
  sampled sources of the full call are checked one by one against the
  oracle's reverse mode run on those sources alone; over all sources the
  linear-response identity sum_s Q_s dL/dQ_s = sum_p dL/dGamma_p Gamma_p ties
  the adjoint to the forward.  On the 128^3 workload, whose column records fit
  in memory, the adjoint that reads them is also checked against the one that
  recomputes."""
import math

import numpy as np
import pytest
import torch

import oracle
from tests.parity import assert_grad_parity, assert_parity
from workloads import make_workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def asora():
    import paper_2311_01492_amd as m
    return m


@pytest.fixture(scope="module")
def bb():
    return oracle.blackbody_table()


_WORKLOADS = {}


def workload(name):
    if name not in _WORKLOADS:
        _WORKLOADS[name] = make_workload(name)
    return _WORKLOADS[name]


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def tuned_context(asora, bb, w):
    """A context with the autotuner's scheduling for the whole workload w
    (forward keeping records + adjoint, as the benchmark tunes it)."""
    ctx = asora.Asora(w.N, w.cell_cm, bb.P, bb.dP, bb.lg_lo, bb.lg_hi)
    ctx.load_tuning(asora.TUNING_CACHE)
    ctx.autotune(_t(w.n_H), _t(w.x_HI), _t(w.src.ijk), _t(w.src.Q), _t(w.src.R),
                 R_max=float(w.src.R.max()), passes=2)
    return ctx


def test_c2_forward_all_sources_against_oracle(asora, bb):
    """The 1000-source 128^3 forward in one call, every cell against the oracle."""
    w = workload("c2")
    print("case c2 forward, all 1000 sources vs oracle", flush=True)
    ctx = tuned_context(asora, bb, w)
    g = ctx.raytrace(_t(w.n_H), _t(w.x_HI), _t(w.src.ijk), _t(w.src.Q), _t(w.src.R))
    ctx.check()
    o = oracle.raytrace(w.N, w.cell_cm, bb, w.n_H, w.x_HI, w.src.ijk, w.src.Q, w.src.R)
    assert_parity(g.cpu().numpy(), o, 1e-5)


# (workload, radius range, sources): sources of the workload's own list with
# radii in the range, seeded choice
FULL_RADII = [("c3", (40.0, 50.0), 8), ("c5", (30.0, 40.0), 8)]
FORMS = [dict(store=False, adj_rate=1), dict(store=False, adj_rate=2), dict(store=True, adj_rate=1)]
FORM_IDS = ["recompute-gathered", "recompute-split", "kept"]


@pytest.mark.parametrize("name,rng_R,n", FULL_RADII, ids=[f[0] for f in FULL_RADII])
def test_adjoint_at_full_radii_against_oracle(asora, bb, name, rng_R, n):
    w = workload(name)
    cand = np.nonzero((w.src.R >= rng_R[0]) & (w.src.R <= rng_R[1]))[0]
    idx = np.sort(np.random.default_rng(31).choice(cand, size=n, replace=False))
    sub = w.src.subset(idx)
    # unclipped: every radius fits the periodic extent of the 250^3 grid
    assert sub.R.max() < w.N // 2 - 1
    print(f"case {name} adjoint at radii {sub.R.min():.1f}..{sub.R.max():.1f}, {n} sources", flush=True)
    g = oracle.raytrace(w.N, w.cell_cm, bb, w.n_H, w.x_HI, sub.ijk, sub.Q, sub.R)
    wt = np.random.default_rng(32).standard_normal(g.shape)
    gbar = wt / ((g + 1e-20) * math.log(10))
    on, ox, oq = oracle.raytrace_grad(w.N, w.cell_cm, bb, w.n_H, w.x_HI, sub.ijk, sub.Q, sub.R, gbar)
    ctx = tuned_context(asora, bb, w)
    tuning = dict(zip(asora.TUNING_KEYS, ctx.get_tuning()))
    assert tuning["pyramid_sweep"] == 3 and sub.R.min() > tuning["R_oct"]   # layer pyramids
    nH, xH, ijk, Q, R, gb = _t(w.n_H), _t(w.x_HI), _t(sub.ijk), _t(sub.Q), _t(sub.R), _t(gbar)
    for form, fid in zip(FORMS, FORM_IDS):
        print(f"  form {fid}", flush=True)
        ctx.set_tuning(adj_rate=form["adj_rate"])
        gam = ctx.raytrace(nH, xH, ijk, Q, R, store=form["store"])
        if form["store"]:
            assert ctx.store_info()[0]
        dn, dx, dq = ctx.backward(nH, xH, ijk, Q, R, gb, store=form["store"])
        ctx.check()
        assert_parity(gam.cpu().numpy(), g, 1e-5, what=f"gamma ({fid})")
        assert_grad_parity(dn.cpu().numpy(), on, 1e-5, what=f"dL/dn_H ({fid})")
        assert_grad_parity(dx.cpu().numpy(), ox, 1e-5, what=f"dL/dx_HI ({fid})")
        np.testing.assert_allclose(dq.cpu().numpy(), oq, rtol=1e-5, err_msg=f"dL/dQ ({fid})")


@pytest.mark.parametrize("name", ["c2", "c3", "c5"])
def test_full_workload_adjoint(asora, bb, name):
    w = workload(name)
    print("case full workload", name, len(w.src), "sources", flush=True)
    ctx = tuned_context(asora, bb, w)
    nH, xH, ijk, Q, R = _t(w.n_H), _t(w.x_HI), _t(w.src.ijk), _t(w.src.Q), _t(w.src.R)
    rng = np.random.default_rng(17)
    gbar = rng.uniform(0.0, 1.0, w.N ** 3)
    gamma = ctx.raytrace(nH, xH, ijk, Q, R, store=True)
    kept = ctx.store_info()[0]
    assert kept == (name == "c2")   # the records of the 250^3 workloads need terabytes
    dn, dx, dq = ctx.backward(nH, xH, ijk, Q, R, _t(gbar), store=kept)
    ctx.check()
    g = gamma.cpu().numpy().astype(np.float64).ravel()
    dq = dq.cpu().numpy()
    # linear response: Gamma from the FP32 forward, dL/dQ from the FP64 adjoint
    lhs, rhs = float(np.dot(w.src.Q, dq)), float(np.dot(gbar, g))
    assert lhs == pytest.approx(rhs, rel=1e-5), (lhs, rhs)
    if kept:
        rc = [a.cpu().numpy() for a in ctx.backward(nH, xH, ijk, Q, R, _t(gbar), store=False)]
        ctx.check()
        for a, b, what in zip((dn.cpu().numpy(), dx.cpu().numpy(), dq), rc, ("dL/dn_H", "dL/dx_HI", "dL/dQ")):
            np.testing.assert_allclose(a, b, rtol=1e-9, atol=1e-12 * np.abs(b).max(), err_msg=what)
    # sampled sources, the largest radius among them, against the oracle
    idx = np.sort(np.append(rng.choice(len(w.src), size=3, replace=False), int(np.argmax(w.src.R))))
    sub = w.src.subset(idx)
    _, _, oq = oracle.raytrace_grad(w.N, w.cell_cm, bb, w.n_H, w.x_HI, sub.ijk, sub.Q, sub.R, gbar)
    np.testing.assert_allclose(dq[idx], oq, rtol=1e-5)
    assert np.all(oq > 0)
