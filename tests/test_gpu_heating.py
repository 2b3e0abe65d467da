"""GPU parity of the photo-heating sweep (asora_raytrace_heating: the rate and
the heating from one sweep, two table lookups per cell) against the oracle's
heating rate (the same sweep with the heating table H in place of P).  Bar:
max relative error 1e-5 on both outputs, as for the rate."""
import math

import numpy as np
import pytest
import torch

import oracle
from tests.parity import assert_grad_parity, assert_parity, floored_rel
from workloads import make_workload

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module")
def asora():
    import paper_2311_01492_amd as m
    return m


@pytest.fixture(scope="module")
def tabs():
    return oracle.blackbody_table(), oracle.blackbody_heat_table()


def _ctx(asora, w, tabs, sweep=3):
    tb, th = tabs
    ctx = asora.Asora(w.N, w.cell_cm, tb.P, tb.dP, tb.lg_lo, tb.lg_hi)
    ctx.set_tuning(pyramid_sweep=abs(sweep), table_place=2 if sweep < 0 else 1)
    ctx.set_heating_table(th.P, th.dP)
    return ctx


def _gpu(ctx, w, src=None, **kw):
    src = src or w.src
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    g, h = ctx.raytrace_heating(t(w.n_H), t(w.x_HI), t(src.ijk), t(src.Q), t(src.R), **kw)
    ctx.check()
    return g.cpu().numpy().astype(np.float64), h.cpu().numpy().astype(np.float64)


def _orc(w, tabs, src=None):
    src = src or w.src
    tb, th = tabs
    args = (w.n_H, w.x_HI, src.ijk, src.Q, src.R)
    return (oracle.raytrace(w.N, w.cell_cm, tb, *args),
            oracle.raytrace_heating(w.N, w.cell_cm, th, *args))


@pytest.mark.parametrize("sweep", [3, 2], ids=["layers", "shells"])
@pytest.mark.parametrize("plain", [False, True])
def test_heating_all_piece_kinds(asora, tabs, sweep, plain):
    """Radii 2..40: whole-source, octant and pyramid pieces."""
    w = make_workload("c2", N=48, n_src=40, R=(2.0, 40.0))
    print("case heating uneven N=48 plain", plain, "sweep", sweep, flush=True)
    og, oh = _orc(w, tabs)
    g, h = _gpu(_ctx(asora, w, tabs, sweep), w, plain=plain)
    assert_parity(g, og, TOL)
    assert_parity(h, oh, TOL, what="heating")


def test_heating_c2_subset_kept_records_and_early_exit(asora, tabs):
    """The 128^3 workload (60 sources): the heating sweep that keeps the
    rate's column records, and the one that stops at the opaque layers, both
    against the oracle; the records it kept give the recomputing adjoint's
    gradients."""
    w = make_workload("c2")
    sub = w.src.subset(np.arange(60))
    print("case heating c2 subset store / early exit", flush=True)
    og, oh = _orc(w, tabs, src=sub)
    ctx = _ctx(asora, w, tabs)
    g, h = _gpu(ctx, w, src=sub, store=True)
    assert_parity(g, og, TOL)
    assert_parity(h, oh, TOL, what="heating (records kept)")
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    nH, xH, ijk, Q, R = t(w.n_H), t(w.x_HI), t(sub.ijk), t(sub.Q), t(sub.R)
    gbar = torch.from_numpy(np.random.default_rng(3).standard_normal(w.N ** 3)).cuda()
    kept = [x.cpu().numpy() for x in ctx.backward(nH, xH, ijk, Q, R, gbar, store=True)]
    again = [x.cpu().numpy() for x in ctx.backward(nH, xH, ijk, Q, R, gbar, store=False)]
    for a, b, name in zip(kept, again, ("dn_H", "dx_HI", "dQ")):
        assert_grad_parity(a, b, 1e-6, what=name)
    g2, h2 = _gpu(ctx, w, src=sub, early_exit=True)
    assert_parity(g2, og, TOL, what="gamma (early exit)")
    assert_parity(h2, oh, TOL, what="heating (early exit)")


def test_heating_full_c2_by_superposition(asora, tabs):
    """All 1000 sources of the 128^3 workload in one heating launch equal the
    sum of four 250-source launches (heating is additive over sources); a
    20-source chunk against the oracle."""
    w = make_workload("c2")
    print("case heating c2 full superposition", flush=True)
    ctx = _ctx(asora, w, tabs)
    g, h = _gpu(ctx, w)
    parts = [_gpu(ctx, w, src=w.src.subset(np.arange(k, k + 250))) for k in range(0, 1000, 250)]
    for full, part, name in ((g, sum(p[0] for p in parts), "gamma"), (h, sum(p[1] for p in parts), "heating")):
        rel, small, _ = floored_rel(full, part)
        assert rel < 1e-6 and small < 1e-6, name
    sub = w.src.subset(np.arange(500, 520))
    og, oh = _orc(w, tabs, src=sub)
    g, h = _gpu(ctx, w, src=sub)
    assert_parity(g, og, TOL)
    assert_parity(h, oh, TOL, what="heating")


def test_heating_thin_limit_closed_form(asora, tabs):
    """Optically thin gas: heating / Gamma is the mean excess energy of the
    photons absorbed at zero depth, H'(0)/P'(0) = kT [J(4-a)/J(3-a) - x0]
    (incomplete-gamma series), in every cell of the ball."""
    from scipy.special import gamma as Gamma, gammaincc
    from oracle.tables import E_TH_EV, K_B_EV
    x0 = E_TH_EV / (K_B_EV * 5e4)
    n = np.arange(1, 61, dtype=np.float64)
    J = lambda s: float(np.sum(n ** -s * gammaincc(s, n * x0) * Gamma(s)))
    exact = K_B_EV * 5e4 * (J(1.2) / J(0.2) - x0)
    w = make_workload("c2", N=40, n_src=3, R=(6.0, 19.0))
    w.x_HI = np.zeros_like(w.x_HI)
    print("case heating thin limit", flush=True)
    g, h = _gpu(_ctx(asora, w, tabs), w)
    lit = g > 0
    assert lit.sum() > 1000 and np.all((h > 0) == lit)
    # FP32 outputs of FP32 divided differences: a few ulp
    np.testing.assert_allclose(h[lit] / g[lit], exact, rtol=2e-6)


def test_heating_requires_table_and_accumulates(asora, tabs):
    w = make_workload("c2", N=24, n_src=3, R=(4.0, 18.0))
    tb, th = tabs
    ctx = asora.Asora(w.N, w.cell_cm, tb.P, tb.dP, tb.lg_lo, tb.lg_hi)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    args = (t(w.n_H), t(w.x_HI), t(w.src.ijk), t(w.src.Q), t(w.src.R))
    with pytest.raises(asora.AsoraError) as e:
        ctx.raytrace_heating(*args)
    assert e.value.status == -4   # ESTATE: no heating table
    with pytest.raises(asora.AsoraError):
        ctx.set_heating_table(th.P, th.dP * 0 + 1.0)   # positive slopes
    with pytest.raises(asora.AsoraError):
        ctx.set_heating_table(th.P[:-1], th.dP[:-1])   # not the table's length
    ctx.set_heating_table(th.P, th.dP)
    g, h = ctx.raytrace_heating(*args)
    g1, h1 = g.clone(), h.clone()
    ctx.raytrace_heating(*args, out=g.reshape(-1), heating_out=h.reshape(-1), accumulate=True)
    np.testing.assert_allclose(h.cpu().numpy(), 2 * h1.cpu().numpy(), rtol=1e-6, atol=0)
    np.testing.assert_allclose(g.cpu().numpy(), 2 * g1.cpu().numpy(), rtol=1e-6, atol=0)
    # the rate alone afterwards is unchanged by the heating sweep
    g0 = ctx.raytrace(*args)
    np.testing.assert_allclose(g0.cpu().numpy(), g1.cpu().numpy(), rtol=1e-6, atol=0)
    assert math.isfinite(float(h1.max())) and float(h1.max()) > 0


@pytest.mark.parametrize("sweep", [3, 2], ids=["layers", "shells"])
def test_heating_edges_and_scaled_table(asora, sweep):
    """Odd grid, sources on faces and corners (periodic wrap), radii beyond
    half the box (extent clip), a duplicate source, R = 0; with the heating
    table E P (grey P = e^-tau), heating = E Gamma in every cell, whatever
    piece or accumulator (standard or transposed) the cell goes through."""
    gt = oracle.grey_table()
    E = 3.75
    w = make_workload("c2", N=19, n_src=6, R=(3.0, 17.0))
    w.n_H = (w.n_H * 2e-3).astype(np.float32)
    w.src.ijk[:] = [[0, 0, 0], [18, 18, 18], [0, 9, 18], [5, 5, 5], [5, 5, 5], [12, 0, 7]]
    w.src.R[:] = [17.0, 9.5, 12.0, 4.0, 4.0, 0.0]
    print("case heating edges sweep", sweep, flush=True)
    ctx = asora.Asora(w.N, w.cell_cm, gt.P, gt.dP, gt.lg_lo, gt.lg_hi)
    ctx.set_tuning(pyramid_sweep=sweep)
    ctx.set_heating_table(E * gt.P, E * gt.dP)
    g, h = _gpu(ctx, w)
    og = oracle.raytrace(w.N, w.cell_cm, gt, w.n_H, w.x_HI, w.src.ijk, w.src.Q, w.src.R)
    assert_parity(g, og, TOL)
    assert_parity(h, E * og, TOL, what="heating")
    # both from FP32 divided differences of tables whose logs differ by ln E;
    # far below the largest rate the FP32 products reach the denormal range
    # (flushed to zero), where only the parity floor applies
    big = og >= 1e-20 * og.max()
    np.testing.assert_allclose(h[big] / g[big], E, rtol=2e-6)
