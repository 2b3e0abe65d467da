"""GPU parity of the forward ray tracing (HIP kernels through the C ABI)
against the FP64 oracle.  Bar: max relative error 1e-5 on Gamma and on the
column density over cells above 1e-20 of the maximum (tests/parity.py);
exact zeros where the oracle is zero."""
import math

import numpy as np
import pytest
import torch

import oracle
from tests.parity import assert_parity, floored_rel
from workloads import make_workload

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module")
def asora():
    import paper_2311_01492_amd as m
    return m


@pytest.fixture(scope="module")
def bb():
    return oracle.blackbody_table()


def _ctx(asora, w, table, sweep=3, **kw):
    """sweep: 3 = large sources as layer pyramids (the default), 2 = shell
    pyramids, -3 = layer pyramids with the table read through the caches."""
    ctx = asora.Asora(w.N, w.cell_cm, table.P, table.dP, table.lg_lo, table.lg_hi, **kw)
    ctx.set_tuning(pyramid_sweep=abs(sweep), table_place=2 if sweep < 0 else 1)
    return ctx


SWEEPS = pytest.mark.parametrize("sweep", [3, -3, 2], ids=["layers", "layers-cached-table", "shells"])


def _dev(w):
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    return t(w.n_H), t(w.x_HI)


def _gpu(ctx, w, src=None, **kw):
    src = src or w.src
    nH, xH = _dev(w)
    out = ctx.raytrace(nH, xH, torch.from_numpy(src.ijk), torch.from_numpy(src.Q),
                       torch.from_numpy(src.R), **kw)
    ctx.check()
    if isinstance(out, tuple):
        return tuple(o.cpu().numpy().astype(np.float64) for o in out)
    return out.cpu().numpy().astype(np.float64)


def _orc(w, table, src=None, **kw):
    src = src or w.src
    return oracle.raytrace(w.N, w.cell_cm, table, w.n_H, w.x_HI, src.ijk, src.Q, src.R, **kw)


@SWEEPS
@pytest.mark.parametrize("plain", [False, True])
def test_c1_gamma_and_column(asora, bb, plain, sweep):
    w = make_workload("c1")
    print("case c1 plain", plain, "sweep", sweep, flush=True)
    o, ocd = _orc(w, bb, coldens=True)
    ctx = _ctx(asora, w, bb, sweep=sweep)
    ctx.set_tuning(R_whole=6.0, R_oct=10.0)   # R = 15: a pyramid source
    g, cd = _gpu(ctx, w, coldens=True, plain=plain)
    assert_parity(g, o, TOL)
    assert_parity(cd, ocd, TOL, what="coldens")
    assert np.count_nonzero(cd) == 14147 - 1


@SWEEPS
@pytest.mark.parametrize("plain", [False, True])
def test_uneven_radii_all_piece_kinds(asora, bb, plain, sweep):
    """Radii 2..40 cover the whole-source, octant and pyramid pieces."""
    w = make_workload("c2", N=48, n_src=40, R=(2.0, 40.0))
    print("case uneven N=48 n_src=40 plain", plain, "sweep", sweep, flush=True)
    o = _orc(w, bb)
    g = _gpu(_ctx(asora, w, bb, sweep=sweep), w, plain=plain)
    assert_parity(g, o, TOL)


@SWEEPS
def test_c2_subset(asora, bb, sweep):
    w = make_workload("c2")
    sub = w.src.subset(np.arange(60))
    print("case c2 subset 60 sweep", sweep, flush=True)
    o = _orc(w, bb, src=sub)
    g = _gpu(_ctx(asora, w, bb, sweep=sweep), w, src=sub)
    assert_parity(g, o, TOL)


def test_c2_full_by_superposition(asora, bb):
    """All 1000 C2 sources in one launch equal the sum of ten 100-source
    launches (Gamma is additive over sources); one chunk is checked against
    the oracle in test_c2_subset's way."""
    w = make_workload("c2")
    print("case c2 full superposition", flush=True)
    ctx = _ctx(asora, w, bb)
    full = _gpu(ctx, w)
    parts = sum(_gpu(ctx, w, src=w.src.subset(np.arange(k, k + 100))) for k in range(0, 1000, 100))
    rel, small, n = floored_rel(full, parts)
    assert rel < 1e-6 and small < 1e-6
    o = _orc(w, bb, src=w.src.subset(np.arange(900, 920)))
    g = _gpu(ctx, w, src=w.src.subset(np.arange(900, 920)))
    assert_parity(g, o, TOL)


def test_c3_shape_subset(asora, bb):
    """250^3 grid, radii U[5,50]: a 120-source subset against the oracle."""
    w = make_workload("c3", n_src=120)
    print("case c3 subset 120", flush=True)
    o = _orc(w, bb)
    g = _gpu(_ctx(asora, w, bb), w)
    assert_parity(g, o, TOL)


def test_c5_shape_subset(asora, bb):
    """250^3 grid, x_HI from the smoothed threshold field (about half the
    volume ionized), radii U[5,40]: a 60-source subset against the oracle,
    with the autotuned scheduling of a small run."""
    w = make_workload("c5", n_src=60)
    print("case c5 subset 60", flush=True)
    o = _orc(w, bb)
    ctx = _ctx(asora, w, bb)
    ctx.set_tuning(R_whole=8.0, R_oct=8.0, max_waves=16, table_place=2)
    g = _gpu(ctx, w)
    assert_parity(g, o, TOL)


@pytest.mark.parametrize("tau_w,scalar", [(math.inf, False), (0.6, True)])
def test_weighting_and_source_readings(asora, bb, tau_w, scalar):
    w = make_workload("c2", N=32, n_src=12, R=(3.0, 20.0))
    print("case readings", tau_w, scalar, flush=True)
    o = _orc(w, bb, tau_w=tau_w, reading=1 if scalar else 0)
    g = _gpu(_ctx(asora, w, bb, tau_w=tau_w, halfpath_scalar=scalar), w)
    assert_parity(g, o, TOL)


def test_grey_table_and_zero_density(asora):
    gt = oracle.grey_table()
    w = make_workload("c2", N=24, n_src=5, R=(2.0, 12.0))
    w.n_H = (w.n_H * 2e-3).astype(np.float32)
    print("case grey", flush=True)
    assert_parity(_gpu(_ctx(asora, w, gt), w), _orc(w, gt), TOL)
    w.n_H = np.zeros_like(w.n_H)
    bb = oracle.blackbody_table()
    assert_parity(_gpu(_ctx(asora, w, bb), w), _orc(w, bb), TOL)


@SWEEPS
def test_edges_odd_grid_wrap_and_clip(asora, bb, sweep):
    """Odd N, sources on the faces and corners of the box (periodic wrap),
    radii beyond half the box (extent clip), a duplicate source, R = 0."""
    w = make_workload("c2", N=19, n_src=6, R=(3.0, 17.0))
    w.src.ijk[:] = [[0, 0, 0], [18, 18, 18], [0, 9, 18], [5, 5, 5], [5, 5, 5], [12, 0, 7]]
    w.src.R[:] = [17.0, 9.5, 12.0, 4.0, 4.0, 0.0]
    print("case edges sweep", sweep, flush=True)
    assert_parity(_gpu(_ctx(asora, w, bb, sweep=sweep), w), _orc(w, bb), TOL)
    # even grid, radius beyond the box
    w = make_workload("c2", N=20, n_src=3, R=(12.0, 30.0))
    w.src.ijk[0] = [19, 0, 19]
    assert_parity(_gpu(_ctx(asora, w, bb, sweep=sweep), w), _orc(w, bb), TOL)


def test_empty_and_accumulate(asora, bb):
    w = make_workload("c2", N=24, n_src=3, R=(4.0, 18.0))
    ctx = _ctx(asora, w, bb)
    nH, xH = _dev(w)
    e = torch.empty(0, 3, dtype=torch.int32)
    g0 = ctx.raytrace(nH, xH, e, torch.empty(0, dtype=torch.float64), torch.empty(0), R_max=0.0)
    assert float(g0.abs().max()) == 0.0
    g1 = _gpu(ctx, w)
    acc = torch.from_numpy(g1.astype(np.float32).reshape(-1)).cuda()
    ctx.raytrace(nH, xH, torch.from_numpy(w.src.ijk), torch.from_numpy(w.src.Q),
                 torch.from_numpy(w.src.R), out=acc, accumulate=True)
    np.testing.assert_allclose(acc.cpu().numpy().reshape(g1.shape), 2 * g1, rtol=1e-6, atol=0)


def test_radius_above_bound_is_flagged(asora, bb):
    w = make_workload("c2", N=20, n_src=3, R=(4.0, 8.0))
    ctx = _ctx(asora, w, bb)
    nH, xH = _dev(w)
    ctx.raytrace(nH, xH, torch.from_numpy(w.src.ijk), torch.from_numpy(w.src.Q),
                 torch.from_numpy(w.src.R), R_max=3.0)
    with pytest.raises(asora.AsoraError) as e:
        ctx.check()
    assert e.value.status == -5
    ctx.check()   # cleared
    with pytest.raises(asora.AsoraError):
        ctx.raytrace(nH, xH, torch.from_numpy(w.src.ijk), torch.from_numpy(w.src.Q),
                     torch.from_numpy(w.src.R), coldens=True)


@pytest.mark.parametrize("case", ["uneven", "c2-subset"])
def test_early_exit_gives_the_full_sweeps_gamma(asora, bb, case):
    """ASORA_EARLY_EXIT stops each layer pyramid after its first opaque layer:
    Gamma equals the full sweep's (every later cell has a zero rate) and the
    oracle's; radii 2..40 also cover the pieces it does not apply to."""
    if case == "uneven":
        w = make_workload("c2", N=48, n_src=40, R=(2.0, 40.0))
        src = w.src
    else:
        w = make_workload("c2")
        src = w.src.subset(np.arange(60))
    print("case early exit", case, flush=True)
    o = _orc(w, bb, src=src)
    ctx = _ctx(asora, w, bb)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    nH, xH, ijk, Q, R = t(w.n_H), t(w.x_HI), t(src.ijk), t(src.Q), t(src.R)
    full = ctx.raytrace(nH, xH, ijk, Q, R)
    early = ctx.raytrace(nH, xH, ijk, Q, R, early_exit=True)
    ctx.check()
    f, e = full.cpu().numpy().astype(np.float64), early.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(e, f, rtol=1e-6, atol=1e-6 * np.abs(f).max())
    assert_parity(e, o, TOL)
    with pytest.raises(asora.AsoraError):
        ctx.raytrace(nH, xH, ijk[:1], Q[:1], R[:1], coldens=True, early_exit=True)


def test_block_level_octant_kernels(asora, bb):
    """Octant pieces whose four-shell ring does not fit several waves' LDS
    regions (R up to 44 on 96^3: about 47 KB per wave next to the 32 KB table,
    two per work-group) run one work-group per piece: the persistent block
    kernel for the batched call and the block kernel per source for the
    plain one.  Both against the oracle, and the adjoint of the same pieces
    (one wave per work-group) against the oracle's reverse mode."""
    print("case block-level octant kernels", flush=True)
    w = make_workload("c2", N=96, n_src=6, R=(30.0, 44.0))
    ctx = _ctx(asora, w, bb)
    ctx.set_tuning(R_oct=45.0)   # every source is swept as eight octants
    o = _orc(w, bb)
    for plain in (False, True):
        assert_parity(_gpu(ctx, w, plain=plain), o, TOL, what=f"gamma (plain={plain})")
    wt = np.random.default_rng(5).standard_normal(o.shape)
    gbar = wt / ((o + 1e-20) * math.log(10))
    on, ox, oq = oracle.raytrace_grad(w.N, w.cell_cm, bb, w.n_H, w.x_HI, w.src.ijk, w.src.Q, w.src.R,
                                      gbar)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    nH, xH = _dev(w)
    dn, dx, dq = ctx.backward(nH, xH, t(w.src.ijk), t(w.src.Q), t(w.src.R), t(gbar))
    ctx.check()
    from tests.parity import assert_grad_parity
    assert_grad_parity(dn.cpu().numpy(), on, 1e-5, what="dL/dn_H")
    assert_grad_parity(dx.cpu().numpy(), ox, 1e-5, what="dL/dx_HI")
    np.testing.assert_allclose(dq.cpu().numpy(), oq, rtol=1e-5)
