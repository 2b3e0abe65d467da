"""The library's per-cell code (cell update, row enumeration, rate numerics
from csrc/asora_dev.h) compiled for the CPU and driven serially, against the
FP64 oracle.  Checks the logic the GPU kernels run -- piece decomposition,
compact shell indexing, neighbour slots, interpolation, divided differences
-- without a GPU.  The parallel driver (wave scan, barriers, atomics) is
covered by the GPU tests."""
import math

import numpy as np
import pytest

import oracle
from tests.native import hostsweep
from tests.parity import assert_parity
from workloads import make_workload

TOL = 1e-5


@pytest.fixture(scope="module")
def bb():
    return oracle.blackbody_table()


# shell piece kinds 0, 1, 2 and the layer pyramids with both tile widths
KINDS = [dict(type_force=0), dict(type_force=1), dict(type_force=2), dict(layers=True)]
KIND_IDS = ["whole", "octants", "shell-pyramids", "layers"]


@pytest.mark.parametrize("kind", KINDS, ids=KIND_IDS)
def test_c1_all_piece_kinds(bb, kind):
    w = make_workload("c1")
    o, ocd = oracle.raytrace(w.N, w.cell_cm, bb, w.n_H, w.x_HI, w.src.ijk, w.src.Q, w.src.R, coldens=True)
    g, cd = hostsweep.raytrace(w.N, w.cell_cm, oracle.SIGMA0, bb, w.n_H, w.x_HI, w.src.ijk, w.src.Q,
                               w.src.R, coldens=True, **kind)
    assert_parity(g, o, TOL)
    assert_parity(cd, ocd, TOL, what="coldens")
    assert np.count_nonzero(cd) == 14147 - 1


@pytest.mark.parametrize("kind", [dict(type_force=-1)] + KINDS, ids=["by-radius"] + KIND_IDS)
@pytest.mark.parametrize("tau_w,reading", [(0.6, 0), (math.inf, 0), (0.6, 1)])
def test_lognormal_sources(bb, kind, tau_w, reading):
    w = make_workload("c2", N=36, n_src=9, R=(3.0, 21.0))
    o = oracle.raytrace(w.N, w.cell_cm, bb, w.n_H, w.x_HI, w.src.ijk, w.src.Q, w.src.R,
                        tau_w=tau_w, reading=reading)
    g = hostsweep.raytrace(w.N, w.cell_cm, oracle.SIGMA0, bb, w.n_H, w.x_HI, w.src.ijk, w.src.Q,
                           w.src.R, tau_w=tau_w, reading=reading, **kind)
    assert_parity(g, o, TOL)


def test_layers_ionized_medium_and_column(bb):
    """Mostly ionized medium (every cell carries a rate) and the column
    density output of a single source through the layer pyramids, with a
    source near the box corner so that offsets wrap."""
    w = make_workload("c2", N=40, n_src=1, R=(19.0, 19.0))
    xH = np.full_like(w.x_HI, 1e-3)
    ijk = np.array([[1, 38, 39]], np.int32)
    o, ocd = oracle.raytrace(w.N, w.cell_cm, bb, w.n_H, xH, ijk, w.src.Q, w.src.R, coldens=True)
    g, cd = hostsweep.raytrace(w.N, w.cell_cm, oracle.SIGMA0, bb, w.n_H, xH, ijk, w.src.Q,
                               w.src.R, coldens=True, layers=True)
    assert_parity(g, o, TOL)
    assert_parity(cd, ocd, TOL, what="coldens")
    assert np.count_nonzero(g) > 0.9 * np.count_nonzero(o)


def test_odd_grid_large_radius_extent_clip(bb):
    """R larger than the box: the periodic extent clips the ball (odd N)."""
    w = make_workload("c2", N=21, n_src=3, R=(14.0, 19.0))
    o = oracle.raytrace(w.N, w.cell_cm, bb, w.n_H, w.x_HI, w.src.ijk, w.src.Q, w.src.R)
    for kind in KINDS:
        g = hostsweep.raytrace(w.N, w.cell_cm, oracle.SIGMA0, bb, w.n_H, w.x_HI, w.src.ijk,
                               w.src.Q, w.src.R, **kind)
        assert_parity(g, o, TOL)
    w = make_workload("c2", N=20, n_src=3, R=(12.0, 30.0))   # even grid, R beyond the box
    o = oracle.raytrace(w.N, w.cell_cm, bb, w.n_H, w.x_HI, w.src.ijk, w.src.Q, w.src.R)
    for kind in KINDS[2:]:
        g = hostsweep.raytrace(w.N, w.cell_cm, oracle.SIGMA0, bb, w.n_H, w.x_HI, w.src.ijk,
                               w.src.Q, w.src.R, **kind)
        assert_parity(g, o, TOL)


def test_grey_and_thin(bb):
    gt = oracle.grey_table()
    w = make_workload("c2", N=24, n_src=4, R=(5.0, 11.0))
    nH = (w.n_H * 2e-3).astype(np.float32)          # a few optical depths per cell (grey)
    o = oracle.raytrace(w.N, w.cell_cm, gt, nH, w.x_HI, w.src.ijk, w.src.Q, w.src.R)
    g = hostsweep.raytrace(w.N, w.cell_cm, oracle.SIGMA0, gt, nH, w.x_HI, w.src.ijk, w.src.Q, w.src.R)
    assert_parity(g, o, TOL)
    thin = (w.n_H * 1e-9).astype(np.float32)        # tau per cell ~ 3e-6
    o = oracle.raytrace(w.N, w.cell_cm, bb, thin, w.x_HI, w.src.ijk, w.src.Q, w.src.R)
    g = hostsweep.raytrace(w.N, w.cell_cm, oracle.SIGMA0, bb, thin, w.x_HI, w.src.ijk, w.src.Q, w.src.R)
    assert_parity(g, o, TOL)
    g = hostsweep.raytrace(w.N, w.cell_cm, oracle.SIGMA0, bb, thin, w.x_HI, w.src.ijk, w.src.Q, w.src.R,
                           layers=True)
    assert_parity(g, o, TOL)
    zero = np.zeros_like(w.n_H)
    o = oracle.raytrace(w.N, w.cell_cm, bb, zero, w.x_HI, w.src.ijk, w.src.Q, w.src.R)
    g = hostsweep.raytrace(w.N, w.cell_cm, oracle.SIGMA0, bb, zero, w.x_HI, w.src.ijk, w.src.Q, w.src.R)
    assert_parity(g, o, TOL)


def test_divided_difference_regimes(bb):
    """-[P(a+dt)-P(a)]/dt of the library's log-space evaluation against the
    oracle's FP64 difference of its own interpolant, over the regimes: both
    ends in one node interval, neighbouring intervals, many intervals, across
    the first node, across the last node, zero width."""
    rng = np.random.default_rng(0)
    a = 10 ** rng.uniform(-6, 4.2, 4000)
    rel = 10 ** rng.uniform(-5, 3, 4000)
    dt = a * rel
    a = np.concatenate([a, [0.0, 0.0, 1e-21, 9999.0, 9990.0, 3.0]])
    dt = np.concatenate([dt, [1e-3, 2.7e3, 5e-21, 5.0, 0.5, 0.0]])
    got = hostsweep.neg_divdiff(bb, a, dt)
    Pa, d1a, _ = oracle.table_eval(bb, a)
    Pb, _, _ = oracle.table_eval(bb, a + dt)
    with np.errstate(invalid="ignore", divide="ignore"):
        want = np.where(dt > 0, -(Pb - Pa) / dt, -d1a)
    # below the first node the interpolant is linear: its difference quotient is
    # the slope there (FP64 cannot resolve 1 - P at tau ~ 1e-21)
    lin = a + dt < 1e-20
    want[lin] = -bb.dP[0]
    ok = want > 0
    # the oracle's FP64 difference itself loses digits when P(a+dt) ~ P(a)
    cond = np.where((dt > 0) & ~lin, np.abs(Pa) * 2.2e-16 / np.maximum(np.abs(Pb - Pa), 1e-300), 0)
    err = np.abs(got[ok] - want[ok]) / want[ok]
    assert np.all(err <= 2e-6 + 4 * cond[ok]), err.max()
    assert np.all(got[~ok] == 0)


def test_layer_chunk_walk_matches_division():
    """The division-free stepping of the layer kernels' chunk walk (64 cells
    forward and backward through a layer rectangle) decodes the same (u, v)
    as g / wv, g % wv for every row width up to 130."""
    assert hostsweep.rectwalk_check(130) == 0


@pytest.mark.parametrize("N", [16, 17])
def test_row_enumeration_matches_brute_force(N):
    """Union of the rows of all pieces of a type = the shell's cells in the
    ball and the periodic extent, each owned once."""
    rng = np.random.default_rng(N)
    off, sh = oracle.shell_order(N, 9.3)
    Rsq = int(math.floor(9.3 * 9.3))
    for q in rng.choice(np.arange(1, sh.max() + 1), 6, replace=False):
        want = {tuple(d) for d, s in zip(off, sh) if s == q}
        for type_ in (0, 1, 2):
            npieces = (1, 8, 24)[type_]
            got = []
            for p in range(npieces):
                blo, cnt = hostsweep.rows(N, type_, p, Rsq, int(q))
                for r in range(len(cnt)):
                    os_, A = divmod(r, int(q) + 1)
                    o = os_ if type_ == 0 else (p if type_ == 1 else p // 3)
                    for B in range(blo[r], blo[r] + cnt[r]):
                        C = q - A - B
                        d = (-A if o & 1 else A, -B if o & 2 else B, -C if o & 4 else C)
                        got.append(d)
            if type_ == 0:
                assert sorted(got) == sorted(want)
            else:
                assert set(got) == want          # ghosts duplicate cells, nothing missing or extra


@pytest.mark.parametrize("kind", [dict(type_force=-1)] + KINDS +
                         [dict(layers=True, split=False), dict(layers=True, kept=True),
                          dict(layers=True, early_exit=True), dict(layers=True, kept=True, early_exit=True)],
                         ids=["by-radius"] + KIND_IDS + ["layers-gathered", "layers-kept", "layers-early",
                                                         "layers-kept-early"])
@pytest.mark.parametrize("tau_w,reading", [(0.6, 0), (math.inf, 0), (0.6, 1)])
def test_adjoint_matches_oracle_reverse(bb, kind, tau_w, reading):
    """The library's per-cell adjoint, driven serially over the reversed
    shells, against the oracle's reverse mode for L = sum w log10(Gamma+1e-20)."""
    w = make_workload("c4", N=24, n_src=6, R=(3.0, 11.0))
    g = oracle.raytrace(w.N, w.cell_cm, bb, w.n_H, w.x_HI, w.src.ijk, w.src.Q, w.src.R,
                        tau_w=tau_w, reading=reading)
    wt = np.random.default_rng(1).standard_normal(g.shape)
    gbar = wt / ((g + 1e-20) * math.log(10))
    on, ox, oq = oracle.raytrace_grad(w.N, w.cell_cm, bb, w.n_H, w.x_HI, w.src.ijk, w.src.Q,
                                      w.src.R, gbar, tau_w=tau_w, reading=reading)
    st = {}
    hn, hx, hq = hostsweep.raytrace_grad(w.N, w.cell_cm, oracle.SIGMA0, bb, w.n_H, w.x_HI,
                                         w.src.ijk, w.src.Q, w.src.R, gbar, tau_w=tau_w,
                                         reading=reading, **kind, **({"stats": st} if "layers" in kind else {}))
    if "layers" in kind:
        if kind.get("early_exit"):
            # some pyramids end their adjoint at an opaque layer (the record
            # beyond it is left unwritten and poisoned in the emulation)
            assert st["n_stopped"] > 0
            assert st["visited"] < st["total"]
        else:   # without the early exit every layer is visited
            assert st["n_stopped"] == 0
            assert st["visited"] == st["total"]
    from tests.parity import assert_grad_parity
    assert_grad_parity(hn, on, 1e-5, what="dL/dn_H")
    assert_grad_parity(hx, ox, 1e-5, what="dL/dx_HI")
    np.testing.assert_allclose(hq, oq, rtol=1e-6)


def test_layer_adjoint_extent_clip_and_wrap(bb):
    """Layer adjoint with radii beyond the box (extent clip, even and odd N)
    and sources on the box faces, against the oracle's reverse mode."""
    for N, ijk in ((15, [[0, 7, 14], [3, 3, 3]]), (16, [[15, 0, 15], [8, 8, 0]])):
        w = make_workload("c4", N=N, n_src=2, R=(9.0, 13.0))
        w.src.ijk[:] = ijk
        g = oracle.raytrace(w.N, w.cell_cm, bb, w.n_H, w.x_HI, w.src.ijk, w.src.Q, w.src.R)
        wt = np.random.default_rng(2).standard_normal(g.shape)
        gbar = wt / ((g + 1e-20) * math.log(10))
        on, ox, oq = oracle.raytrace_grad(w.N, w.cell_cm, bb, w.n_H, w.x_HI, w.src.ijk, w.src.Q,
                                          w.src.R, gbar)
        from tests.parity import assert_grad_parity
        for split, kept in ((True, False), (False, False), (False, True)):
            hn, hx, hq = hostsweep.raytrace_grad(w.N, w.cell_cm, oracle.SIGMA0, bb, w.n_H, w.x_HI,
                                                 w.src.ijk, w.src.Q, w.src.R, gbar, layers=True,
                                                 split=split, kept=kept)
            assert_grad_parity(hn, on, 1e-5, what="dL/dn_H")
            assert_grad_parity(hx, ox, 1e-5, what="dL/dx_HI")
            np.testing.assert_allclose(hq, oq, rtol=1e-6)


def test_rate_derivatives_of_thin_cells(bb):
    """The adjoint's rate derivatives where the in-cell depth is below 1e-4 of
    the entry one: Gauss rules over [a, a + dt] whose nodes share the
    logarithm of a (ln a + ln(1 + g dt / a)).  Against the same rules on the
    library's interpolant with every node's own logarithm, and D against its
    definition P'(a) + dt/2 dD/da; inside the table, across its first node
    (a just below it) and at zero width.  Then against the oracle's own
    interpolant inside the table (its second derivative, to the agreement of
    the two interpolants)."""
    rng = np.random.default_rng(5)
    a = 10 ** rng.uniform(-19.5, 3.9, 3000)
    dt = a * 10 ** rng.uniform(-9, -4, 3000)
    a = np.concatenate([a, [1e-20 * (1 - 3e-5), 1e-20 * (1 - 1e-9), 7.0]])
    # (the first node: some quadrature nodes of the last two points lie above it)
    dt = np.concatenate([dt, [0.99e-24, 5e-29, 0.0]])
    assert np.all(dt <= 1e-4 * a)
    got = hostsweep.rate_derivs64(bb, a, dt)
    g1, g2 = 0.5 - 0.5 / math.sqrt(3), 0.5 + 0.5 / math.sqrt(3)
    j1, j2 = (6 - math.sqrt(6)) / 10, (6 + math.sqrt(6)) / 10
    w1, w2 = (9 + math.sqrt(6)) / 36, (9 - math.sqrt(6)) / 36
    for lib, d2 in ((True, lambda x: hostsweep.tab_eval64(bb, x)[:, 2]),
                    (False, lambda x: oracle.table_eval(bb, x)[2])):
        Da = 0.5 * (d2(a + g1 * dt) + d2(a + g2 * dt))
        Ddt = w1 * d2(a + j1 * dt) + w2 * d2(a + j2 * dt)
        if lib:
            # the per-node logarithms (1e-14 absolute) move a node's second
            # derivative by up to ~1e-10 where its terms nearly cancel
            d1a = hostsweep.tab_eval64(bb, a)[:, 1]
            D = d1a + 0.5 * dt * Da
            assert np.all(np.abs(got[:, 1] - Da) <= 1e-9 * np.abs(Da))
            assert np.all(np.abs(got[:, 2] - Ddt) <= 1e-9 * np.abs(Ddt))
            assert np.all(np.abs(got[:, 0] - D) <= 1e-12 * np.abs(D))
        else:
            # the two interpolants agree to ~1e-8 in ln P; a second derivative
            # is held to that on the scale |P'| / tau of its own size (it
            # crosses zero)
            inside = a >= 1.001e-20
            sc = 1e-6 * (np.abs(Da) + np.abs(hostsweep.tab_eval64(bb, a)[:, 1]) / a)
            assert np.all(np.abs(got[inside, 1] - Da[inside]) <= sc[inside])
            assert np.all(np.abs(got[inside, 2] - Ddt[inside]) <= sc[inside])


def test_kernel_logarithms():
    """The kernels' FP64 logarithms: log_fast (the rate's table position,
    2e-11 absolute) and log_f64 (the FP64 derivatives of the adjoint, 1e-14)."""
    rng = np.random.default_rng(11)
    for a in 10.0 ** rng.uniform(-20, 4.5, 3000):
        assert abs(hostsweep.log_fast(a) - math.log(a)) < 2.5e-11
        assert abs(hostsweep.log_f64(a) - math.log(a)) < 1e-14


def test_layer_adjoint_at_full_radii_of_the_250_grid(bb):
    """The kernels' per-cell adjoint code, emulated on the CPU, on sources of
    R in [40, 50] of the 1e5-source 250^3 workload (unclipped), against the
    oracle's reverse mode: the long columns and deep optical depths of these
    radii are where the rate derivatives' difference quotients magnify an
    error of the table position (the case that needs log_f64)."""
    w = make_workload("c3")
    cand = np.nonzero((w.src.R >= 40) & (w.src.R <= 50))[0]
    idx = np.sort(np.random.default_rng(31).choice(cand, size=4, replace=False))
    sub = w.src.subset(idx)
    g = oracle.raytrace(w.N, w.cell_cm, bb, w.n_H, w.x_HI, sub.ijk, sub.Q, sub.R)
    wt = np.random.default_rng(32).standard_normal(g.shape)
    gbar = wt / ((g + 1e-20) * math.log(10))
    on, ox, oq = oracle.raytrace_grad(w.N, w.cell_cm, bb, w.n_H, w.x_HI, sub.ijk, sub.Q, sub.R, gbar)
    from tests.parity import assert_grad_parity
    for split, kept in ((False, False), (True, False), (False, True)):
        hn, hx, hq = hostsweep.raytrace_grad(w.N, w.cell_cm, oracle.SIGMA0, bb, w.n_H, w.x_HI, sub.ijk, sub.Q,
                                             sub.R, gbar, layers=True, split=split, kept=kept)
        assert_grad_parity(hn, on, 1e-6, what="dL/dn_H")
        assert_grad_parity(hx, ox, 1e-6, what="dL/dx_HI")
        np.testing.assert_allclose(hq, oq, rtol=1e-8)
