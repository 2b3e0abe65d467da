"""Pins of the oracle sweep against closed forms, invariants and brute force.

Each test states the property of the method it checks.  Nothing here re-types
the oracle's formulas: expected values come from geometry (exact columns on
grid lines), symmetry, the optically thin limit of eq. gamma, the grey
closed form, lattice counting, linear algebra of the interpolation, or a
long-characteristics brute force.
"""
import itertools
import math

import numpy as np
import pytest

import oracle
from oracle import lc
from workloads import gaussian_field, lognormal_density

SIG = oracle.SIGMA0
ALPHA = 4.3e24


def _single(N, nH, xHI, src, Q=1e54, R=10.0, table=None, tau_w=0.6, reading=0):
    table = table or oracle.blackbody_table()
    return oracle.raytrace(N, ALPHA, table, nH, xHI, np.array([src], np.int32), [Q], [R],
                           tau_w=tau_w, reading=reading, coldens=True)


def _lognormal(N, seed):
    return lognormal_density(gaussian_field(N, np.random.default_rng(seed)))


# ---------------------------------------------------------------- P1 ---
def test_uniform_columns_exact_on_axes_and_diagonals():
    """Uniform medium: along axes and face/body diagonals the ray passes
    through cell centres only, so N_in = n alpha sqrt(d) (m - 1/2)."""
    N, s = 32, (16, 16, 16)
    n = 1.5e-4
    nH = np.full((N,) * 3, n, np.float32)
    xHI = np.ones((N,) * 3, np.float32)
    _, cd = _single(N, nH, xHI, s, R=15.0)
    nal = float(np.float32(n)) * ALPHA
    for m in range(1, 9):
        for dirv in [(0, 0, 1), (0, -1, 0), (1, 0, 0), (1, 1, 0), (0, -1, 1), (-1, 1, 1), (1, 1, 1)]:
            d = np.array(dirv) * m
            p = tuple(np.array(s) + d)
            exact = nal * math.sqrt(sum(abs(x) for x in dirv)) * (m - 0.5)
            assert cd[p] == pytest.approx(exact, rel=1e-13), (dirv, m)


def test_lines_equal_long_characteristics_in_random_medium():
    """On grid axes and diagonals short characteristics are exact in any medium:
    they equal the long-characteristics column to the cell centre minus half
    the cell's own path."""
    N, s = 24, (11, 13, 12)
    nH = _lognormal(N, 3)
    xHI = np.where(np.random.default_rng(4).random((N,) * 3) < 0.3, 1e-3, 1.0).astype(np.float32)
    _, cd = _single(N, nH, xHI, s, R=11.0, tau_w=0.6)
    nhi = oracle.n_HI(nH, xHI)
    for dirv in [(0, 0, -1), (0, 1, 0), (1, 0, 0), (1, -1, 0), (-1, 0, 1), (0, 1, 1), (1, 1, -1), (-1, -1, -1)]:
        for m in range(1, 7):
            d = np.array(dirv) * m
            p = tuple((np.array(s) + d) % N)
            ds = math.sqrt(sum(abs(x) for x in dirv))
            centre = lc.column_to_centre(nhi, ALPHA, s, d)
            assert cd[p] + 0.5 * nhi[p] * ALPHA * ds == pytest.approx(centre, rel=1e-12)


# ---------------------------------------------------------------- P2 ---
def _sym48():
    for perm in itertools.permutations(range(3)):
        for signs in itertools.product([1, -1], repeat=3):
            yield perm, signs


def test_octahedral_symmetry_48fold():
    """A centred source in a medium invariant under the 48 symmetries of the
    cube gives N and Gamma with the same symmetry (odd N so that the periodic
    extent is symmetric)."""
    N, c = 25, 12
    rng = np.random.default_rng(11)
    base = rng.lognormal(0, 0.5, size=(N, N, N))
    sym = np.zeros_like(base)
    for perm, signs in _sym48():
        t = np.transpose(base - 0, perm)
        for ax, sg in enumerate(signs):
            if sg < 0:
                t = np.roll(np.flip(t, ax), 2 * c + 1 - N, axis=ax)
        sym += t
    nH = (1e-4 * sym / 48).astype(np.float32)
    xHI = np.full((N,) * 3, 1e-2, np.float32)
    g, cd = _single(N, nH, xHI, (c, c, c), R=11.5, Q=1e53)
    assert np.count_nonzero(g) > 1000
    for perm, signs in _sym48():
        tg, tc = np.transpose(g, perm), np.transpose(cd, perm)
        for ax, sg in enumerate(signs):
            if sg < 0:
                tg = np.roll(np.flip(tg, ax), 2 * c + 1 - N, axis=ax)
                tc = np.roll(np.flip(tc, ax), 2 * c + 1 - N, axis=ax)
        np.testing.assert_allclose(tg, g, rtol=1e-13, atol=1e-300)
        np.testing.assert_allclose(tc, cd, rtol=1e-13, atol=0)


# ---------------------------------------------------------------- P3 ---
def test_shell_sizes_and_causality():
    """|S_q| = 4q^2+2 (Section 3.3), the top half k >= k_s has 2q(q+1)+1 cells
    (Appendix A), and every neighbour with non-zero weight lies in a strictly
    earlier shell, at most three shells back."""
    R = 12.0
    off, sh = oracle.shell_order(64, 30.0)          # ball of radius 30 covers shells q <= 30
    for q in range(0, 31):
        cells = off[sh == q]
        assert len(cells) == (4 * q * q + 2 if q > 0 else 1)
        if q > 0:
            assert np.sum(cells[:, 2] >= 0) == 2 * q * (q + 1) + 1
            assert np.sum(cells[:, 2] < 0) == 2 * q * q - 2 * q + 1
    off, sh = oracle.shell_order(64, R)
    for d, q in zip(off[1:], sh[1:]):
        e, s = oracle.neighbours(d)
        assert len(e) >= 1 and np.isclose(s.sum(), 1.0)
        L1 = np.abs(e).sum(axis=1)
        assert np.all(L1 < q) and np.all(L1 >= q - 3)


# ---------------------------------------------------------------- P4 ---
@pytest.mark.parametrize("R,count", [(15, 14147), (20, 33401), (30, 113081), (50, 523305)])
def test_ball_lattice_counts(R, count):
    r = np.arange(-R, R + 1)
    brute = int(np.sum((r[:, None, None] ** 2 + r[None, :, None] ** 2 + r[None, None, :] ** 2) <= R * R))
    assert brute == count
    off, _ = oracle.shell_order(2 * R + 4, float(R))
    assert len(off) == count


def test_periodic_extent_even_and_odd():
    """Appendix A: at most N/2 on the negative side and N/2-1 on the positive
    side of the source (even N); (N-1)/2 on both sides (odd N)."""
    off, _ = oracle.shell_order(10, 100.0)
    assert len(off) == 1000 and off.min() == -5 and off.max() == 4
    off, _ = oracle.shell_order(9, 100.0)
    assert len(off) == 729 and off.min() == -4 and off.max() == 4


# ---------------------------------------------------------------- P5 ---
def test_optically_thin_limit():
    """Thin limit of eq. gamma: Gamma -> Q sigma0 (-P'(0)) / (4 pi alpha^2 r^2),
    i.e. eq. gammalocal with the frequency-averaged cross-section.  Exact for
    n_HI = 0 (the interpolant is linear below its first node); for small
    n_HI the deviation is bounded by the curvature of P over tau_out."""
    tb = oracle.blackbody_table()
    N, s, Q = 24, (12, 12, 12), 1e52
    d = np.indices((N,) * 3).reshape(3, -1).T - np.array(s)
    r2 = (d ** 2).sum(axis=1).reshape((N,) * 3).astype(float)
    for xval, tol in [(0.0, 1e-14), (1e-9, 3e-4)]:
        nH = np.full((N,) * 3, 1e-4, np.float32)
        xHI = np.full((N,) * 3, xval, np.float32)
        g, _ = _single(N, nH, xHI, s, Q=Q, R=10.0, table=tb)
        inside = (r2 > 0) & (r2 <= 100)
        ratio = g[inside] * 4 * math.pi * ALPHA ** 2 * r2[inside] / (Q * SIG)
        np.testing.assert_allclose(ratio, -tb.dP[0], rtol=tol)
        # source cell: half path, volume alpha^3
        assert g[s] * 2 * ALPHA ** 2 / (Q * SIG) == pytest.approx(-tb.dP[0], rel=tol)
        assert np.all(g[~inside & (r2 > 0)] == 0)


# ---------------------------------------------------------------- P6 ---
def test_grey_uniform_axis_closed_form():
    """Grey opacity, uniform medium, on an axis (ds = 1, V = 4 pi (alpha m)^2
    alpha): Gamma = Q (e^-tau_in - e^-tau_out) / (n_HI alpha^3 4 pi m^2) with
    tau_in = sigma0 n alpha (m - 1/2)."""
    tb = oracle.grey_table()
    N, s, Q = 32, (16, 16, 16), 1e50
    n = 2e-7                                   # ~5.4 optical depths per cell /1000
    nH = np.full((N,) * 3, n, np.float32)
    xHI = np.ones((N,) * 3, np.float32)
    g, _ = _single(N, nH, xHI, s, Q=Q, R=14.0, table=tb, tau_w=0.6)
    nf = float(np.float32(n))
    tcell = SIG * nf * ALPHA
    for m in range(1, 14):
        ti, to = tcell * (m - 0.5), tcell * (m + 0.5)
        exact = Q * (math.exp(-ti) - math.exp(-to)) / (nf * ALPHA ** 3 * 4 * math.pi * m * m)
        for ax in range(3):
            for sg in (1, -1):
                p = list(s)
                p[ax] += sg * m
                assert g[tuple(p)] == pytest.approx(exact, rel=1e-7)
    exact_src = Q * (1 - math.exp(-tcell / 2)) / (nf * ALPHA ** 3)
    assert g[s] == pytest.approx(exact_src, rel=1e-7)


# ------------------------------------------------------- interpolation --
@pytest.mark.parametrize("d", [(3, 1, 5), (-2, 4, 1), (5, -5, 2), (1, 2, -3), (4, 4, 4), (0, 3, -7), (6, 0, 6)])
def test_interpolation_linear_precision(d):
    """With geometric weights, the interpolation reproduces any affine
    function of position exactly at the point where the ray from the source
    centre to the cell centre crosses the plane of the neighbour layer, i.e.
    at d (m-1)/m (the weights are the bilinear 'xy-distance' weights)."""
    d = np.array(d)
    m = np.abs(d).max()
    e, s = oracle.neighbours(d)
    assert np.allclose(s @ e, d * (m - 1) / m)
    c = np.array([0.3, -1.7, 2.2])
    f = lambda x: 5.0 + x @ c
    # full e1..e4 list: recover it from the non-zero ones (zero-weight entries unused)
    M4 = np.zeros(4)
    _, s4 = oracle.interp(d, M4, tau_w=math.inf)
    k = 0
    for nidx in range(4):
        if s4[nidx] > 0:
            M4[nidx] = f(e[k])
            k += 1
    v, _ = oracle.interp(d, M4, tau_w=math.inf)
    assert v == pytest.approx(f(d * (m - 1) / m), rel=1e-14)


def test_interpolation_tau_weights():
    """Optical-depth weights w = s / max(sigma0 M, tau_w): equal neighbours give
    that value; all-thin neighbours reduce to geometric weights; all-thick
    neighbours give the weighted harmonic mean of the optical depths."""
    d = np.array([3, 2, 5])
    _, s4 = oracle.interp(d, np.ones(4), tau_w=0.6)
    v, _ = oracle.interp(d, np.full(4, 7e20), tau_w=0.6)
    assert v == pytest.approx(7e20, rel=1e-15)
    M = np.array([1e15, 3e15, 2e15, 5e15])             # tau = 6.3e-3 .. 3.2e-2 < 0.6
    v, _ = oracle.interp(d, M, tau_w=0.6)
    assert v == pytest.approx(float(s4 @ M), rel=1e-14)
    M = np.array([1e18, 3e18, 2e18, 5e18])              # tau = 6.3 .. 31.5 > 0.6
    v, _ = oracle.interp(d, M, tau_w=0.6)
    tau = SIG * M
    assert SIG * v == pytest.approx(1.0 / float(s4 @ (1.0 / tau)), rel=1e-13)


def test_single_absorber_hand_values():
    """Only the source cell absorbs (geometric weights, reading A).  Hand
    derivation: a cell that interpolates from the source sees the exit column
    of the source along its own ray, n alpha ds/2 (ds = r/m); every other cell
    adds nothing.  (1,0,0): 1/2; (1,1,0): sqrt2/2; (1,1,1): sqrt3/2;
    (2,1,0) dominant i with a = 1/2: (1/2)(1/2) + (1/2)(sqrt2/2);
    (2,1,1): a = b = 1/2 over (1,1,1),(1,0,1),(1,1,0),(1,0,0).
    Reading B replaces every source column by 1/2."""
    N, s = 16, (8, 8, 8)
    nH = np.zeros((N,) * 3, np.float32)
    nH[s] = 1e-4
    xHI = np.ones((N,) * 3, np.float32)
    nal = float(np.float32(1e-4)) * ALPHA
    r2, r3 = math.sqrt(2), math.sqrt(3)
    expect_A = {(1, 0, 0): 0.5, (1, 1, 0): r2 / 2, (1, 1, 1): r3 / 2,
                (2, 1, 0): 0.5 * 0.5 + 0.5 * r2 / 2,
                (2, 1, 1): 0.25 * (r3 / 2 + r2 / 2 + r2 / 2 + 0.5)}
    _, cd = _single(N, nH, xHI, s, R=6.0, tau_w=math.inf, reading=0)
    for d, v in expect_A.items():
        for perm in itertools.permutations(range(3)):
            dd = np.array(d)[list(perm)]
            assert cd[tuple(np.array(s) + dd)] == pytest.approx(v * nal, rel=1e-14), d
    _, cdB = _single(N, nH, xHI, s, R=6.0, tau_w=math.inf, reading=1)
    for d in expect_A:
        assert cdB[tuple(np.array(s) + np.array(d))] == pytest.approx(0.5 * nal, rel=1e-14)


# ---------------------------------------------------------------- P8 ---
@pytest.mark.parametrize("medium", ["uniform", "lognormal"])
def test_short_vs_long_characteristics_bound(medium):
    """SC approximates LC to the cell centre (N_in + half the cell's own path).
    Uniform medium: within a few per cent at r >= 4.  Lognormal medium: the
    median error stays at the per-cent level, single cells behind density
    contrasts deviate more, and the optical-depth weighting removes most of
    the bias of pure geometric weights."""
    N, s, R = 16, (8, 8, 8), 7.5
    nH = np.full((N,) * 3, 1e-4, np.float32) if medium == "uniform" else _lognormal(N, 21) * 0.66
    xHI = np.ones((N,) * 3, np.float32)
    nhi = oracle.n_HI(nH, xHI)
    off, _ = oracle.shell_order(N, R)
    stats = {}
    for tau_w in (math.inf, 0.6):
        _, cd = _single(N, nH, xHI, s, R=R, tau_w=tau_w)
        errs = []
        for d in off[1:]:
            r = math.sqrt((d ** 2).sum())
            if r < 4:
                continue
            p = tuple((np.array(s) + d) % N)
            sc = cd[p] + 0.5 * nhi[p] * ALPHA * r / np.abs(d).max()
            errs.append(sc / lc.column_to_centre(nhi, ALPHA, s, d) - 1)
        errs = np.array(errs)
        stats[tau_w] = errs
        if medium == "uniform":
            assert np.abs(errs).max() < 0.08
        else:
            assert np.median(np.abs(errs)) < 0.06 and np.abs(errs).max() < 0.45
    if medium == "lognormal":
        assert abs(stats[0.6].mean()) < 0.5 * abs(stats[math.inf].mean())


# --------------------------------------------------------- P10-P12 ---
def _rand_case(N=20, nsrc=5, seed=5):
    rng = np.random.default_rng(seed)
    nH = _lognormal(N, seed)
    xHI = np.where(rng.random((N,) * 3) < 0.4, 1e-3, 1.0).astype(np.float32)
    ijk = rng.integers(0, N, size=(nsrc, 3)).astype(np.int32)
    Q = 10 ** rng.uniform(51, 54, nsrc)
    R = rng.uniform(3, 9, nsrc)
    return N, nH, xHI, ijk, Q, R


def _ray(N, nH, xHI, ijk, Q, R):
    return oracle.raytrace(N, ALPHA, oracle.blackbody_table(), nH, xHI, ijk, Q, R)


def test_linearity_superposition_and_merge():
    N, nH, xHI, ijk, Q, R = _rand_case()
    g = _ray(N, nH, xHI, ijk, Q, R)
    np.testing.assert_allclose(_ray(N, nH, xHI, ijk, 3.5 * Q, R), 3.5 * g, rtol=1e-14, atol=0)
    gA = _ray(N, nH, xHI, ijk[:2], Q[:2], R[:2])
    gB = _ray(N, nH, xHI, ijk[2:], Q[2:], R[2:])
    np.testing.assert_allclose(gA + gB, g, rtol=1e-14, atol=0)
    # two sources in the same cell with equal R act as one with the summed Q (Section 3)
    two = _ray(N, nH, xHI, np.repeat(ijk[:1], 2, 0), [Q[0], 2 * Q[0]], [R[0], R[0]])
    one = _ray(N, nH, xHI, ijk[:1], [3 * Q[0]], R[:1])
    np.testing.assert_allclose(two, one, rtol=1e-14, atol=0)


def test_periodic_translation():
    N, nH, xHI, ijk, Q, R = _rand_case(seed=8)
    g = _ray(N, nH, xHI, ijk, Q, R)
    sh = (3, -7, 11)
    gt = _ray(N, np.roll(nH, sh, (0, 1, 2)), np.roll(xHI, sh, (0, 1, 2)),
              ((ijk + np.array(sh)) % N).astype(np.int32), Q, R)
    np.testing.assert_allclose(gt, np.roll(g, sh, (0, 1, 2)), rtol=1e-14, atol=0)


def test_radius_monotonicity():
    """Cells within R1 get bitwise identical N and Gamma for any larger R."""
    N, nH, xHI, ijk, Q, R = _rand_case(seed=9, nsrc=1)
    tb = oracle.blackbody_table()
    g1, c1 = oracle.raytrace(N, ALPHA, tb, nH, xHI, ijk, Q, [5.5], coldens=True)
    g2, c2 = oracle.raytrace(N, ALPHA, tb, nH, xHI, ijk, Q, [8.0], coldens=True)
    mask = g1 != 0
    assert mask.sum() > 400
    assert np.array_equal(g1[mask], g2[mask]) and np.array_equal(c1[mask], c2[mask])


# ------------------------------------------------- photo-heating (H table) ---
def test_heating_thin_limit_and_hardening():
    """Photo-heating per HI atom from the heating table H (eV): in the thin
    limit heating / Gamma -> H'(0) / P'(0) = kT [J(4-a)/J(3-a) - x0], the mean
    excess energy of the photons absorbed at zero depth (J(s) = int_x0^inf
    x^(s-1)/(e^x-1) dx as an incomplete-gamma series); in a thick uniform
    medium the ratio grows along an axis (the spectrum hardens)."""
    from scipy.special import gamma as Gamma, gammaincc
    from oracle.tables import E_TH_EV, K_B_EV
    tb, th = oracle.blackbody_table(), oracle.blackbody_heat_table()
    T, a = 5e4, 2.8
    x0 = E_TH_EV / (K_B_EV * T)
    n = np.arange(1, 61, dtype=np.float64)
    J = lambda s: float(np.sum(n ** -s * gammaincc(s, n * x0) * Gamma(s)))
    exact = K_B_EV * T * (J(4 - a) / J(3 - a) - x0)
    N, s, Q = 24, (12, 12, 12), 1e52
    d = np.indices((N,) * 3).reshape(3, -1).T - np.array(s)
    r2 = (d ** 2).sum(axis=1).reshape((N,) * 3).astype(float)
    inside = (r2 > 0) & (r2 <= 100)
    ijk = np.array([s], np.int32)
    for xval, tol in [(0.0, 1e-10), (1e-9, 3e-4)]:
        nH = np.full((N,) * 3, 1e-4, np.float32)
        xHI = np.full((N,) * 3, xval, np.float32)
        g = oracle.raytrace(N, ALPHA, tb, nH, xHI, ijk, [Q], [10.0])
        h = oracle.raytrace_heating(N, ALPHA, th, nH, xHI, ijk, [Q], [10.0])
        np.testing.assert_allclose(h[inside] / g[inside], exact, rtol=tol)
        assert h[s] / g[s] == pytest.approx(exact, rel=tol)
        assert np.all(h[~inside & (r2 > 0)] == 0)
    # thick: neutral gas of tau ~ 2.7 per cell
    nH = np.full((N,) * 3, 1e-7, np.float32)
    xHI = np.ones((N,) * 3, np.float32)
    g = oracle.raytrace(N, ALPHA, tb, nH, xHI, ijk, [Q], [10.0])
    h = oracle.raytrace_heating(N, ALPHA, th, nH, xHI, ijk, [Q], [10.0])
    line = h[12, 12, 12:23] / g[12, 12, 12:23]
    assert np.all(np.diff(line) > 0) and line[0] > exact
