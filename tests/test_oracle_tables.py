"""Pins of the oracle's photoionization tables and their interpolant.

P(tau) = gamma(tau/sigma0)/gamma(0) (eq. tables, Section 2.2).  The oracle
builds it with adaptive QUADPACK quadrature; here it is checked against
closed forms (series of incomplete gamma functions), against an independent
composite Gauss-Legendre quadrature written in this file, and the Hermite
interpolant against quadrature between the nodes.
"""
import math

import numpy as np
import pytest
from scipy.special import gamma as Gamma, gammaincc

import oracle
from oracle.tables import E_TH_EV, K_B_EV, blackbody_P

T_BB, ALPHA = 5e4, 2.8
X0 = E_TH_EV / (K_B_EV * T_BB)


def _series_norm(x0, nterms=60):
    """int_x0^inf x^2/(e^x-1) dx = sum_n e^{-n x0} (x0^2/n + 2 x0/n^2 + 2/n^3)."""
    n = np.arange(1, nterms + 1, dtype=np.float64)
    return float(np.sum(np.exp(-n * x0) * (x0 ** 2 / n + 2 * x0 / n ** 2 + 2 / n ** 3)))


def _series_moment(x0, alpha, nterms=60):
    """int_x0^inf x^2 (x/x0)^-alpha/(e^x-1) dx = x0^alpha sum_n n^-(3-alpha) Gamma(3-alpha, n x0)."""
    s = 3.0 - alpha
    n = np.arange(1, nterms + 1, dtype=np.float64)
    return float(x0 ** alpha * np.sum(n ** -s * gammaincc(s, n * x0) * Gamma(s)))


def _gl_P(tau, x0=X0, alpha=ALPHA, panels=4000, upper=800.0):
    """Independent quadrature: 16-point Gauss-Legendre on panels that are
    uniform in sqrt(x - x0) (dense near the threshold)."""
    g, w = np.polynomial.legendre.leggauss(16)
    u_hi = math.sqrt(upper - x0)
    edges = np.linspace(0.0, u_hi, panels + 1)
    a, b = edges[:-1, None], edges[1:, None]
    u = 0.5 * (b - a) * g[None, :] + 0.5 * (a + b)
    wu = 0.5 * (b - a) * w[None, :]
    x = x0 + u * u
    jac = 2 * u
    phi = x * x * np.exp(-x) / -np.expm1(-x)
    sig = (x / x0) ** -alpha
    f = phi * np.exp(-tau * sig)
    norm = np.sum(phi * jac * wu)
    return float(np.sum(f * jac * wu) / norm), float(-np.sum(f * sig * jac * wu) / norm)


def test_threshold_parameter():
    # x0 = 13.6 eV / (k 5e4 K)
    assert abs(X0 - 3.156432) < 1e-5


def test_normalisation_and_slope_at_zero_closed_form():
    P0, dP0 = blackbody_P(0.0)
    assert P0 == pytest.approx(1.0, rel=1e-13)
    exact = -_series_moment(X0, ALPHA) / _series_norm(X0)
    assert dP0 == pytest.approx(exact, rel=1e-10)
    assert dP0 == pytest.approx(-0.455050, abs=2e-6)


@pytest.mark.parametrize("tau", [1e-6, 0.3, 1.0, 10.0, 100.0, 1e3, 1e4])
def test_table_values_against_independent_quadrature(tau):
    P, dP = blackbody_P(tau)
    Pg, dPg = _gl_P(tau)
    assert P == pytest.approx(Pg, rel=1e-10)
    assert dP == pytest.approx(dPg, rel=1e-10)


def test_table_shape_and_monotonicity():
    tb = oracle.blackbody_table()
    assert tb.n == 2000 and tb.lg_lo == -20 and tb.lg_hi == 4
    assert np.all(tb.P > 0) and np.all(np.diff(tb.P) <= 0)
    big = tb.tau[1:] > 1e-12          # below this P rounds to 1 in FP64
    assert np.all(np.diff(tb.P)[big] < 0)
    assert np.all(tb.dP < 0) and np.all(np.diff(-tb.dP) <= 0)   # convex, decreasing
    assert tb.P[0] == pytest.approx(1.0, abs=1e-15)


def test_interpolant_between_nodes_blackbody():
    tb = oracle.blackbody_table()
    lg = np.linspace(tb.lg_lo, tb.lg_hi, tb.n)
    rng = np.random.default_rng(7)
    ks = rng.choice(tb.n - 1, size=40, replace=False)
    for k in ks:
        tau = 10 ** (0.5 * (lg[k] + lg[k + 1]))
        P, _, _ = oracle.table_eval(tb, tau)
        Pq, _ = blackbody_P(float(tau))
        assert P[0] == pytest.approx(Pq, rel=1e-7)


def test_interpolant_grey_is_exp():
    tb = oracle.grey_table()
    taus = 10 ** np.linspace(-19.5, math.log10(79.0), 301)
    P, d1, d2 = oracle.table_eval(tb, taus)
    # cubic Hermite error bound for y = ln P = -tau = -e^x: |dy| <= h^4/384 max|y''''|
    h = (tb.lg_hi - tb.lg_lo) * math.log(10) / (tb.n - 1)
    bound = h ** 4 / 384 * taus * math.exp(h) + 1e-15
    assert np.all(np.abs(np.log(P) + taus) <= bound)
    # derivatives: below tau ~ 1e-8 the node values ln P round to a few ulp of
    # zero in FP64, so only the well-resolved range is compared
    ok = taus > 1e-8
    np.testing.assert_allclose(d1[ok], -np.exp(-taus[ok]), rtol=1e-6)
    # a cubic Hermite spline is only C1: its second derivative is O(h) accurate
    np.testing.assert_allclose(d2[taus > 1e-3], np.exp(-taus[taus > 1e-3]), rtol=2 * h)


def test_interpolant_pieces():
    tb = oracle.blackbody_table()
    # at the nodes the interpolant reproduces the table and its slope
    for k in [0, 1, 517, 1998]:
        tau = 10 ** (tb.lg_lo + k * (tb.lg_hi - tb.lg_lo) / (tb.n - 1))
        P, d1, _ = oracle.table_eval(tb, tau)
        assert P[0] == pytest.approx(tb.P[k], rel=1e-12)
        assert d1[0] == pytest.approx(tb.dP[k], rel=1e-9)
    # linear below the first node, constant above the last
    P, d1, _ = oracle.table_eval(tb, [0.0, 5e-21])
    assert P[0] == pytest.approx(tb.P[0] - tb.dP[0] * 1e-20, rel=1e-15)
    assert d1[0] == tb.dP[0] and d1[1] == tb.dP[0]
    P, d1, _ = oracle.table_eval(tb, [1e4 * 1.0000001, 1e6])
    assert np.all(P == tb.P[-1]) and np.all(d1 == 0.0)
    # the derivative is the derivative of the interpolant (central differences);
    # below tau ~ 1e-8 the FP64 node values P ~ 1 - 0.455 tau only resolve
    # 1 - P to ~1e-16, so the interpolant's slope is not meaningful there
    taus = np.array([3e-8, 2.2e-3, 0.77, 13.3, 431.0, 7777.0])
    P, d1, d2 = oracle.table_eval(tb, taus)
    h = np.maximum(taus * 1e-6, 1e-9)
    Pp, d1p, _ = oracle.table_eval(tb, taus + h)
    Pm, d1m, _ = oracle.table_eval(tb, taus - h)
    np.testing.assert_allclose(d1, (Pp - Pm) / (2 * h), rtol=1e-6)
    # (the second derivative divides by tau^2: only meaningful for tau >~ 1e-3)
    np.testing.assert_allclose(d2[1:], ((d1p - d1m) / (2 * h))[1:], rtol=1e-4)


# ---- photo-heating table H(tau) (eV): the energy analogue of eq. tables ----

KT_EV = K_B_EV * T_BB


def _series_J(s, x0, nterms=60):
    """int_x0^inf x^(s-1)/(e^x-1) dx = sum_n n^-s Gamma(s, n x0) (upper incomplete gamma)."""
    n = np.arange(1, nterms + 1, dtype=np.float64)
    return float(np.sum(n ** -s * gammaincc(s, n * x0) * Gamma(s)))


def _gl_H(tau, x0=X0, alpha=ALPHA, panels=4000, upper=800.0):
    """Independent quadrature of (H, H') in eV, as _gl_P with the weight (x - x0) kT."""
    g, w = np.polynomial.legendre.leggauss(16)
    u_hi = math.sqrt(upper - x0)
    edges = np.linspace(0.0, u_hi, panels + 1)
    a, b = edges[:-1, None], edges[1:, None]
    u = 0.5 * (b - a) * g[None, :] + 0.5 * (a + b)
    wu = 0.5 * (b - a) * w[None, :]
    x = x0 + u * u
    jac = 2 * u
    phi = x * x * np.exp(-x) / -np.expm1(-x)
    sig = (x / x0) ** -alpha
    f = phi * (x - x0) * np.exp(-tau * sig)
    norm = np.sum(phi * jac * wu)
    kT = E_TH_EV / x0
    return float(kT * np.sum(f * jac * wu) / norm), float(-kT * np.sum(f * sig * jac * wu) / norm)


def test_heating_at_zero_depth_closed_form():
    """H(0) = kT (I_3 - x0 I_2) / I_2, the mean energy above threshold of the
    emitted ionizing photons, with I_n = int_x0^inf x^n/(e^x-1) dx from the
    polylogarithm series (exact for integer n)."""
    I2 = _series_norm(X0)
    I3 = _series_J(4.0, X0)
    n = np.arange(1, 61, dtype=np.float64)
    I3_int = float(np.sum(np.exp(-n * X0) * (X0 ** 3 / n + 3 * X0 ** 2 / n ** 2 + 6 * X0 / n ** 3 + 6 / n ** 4)))
    assert I3 == pytest.approx(I3_int, rel=1e-13)
    H0, _ = oracle.tables.blackbody_H(0.0)
    assert H0 == pytest.approx(KT_EV * (I3 - X0 * I2) / I2, rel=1e-11)


@pytest.mark.parametrize("alpha", [2.8, 2.0])
def test_heating_slope_at_zero_closed_form(alpha):
    """-H'(0) = kT x0^alpha [J(4-alpha) - x0 J(3-alpha)] / I_2; for alpha = 2
    J(1) = -ln(1 - e^-x0) and J(2) = sum e^{-n x0} (x0/n + 1/n^2)."""
    _, dH0 = oracle.tables.blackbody_H(0.0, T_BB, alpha)
    I2 = _series_norm(X0)
    if alpha == 2.0:
        n = np.arange(1, 61, dtype=np.float64)
        J1 = -math.log(-math.expm1(-X0))
        J2 = float(np.sum(np.exp(-n * X0) * (X0 / n + 1 / n ** 2)))
    else:
        J1, J2 = _series_J(3.0 - alpha, X0), _series_J(4.0 - alpha, X0)
    exact = -KT_EV * X0 ** alpha * (J2 - X0 * J1) / I2
    assert dH0 == pytest.approx(exact, rel=1e-10)


@pytest.mark.parametrize("tau", [1e-6, 0.3, 1.0, 10.0, 100.0, 1e3, 1e4])
def test_heating_table_against_independent_quadrature(tau):
    H, dH = oracle.tables.blackbody_H(tau)
    Hg, dHg = _gl_H(tau)
    assert H == pytest.approx(Hg, rel=1e-10)
    assert dH == pytest.approx(dHg, rel=1e-10)


def test_heating_table_hardening():
    """Behind more absorber the photons left are harder: the mean excess
    energy of the transmitted photons (H/P) and of the absorbed ones (H'/P')
    grow with tau; H itself falls."""
    tb = oracle.blackbody_table(n=200)
    th = oracle.blackbody_heat_table(n=200)
    assert np.all(th.P > 0) and np.all(np.diff(th.P) <= 0) and np.all(th.dP < 0)
    ok = tb.tau > 1e-6   # where 1 - P is resolved in FP64
    mean_t = (th.P / tb.P)[ok]
    mean_a = (th.dP / tb.dP)[ok]
    assert np.all(np.diff(mean_t) > 0) and np.all(np.diff(mean_a) > 0)
    # absorbed photons are softer than the transmitted ones (sigma falls with nu)
    assert np.all(mean_a < mean_t)
