"""Pins of the oracle's two-absorber sweep (hydrogen and helium, the
extension the paper plans in Sections 2 and 6) against what the mathematics
fixes: the band tables add up to the hydrogen table; without helium the rate
of HI is the hydrogen-only sweep's; grey bands give closed forms on the axes
of a uniform medium; the thin limit is the bands' threshold slopes; the
columns are exact on axes and diagonals; both columns share the hydrogen
method's weights (a helium column proportional to the hydrogen one stays
proportional in any medium); superposition and linearity in Q."""
import math

import numpy as np
import pytest

import oracle
from oracle.tables import blackbody_P, blackbody_band_P
from tests.parity import assert_parity
from workloads import (HE_ABUNDANCE, HE_BAND_EDGES_EV, HE_BAND_LG_HI, helium_cross_sections,
                       make_workload)

SIG0 = oracle.SIGMA0


@pytest.fixture(scope="module")
def bands():
    sH, sHe = helium_cross_sections()
    out = []
    for b in range(len(sH)):
        t = oracle.blackbody_band_table(HE_BAND_EDGES_EV[b], HE_BAND_EDGES_EV[b + 1], n=2000,
                                        lg_hi=HE_BAND_LG_HI[b])
        out.append((t, sH[b], sHe[b]))
    return out


def test_band_tables_add_up_to_the_spectrum():
    """With the HI cross-section's shape in every band, the bands' surviving
    photons at tau_b = tau (E_b / 13.6 eV)^-2.8 add up to P(tau)."""
    sH, _ = helium_cross_sections()
    for tau in (0.0, 1e-3, 0.3, 2.0, 15.0):
        tot = sum(blackbody_band_P(tau * sH[b] / SIG0, HE_BAND_EDGES_EV[b], HE_BAND_EDGES_EV[b + 1])[0]
                  for b in range(len(sH)))
        assert tot == pytest.approx(blackbody_P(tau)[0], rel=1e-11)
        dtot = sum(sH[b] / SIG0 * blackbody_band_P(tau * sH[b] / SIG0, HE_BAND_EDGES_EV[b],
                                                   HE_BAND_EDGES_EV[b + 1])[1] for b in range(len(sH)))
        assert dtot == pytest.approx(blackbody_P(tau)[1], rel=1e-11)


def test_band_tables_end_where_their_photons_are_absorbed(bands):
    """Each band's table ends where less than 1e-20 of its photons survive,
    with values still normal FP32 numbers (the library's table format)."""
    for t, _, _ in bands:
        assert 1.2e-38 <= t.P[-1] <= 1e-20 * t.P[0]
        assert np.all(np.diff(t.P) <= 0) and np.all(t.dP <= 0)


def _he(w, bands, x_He=None, n_He=None, **kw):
    nHe = HE_ABUNDANCE * w.n_H if n_He is None else n_He
    xHe = w.x_HI if x_He is None else x_He
    return oracle.raytrace_helium(w.N, w.cell_cm, bands, w.n_H, w.x_HI, nHe, xHe, w.src.ijk, w.src.Q,
                                  w.src.R, **kw)


def test_no_helium_gives_the_hydrogen_sweep(bands):
    """x_HeI = 0: the HI rate is the hydrogen-only sweep with the full
    spectrum's table (the bands are interpolated separately, so up to the
    tables' interpolation error), and the helium column is zero.  The medium
    (lognormal density, x_HI = 0.01) keeps every optical depth of the balls
    inside both the full table (tau <= 1e4) and the bands' tables, so that
    neither side's end of table (nothing absorbed beyond it) is reached."""
    w = make_workload("c2", N=24, n_src=5, R=(3.0, 11.0))
    w.x_HI[:] = 0.01
    gH, gHe, = _he(w, bands, x_He=np.zeros_like(w.x_HI))
    o = oracle.raytrace(w.N, w.cell_cm, oracle.blackbody_table(), w.n_H, w.x_HI, w.src.ijk, w.src.Q,
                        w.src.R)
    assert_parity(gH, o, 1e-6, what="Gamma_HI without helium")
    w1 = make_workload("c2", N=24, n_src=1, R=(9.0, 9.0))
    _, _, cH, cHe = _he(w1, bands, x_He=np.zeros_like(w1.x_HI), coldens=True)
    assert np.all(cHe == 0)


def _uniform(N, nH, xH, src=(16, 16, 16), R=12.0):
    w = make_workload("c1", N=N)
    w.n_H[:] = nH
    w.x_HI[:] = xH
    w.src.ijk[:] = src
    w.src.R[:] = R
    return w


def test_grey_bands_closed_form_on_axes():
    """Grey bands P_b = w_b e^-T in a uniform medium: along the axes the
    entry optical depth of band b is (sH_b n_HI + sHe_b n_HeI) alpha (m - 1/2)
    (reading A) and the in-cell one (sH_b n_HI + sHe_b n_HeI) alpha, so each
    species' rate is Q sum_b w_b (e^-Tin - e^-Tout) s_b / (dT 4 pi alpha^2 m^2)."""
    g = oracle.grey_table()
    wts = [0.45, 0.3, 0.17, 0.08]
    sH = np.array([6.3e-18, 2.3e-18, 1.1e-18, 3.2e-19])
    sHe = np.array([0.0, 7.4e-18, 4.3e-18, 2.0e-18])
    bands = [(oracle.Table(g.lg_lo, g.lg_hi, wb * g.P, wb * g.dP), a, b) for wb, a, b in zip(wts, sH, sHe)]
    N, alpha = 32, 4.3e24
    # band optical depth per cell 0.05 .. 0.6; the fields are FP32
    nH, nHe = float(np.float32(2.0e-8)), float(np.float32(3.0e-8))
    w = _uniform(N, nH, 1.0)
    gH, gHe = oracle.raytrace_helium(N, alpha, bands, w.n_H, w.x_HI, np.full_like(w.n_H, nHe),
                                     np.ones_like(w.x_HI), w.src.ijk, w.src.Q, w.src.R)
    Q = float(w.src.Q[0])
    for m in range(1, 12):
        for d in ((m, 0, 0), (0, -m, 0), (0, 0, m)):
            c = tuple(16 + x for x in d)
            want = [0.0, 0.0]
            for wb, a, b in zip(wts, sH, sHe):
                k = (a * nH + b * nHe) * alpha
                Tin, dT = k * (m - 0.5), k
                A = Q * wb * (math.exp(-Tin) - math.exp(-Tin - dT))
                want[0] += A * a / (dT * 4 * math.pi * alpha ** 2 * m * m)
                want[1] += A * b / (dT * 4 * math.pi * alpha ** 2 * m * m)
            assert gH[c] == pytest.approx(want[0], rel=1e-7)
            assert gHe[c] == pytest.approx(want[1], rel=1e-7)


def test_thin_limit_is_the_bands_threshold_slope(bands):
    """n -> 0: Gamma_i 4 pi alpha^2 r^2 / Q -> sum_b s_i,b (-P_b'(0)), with
    P_b'(0) from the quadrature itself (independent of the table nodes)."""
    N, alpha = 32, 4.3e24
    w = _uniform(N, 1e-16, 1.0)
    gH, gHe = _he(w, bands, n_He=np.full_like(w.n_H, 1e-16), x_He=np.ones_like(w.x_HI))
    sH, sHe = helium_cross_sections()
    slopes = [-blackbody_band_P(0.0, HE_BAND_EDGES_EV[b], HE_BAND_EDGES_EV[b + 1])[1] for b in range(len(sH))]
    wantH = sum(a * s for a, s in zip(sH, slopes))
    wantHe = sum(a * s for a, s in zip(sHe, slopes))
    Q = float(w.src.Q[0])
    for d in ((3, 0, 0), (2, 2, 1), (5, -4, 3), (0, 0, -11)):
        c = tuple(16 + x for x in d)
        r2 = sum(x * x for x in d)
        k = 4 * math.pi * alpha ** 2 * r2 / Q
        assert gH[c] * k == pytest.approx(wantH, rel=1e-6)
        assert gHe[c] * k == pytest.approx(wantHe, rel=1e-6)


def test_columns_exact_on_axes_and_diagonals(bands):
    """Uniform medium, reading A: both entry columns are n alpha sqrt(d) (m - 1/2)
    along axes (d = 1) and face and body diagonals (d = 2, 3)."""
    N, alpha = 32, 4.3e24
    nH, nHe = float(np.float32(1.5e-4)), float(np.float32(1.2e-5))   # the fields are FP32
    w = _uniform(N, nH, 1.0, R=14.0)
    _, _, cH, cHe = _he(w, bands, n_He=np.full_like(w.n_H, nHe), x_He=np.ones_like(w.x_HI), coldens=True)
    for m in range(1, 8):
        for d, k in (((m, 0, 0), 1), ((0, m, -m), 2), ((-m, m, m), 3)):
            c = tuple(16 + x for x in d)
            assert cH[c] == pytest.approx(nH * alpha * math.sqrt(k) * (m - 0.5), rel=1e-12)
            assert cHe[c] == pytest.approx(nHe * alpha * math.sqrt(k) * (m - 0.5), rel=1e-12)


def test_columns_share_the_hydrogen_weights(bands):
    """A helium density proportional to the hydrogen one (n_HeI = c n_HI in
    every cell) gives a helium column c times the hydrogen one everywhere, in
    a lognormal medium where the optical-depth weights vary from cell to cell:
    both columns are carried with the same weights."""
    w = make_workload("c2", N=24, n_src=1, R=(11.0, 11.0))
    c = 0.37
    _, _, cH, cHe = _he(w, bands, n_He=c * w.n_H.astype(np.float64), x_He=w.x_HI, coldens=True)
    ball = cH > 0
    np.testing.assert_allclose(cHe[ball], c * cH[ball], rtol=1e-12)


def test_superposition_and_linearity(bands):
    w = make_workload("c2", N=20, n_src=4, R=(3.0, 8.0))
    gH, gHe = _he(w, bands)
    w3 = make_workload("c2", N=20, n_src=4, R=(3.0, 8.0))
    w3.src.Q[:] *= 3.0
    gH3, gHe3 = _he(w3, bands)
    np.testing.assert_allclose(gH3, 3.0 * gH, rtol=1e-13, atol=0)
    np.testing.assert_allclose(gHe3, 3.0 * gHe, rtol=1e-13, atol=0)
    tot = [0.0, 0.0]
    for idx in ([0, 1], [2, 3]):
        part = make_workload("c2", N=20, n_src=4, R=(3.0, 8.0))
        part.src = w.src.subset(idx)
        h, he = _he(part, bands)
        tot = [tot[0] + h, tot[1] + he]
    np.testing.assert_allclose(tot[0], gH, rtol=1e-12, atol=1e-14 * gH.max())
    np.testing.assert_allclose(tot[1], gHe, rtol=1e-12, atol=1e-14 * gHe.max())
