"""Pins of the chemistry oracle (oracle/chemistry.py): the time-averaged
solution of the chemistry equation against an independent ODE integration,
its fixed points and limits, and the single-source H II region of Test 1
(Section 4.1) end to end against the paper's printed Stromgren values and the
analytic I-front."""
import json
import math
import os

import numpy as np
import pytest
from scipy.integrate import solve_ivp

import oracle
from oracle import chemistry as ch

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "test1_stromgren.json")))


def test_stromgren_values_printed_in_the_paper():
    r_s, t_rec = ch.stromgren(GOLD["ndot_per_s"], GOLD["n_H_cm3"], GOLD["alpha_B_cm3_per_s"])
    assert round(r_s / ch.KPC, 2) == GOLD["r_S_kpc"]
    assert round(t_rec / ch.MYR, 2) == GOLD["t_rec_Myr"]


@pytest.mark.parametrize("gamma,n_e,y0,dt,c_h", [
    (1e-13, 1e-3, 1.0, 3e14, 0.0),          # neutral gas lit up
    (2e-14, 5e-4, 0.3, 1e15, 1e-15),        # partly ionized, with collisions
    (0.0, 1e-3, 1e-4, 2e15, 0.0),           # recombination only
    (5e-12, 1e-2, 0.7, 1e12, 3e-16),        # fast ionization, short step
])
def test_time_average_matches_ode(gamma, n_e, y0, dt, c_h):
    """With n_e held fixed the chemistry equation is linear in y; integrate it
    (and its running integral) numerically and compare <y> and y(dt)."""
    alpha = ch.ALPHA_B_1E4

    def rhs(t, s):
        y = s[0]
        dy = (1.0 - y) * n_e * alpha - y * (gamma + n_e * c_h)   # d(1 - x)/dt = -dx/dt
        return [dy, y]

    sol = solve_ivp(rhs, (0.0, dt), [y0, 0.0], method="Radau", rtol=1e-12, atol=1e-20)
    y_end_ode, integral = sol.y[0, -1], sol.y[1, -1]
    y_avg, y_end = ch.time_average(np.array(gamma), np.array(n_e), np.array(y0), dt, alpha, c_h)
    np.testing.assert_allclose(y_end, y_end_ode, rtol=1e-8, atol=1e-14)
    np.testing.assert_allclose(y_avg, integral / dt, rtol=1e-8, atol=1e-14)


def test_equilibrium_is_a_fixed_point():
    """A cell already at the equilibrium of its own electron density stays."""
    rng = np.random.default_rng(3)
    n_H = 10 ** rng.uniform(-4, -2, 50)
    y0 = 10 ** rng.uniform(-5, -0.01, 50)
    alpha, c_h = ch.ALPHA_B_1E4, 1e-16
    n_e = n_H * (1.0 - y0)
    gamma = n_e * alpha / y0 - n_e * (c_h + alpha)       # y_eq(gamma, n_e) = y0
    y_avg, y_end, _ = ch.chemistry_step(gamma, n_H, y0, 5e14, alpha, c_h)
    np.testing.assert_allclose(y_avg, y0, rtol=1e-10)
    np.testing.assert_allclose(y_end, y0, rtol=1e-10)


def test_electron_density_iteration_is_self_consistent():
    rng = np.random.default_rng(4)
    n = 200
    gamma = np.where(rng.random(n) < 0.2, 0.0, 10 ** rng.uniform(-16, -11, n))
    n_H = 10 ** rng.uniform(-4, -2, n)
    y0 = rng.uniform(0, 1, n)
    y_avg, y_end, passes = ch.chemistry_step(gamma, n_H, y0, 1.6e15)
    assert passes.max() < 100
    a, e = ch.time_average(gamma, n_H * (1.0 - y_avg), y0, 1.6e15, ch.ALPHA_B_1E4, 0.0)
    np.testing.assert_allclose(a, y_avg, rtol=1e-11)
    np.testing.assert_allclose(e, y_end, rtol=1e-10)
    assert np.all((y_avg >= 0) & (y_avg <= 1)) and np.all((y_end >= 0) & (y_end <= 1))


def test_zero_step_keeps_the_state():
    y0 = np.array([1.0, 0.5, 1e-6])
    y_avg, y_end, _ = ch.chemistry_step(np.array([1e-12, 0.0, 1e-10]), np.full(3, 1e-3), y0, 0.0)
    np.testing.assert_array_equal(y_avg, y0)
    np.testing.assert_array_equal(y_end, y0)


def _run_test1(N, steps, dt_myr):
    box = GOLD["box_kpc"] * ch.KPC
    cell = box / N
    ndot, nH0 = GOLD["ndot_per_s"], GOLD["n_H_cm3"]
    tab = oracle.grey_table()
    c = N // 2
    ijk = np.array([[c, c, c]], np.int32)
    Q, R = np.array([ndot]), np.array([N / 2 - 0.5])
    n_H = np.full((N, N, N), nH0)
    y = np.ones((N, N, N))
    out = []
    for k in range(steps):
        rt = lambda yv: oracle.raytrace(N, cell, tab, n_H, yv, ijk, Q, R)
        y, y_avg, gam, passes = ch.time_step(rt, n_H, y, dt_myr * ch.MYR)
        out.append(ch.ifront_along_axis(y[c, c, :], cell, c))
    return np.array(out), y, n_H, cell


def test_single_source_hii_region_end_to_end():
    """Test 1 on a 40^3 grid with the paper's parameters and coarse step: the
    I-front follows r_S (1 - exp(-t/t_rec))^(1/3) within the few percent the
    paper reports (an overshoot of up to 6 % late), and after about four
    recombination times recombinations balance the source's photons."""
    dt = GOLD["dt_coarse_Myr"]
    steps = int(round(GOLD["t_evo_Myr"] / dt))
    r_i, y, n_H, cell = _run_test1(40, steps, dt)
    r_s, t_rec = ch.stromgren(GOLD["ndot_per_s"], GOLD["n_H_cm3"])
    t = dt * ch.MYR * np.arange(1, steps + 1)
    ratio = r_i / ch.ifront_radius(t, r_s, t_rec)
    assert np.all(ratio > 0.93) and np.all(ratio < 1.0 + GOLD["late_overshoot_max"] + 0.04), ratio
    rec = np.sum(ch.ALPHA_B_1E4 * (n_H * (1.0 - y)) ** 2) * cell ** 3
    assert 0.9 < rec / GOLD["ndot_per_s"] < 1.0 + 1e-6
