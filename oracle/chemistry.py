"""FP64 oracle of the hydrogen chemistry step and of one time step of the
ray-tracing <-> chemistry iteration -- TEST INFRASTRUCTURE ONLY (tests, the
smoke check and the CPU-baseline leg of the benchmark may use it).

The chemistry equation (Section 2.1, eq. chemistry) is

    dx/dt = (1 - x) (Gamma + n_e C_H) - x n_e alpha_H,     x = x_HII,

and the chemistry step takes its time-averaged solution over a step dt with
Gamma, n_e, C_H and alpha_H held fixed (Section 2.1, eq. time_avrg_sol):

    x_eq = (Gamma + n_e C_H) / (Gamma + n_e (C_H + alpha_H)),
    t_i  = 1 / (Gamma + n_e (C_H + alpha_H)),
    <x>  = x_eq + (x0 - x_eq) (1 - exp(-dt/t_i)) t_i / dt,

iterating the electron density n_e = n_H <x> until <x> converges (Section
2.1).  The end-of-step state is the same solution at t = dt,
x(dt) = x_eq + (x0 - x_eq) exp(-dt/t_i).

Everything here is carried in the neutral fraction y = 1 - x, for which the
same formulas read y_eq = n_e alpha_H t_i, <y> = y_eq + (y0 - y_eq)(1 -
exp(-dt/t_i)) t_i/dt, y(dt) = y_eq + (y0 - y_eq) exp(-dt/t_i): no
difference of nearly equal numbers where the gas is almost fully ionized.

Readings of points the paper leaves open:
  * n_e = n_H <x_HII> (the paper: "roughly n_e ~ x_HII n_H"; hydrogen only,
    no electrons from other species), starting from n_H x0;
  * the n_e iteration of a cell stops when |<y>_new - <y>_old| <= rtol <y>_new
    (rtol = 1e-12) or after max_iter = 100 passes;
  * (1 - exp(-dt/t_i)) t_i/dt is taken as -expm1(-u)/u with u = dt/t_i, and
    as 1 for u = 0;
  * one time step (Section 2.1, the flowchart): the ray tracing runs on the
    time-averaged neutral fraction <y> (the start-of-step y0 the first
    time), the chemistry step turns the summed Gamma into a new <y>, and the
    two alternate until at most conv_frac of the cells changed <y> by more
    than conv_rtol relative (1e-3 and 1e-4 here: the paper implies a
    convergence test without giving one), or n_iter passes if given.
"""
from __future__ import annotations

import numpy as np

# case-B recombination coefficient of hydrogen at T = 1e4 K (Section 4.1, Test 1)
ALPHA_B_1E4 = 2.59e-13
MYR = 3.15576e13          # seconds per Myr (Julian years)
KPC = 3.0856775814913673e21   # cm


def time_average(gamma, n_e, y0, dt, alpha, c_h):
    """(<y>, y(dt)) of the time-averaged solution for fixed Gamma, n_e
    (arrays of the grid's shape), dt, alpha_H and C_H."""
    rate = gamma + n_e * (c_h + alpha)
    y_eq = np.where(rate > 0, n_e * alpha / np.where(rate > 0, rate, 1.0), 1.0)
    u = rate * dt
    decay = np.exp(-u)
    frac = np.where(u > 0, -np.expm1(-u) / np.where(u > 0, u, 1.0), 1.0)   # (1 - e^-u) / u
    y_avg = y_eq + (y0 - y_eq) * frac
    y_end = y_eq + (y0 - y_eq) * decay
    return y_avg, y_end


def chemistry_step(gamma, n_H, y0, dt, alpha=ALPHA_B_1E4, c_h=0.0, rtol=1e-12, max_iter=100):
    """One chemistry step, cell by cell: the time-averaged neutral fraction
    <y> and the end-of-step y(dt) for the time-averaged rate gamma, with the
    electron density iterated as n_e = n_H (1 - <y>).  Returns
    (y_avg, y_end, passes) with passes the number of n_e passes per cell."""
    gamma = np.asarray(gamma, np.float64)
    n_H = np.asarray(n_H, np.float64)
    y0 = np.asarray(y0, np.float64)
    y_avg = y0.copy()
    y_end = y0.copy()
    passes = np.zeros(y0.shape, np.int32)
    active = np.ones(y0.shape, bool)
    for _ in range(max_iter):
        n_e = n_H * (1.0 - y_avg)
        a, e = time_average(gamma, n_e, y0, dt, alpha, c_h)
        done = np.abs(a - y_avg) <= rtol * a
        y_end = np.where(active, e, y_end)
        y_avg = np.where(active, a, y_avg)
        passes = passes + active
        active = active & ~done
        if not active.any():
            break
    return y_avg, y_end, passes


def time_step(rt, n_H, y0, dt, alpha=ALPHA_B_1E4, c_h=0.0, conv_rtol=1e-3, conv_frac=1e-4,
              max_passes=50, n_iter=None):
    """One time step of the ray-tracing <-> chemistry iteration.  rt(y) is
    the ray tracing: the summed Gamma of all sources for neutral fraction y.
    Returns (y_end, y_avg, gamma, passes)."""
    y_avg = np.asarray(y0, np.float64).copy()
    n = y_avg.size
    passes = 0
    while True:
        gamma = rt(y_avg)
        new_avg, y_end, _ = chemistry_step(gamma, n_H, y0, dt, alpha, c_h)
        changed = np.count_nonzero(np.abs(new_avg - y_avg) > conv_rtol * new_avg)
        y_avg = new_avg
        passes += 1
        if n_iter is not None:
            if passes >= n_iter:
                break
        elif changed <= conv_frac * n or passes >= max_passes:
            break
    return y_end, y_avg, gamma, passes


def stromgren(ndot, n_H, alpha=ALPHA_B_1E4):
    """(r_S [cm], t_rec [s]) of a source of ndot ionizing photons per second in
    uniform gas of density n_H (Section 4.1, Test 1)."""
    r_s = (3.0 * ndot / (4.0 * np.pi * alpha * n_H ** 2)) ** (1.0 / 3.0)
    return r_s, 1.0 / (alpha * n_H)


def ifront_radius(t, r_s, t_rec):
    """Analytic I-front radius r_S (1 - exp(-t/t_rec))^(1/3) (Section 4.1,
    eq. rI1)."""
    return r_s * (1.0 - np.exp(-np.asarray(t, np.float64) / t_rec)) ** (1.0 / 3.0)


def ifront_along_axis(y_line, cell_cm, start):
    """Distance from the source cell at index `start` of a line of cells to
    where the neutral fraction first reaches 0.5 outward (+ direction),
    located within a cell by linear interpolation between cell centres
    (Section 4.1: the radius where x_HI = 0.5)."""
    y = np.asarray(y_line, np.float64)[start:]
    above = np.nonzero(y >= 0.5)[0]
    if len(above) == 0:
        return float(len(y)) * cell_cm
    k = above[0]
    if k == 0:
        return 0.0
    f = (0.5 - y[k - 1]) / (y[k] - y[k - 1])
    return (k - 1 + f) * cell_cm
