"""Oracle photoionization tables (test infrastructure only).

P(tau) = gamma(tau / sigma0) / gamma(0), eq. tables of Section 2.2 normalised
so that P(0) = 1, and its derivative dP/dtau, for

* a black-body source of temperature T with a power-law cross-section
  sigma(nu) = sigma0 (nu / nu_th)^-alpha (the spectra of Section 4.1, Test 3):
  with x = h nu / k T and x0 = 13.6 eV / k T,
      P(tau)  =  int_x0^inf phi(x) exp(-tau (x/x0)^-alpha) dx / int_x0^inf phi(x) dx,
      P'(tau) = -int_x0^inf phi(x) (x/x0)^-alpha exp(-tau (x/x0)^-alpha) dx / (same),
  where phi(x) = x^2 / (e^x - 1) is the photon-number spectrum L_nu/(h nu);
* grey opacity (sigma = sigma0), where P = exp(-tau) exactly;

the band tables of the same black body split at photon energies (several
absorbers, hydrogen and helium): with a band [x_a, x_b) and its optical depth
tau measured at the lower edge x_a,
      P_b(tau)  =  int_xa^xb phi(x) exp(-tau (x/x_a)^-alpha) dx / int_x0^inf phi(x) dx,
so that the bands of a spectrum with tau_b = tau (x_a/x0)^-alpha add up to
P(tau);

and the photo-heating table of the same black body (the energy analogue of
eq. tables: the paper leaves heating out and names it as a planned
extension, Sections 2 and 6), in eV per emitted photon,
      H(tau)  =  k T int_x0^inf phi(x) (x - x0) exp(-tau (x/x0)^-alpha) dx / int_x0^inf phi(x) dx,
      H'(tau) = -k T int_x0^inf phi(x) (x - x0) (x/x0)^-alpha exp(..) dx / (same):
the energy above the threshold that the photons still carry after optical
depth tau, so that Q [H(tau_in) - H(tau_out)] is what a cell absorbs as
photo-electron energy, exactly as Q [P(tau_in) - P(tau_out)] counts its
ionizations.

The integrals use SciPy's adaptive QUADPACK quadrature over fixed sub-ranges
(the paper's table build also used SciPy quad, Section 3.4).  The upper limit
800 stands for infinity: the integrand is below e^-700 relative there.
"""
from __future__ import annotations

import dataclasses
import functools
import math

import numpy as np
from scipy.integrate import quad

K_B_EV = 8.617333262e-5       # Boltzmann constant, eV / K
E_TH_EV = 13.6                # hydrogen ionization threshold, eV
SIGMA0 = 6.3e-18              # HI cross-section at threshold, cm^2


@dataclasses.dataclass(frozen=True)
class Table:
    lg_lo: float
    lg_hi: float
    P: np.ndarray        # float64 [n]
    dP: np.ndarray       # float64 [n]

    @property
    def n(self) -> int:
        return int(self.P.shape[0])

    @property
    def tau(self) -> np.ndarray:
        return 10.0 ** np.linspace(self.lg_lo, self.lg_hi, self.n)


_BREAKS = (1.0, 3.0, 6.0, 10.0, 20.0, 40.0, 80.0, 160.0, 320.0, 800.0)


def _integral(f, x0: float) -> float:
    pts = [x0] + [b for b in _BREAKS if b > x0 + 1e-9]
    tot = 0.0
    for a, b in zip(pts[:-1], pts[1:]):
        tot += quad(f, a, b, epsabs=0.0, epsrel=1e-13, limit=400)[0]
    return tot


def blackbody_P(tau: float, T: float = 5e4, alpha: float = 2.8):
    """(P(tau), P'(tau)) for a black body of temperature T."""
    x0 = E_TH_EV / (K_B_EV * T)
    phi = lambda x: x * x * math.exp(-x) / -math.expm1(-x)   # x^2/(e^x-1)
    norm = _integral(phi, x0)
    P = _integral(lambda x: phi(x) * math.exp(-tau * (x / x0) ** -alpha), x0) / norm
    dP = -_integral(lambda x: phi(x) * (x / x0) ** -alpha * math.exp(-tau * (x / x0) ** -alpha), x0) / norm
    return P, dP


def blackbody_band_P(tau: float, e_lo: float, e_hi: float, T: float = 5e4, alpha: float = 2.8):
    """(P_b(tau), P_b'(tau)) of the band [e_lo, e_hi) eV (e_hi = inf: open),
    tau measured at e_lo, per photon emitted above 13.6 eV."""
    kT = K_B_EV * T
    x0, xa = E_TH_EV / kT, e_lo / kT
    xb = e_hi / kT if math.isfinite(e_hi) else _BREAKS[-1]
    phi = lambda x: x * x * math.exp(-x) / -math.expm1(-x)
    norm = _integral(phi, x0)

    def band(f):
        pts = [xa] + [b for b in _BREAKS if xa + 1e-9 < b < xb] + [xb]
        return sum(quad(f, a, b, epsabs=0.0, epsrel=1e-13, limit=400)[0] for a, b in zip(pts[:-1], pts[1:]))

    P = band(lambda x: phi(x) * math.exp(-tau * (x / xa) ** -alpha)) / norm
    dP = -band(lambda x: phi(x) * (x / xa) ** -alpha * math.exp(-tau * (x / xa) ** -alpha)) / norm
    return P, dP


@functools.lru_cache(maxsize=16)
def blackbody_band_table(e_lo: float, e_hi: float, T: float = 5e4, alpha: float = 2.8, n: int = 2000,
                         lg_lo: float = -20.0, lg_hi: float = 2.5) -> Table:
    """P_b and P_b' of one band on n nodes uniform in log10 tau."""
    taus = 10.0 ** np.linspace(lg_lo, lg_hi, n)
    P = np.empty(n)
    dP = np.empty(n)
    for k, t in enumerate(taus):
        P[k], dP[k] = blackbody_band_P(float(t), e_lo, e_hi, T, alpha)
    P.setflags(write=False)
    dP.setflags(write=False)
    return Table(lg_lo, lg_hi, P, dP)


def blackbody_H(tau: float, T: float = 5e4, alpha: float = 2.8):
    """(H(tau), H'(tau)) in eV for a black body of temperature T."""
    kT = K_B_EV * T
    x0 = E_TH_EV / kT
    phi = lambda x: x * x * math.exp(-x) / -math.expm1(-x)
    norm = _integral(phi, x0)
    H = _integral(lambda x: phi(x) * (x - x0) * math.exp(-tau * (x / x0) ** -alpha), x0) / norm
    dH = -_integral(lambda x: phi(x) * (x - x0) * (x / x0) ** -alpha * math.exp(-tau * (x / x0) ** -alpha),
                    x0) / norm
    return kT * H, kT * dH


@functools.lru_cache(maxsize=8)
def blackbody_heat_table(T: float = 5e4, alpha: float = 2.8, n: int = 2000,
                         lg_lo: float = -20.0, lg_hi: float = 4.0) -> Table:
    """H(tau) and H'(tau) (eV) on the node grid of blackbody_table."""
    taus = 10.0 ** np.linspace(lg_lo, lg_hi, n)
    H = np.empty(n)
    dH = np.empty(n)
    for k, t in enumerate(taus):
        H[k], dH[k] = blackbody_H(float(t), T, alpha)
    H.setflags(write=False)
    dH.setflags(write=False)
    return Table(lg_lo, lg_hi, H, dH)


@functools.lru_cache(maxsize=8)
def blackbody_table(T: float = 5e4, alpha: float = 2.8, n: int = 2000,
                    lg_lo: float = -20.0, lg_hi: float = 4.0) -> Table:
    taus = 10.0 ** np.linspace(lg_lo, lg_hi, n)
    P = np.empty(n)
    dP = np.empty(n)
    for k, t in enumerate(taus):
        P[k], dP[k] = blackbody_P(float(t), T, alpha)
    P.setflags(write=False)
    dP.setflags(write=False)
    return Table(lg_lo, lg_hi, P, dP)


@functools.lru_cache(maxsize=8)
def grey_table(n: int = 2000, lg_lo: float = -20.0, lg_hi: float = math.log10(80.0)) -> Table:
    """P = exp(-tau): exact, no quadrature.  The upper end stays below the
    FP32 underflow of exp(-tau)."""
    taus = 10.0 ** np.linspace(lg_lo, lg_hi, n)
    P = np.exp(-taus)
    dP = -np.exp(-taus)
    P.setflags(write=False)
    dP.setflags(write=False)
    return Table(lg_lo, lg_hi, P, dP)
