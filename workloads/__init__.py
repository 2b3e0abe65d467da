"""Seeded synthetic inputs for the ASORA ray-tracing step.

This module is shared by the FP64 oracle, the tests and the benchmark.  It
holds no arithmetic of the method itself: it only draws density fields,
neutral-fraction fields and source lists, with the shapes, value
distributions and structure of the workloads the paper benchmarks (a 250^3
cosmological grid with 1.4 Mpc cells, thousands to a million halo sources,
ray-tracing radii of tens of cells; Section 4.2 and Section 5).  The paper's
N-body density fields and halo catalogues are not available, so a lognormal
Gaussian-random field and uniformly placed sources with log-uniform photon
rates stand in for them.

Every generator takes an explicit seed and uses numpy's PCG64.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

MPC_CM = 3.0856775814913673e24

__all__ = [
    "Sources", "Workload", "gaussian_field", "lognormal_density",
    "bubble_xhi", "smoothed_threshold_xhi", "random_sources", "make_workload",
    "CONFIGS", "HE_BAND_EDGES_EV", "HE_BAND_LG_HI", "HE_ABUNDANCE", "helium_cross_sections",
]


@dataclasses.dataclass
class Sources:
    ijk: np.ndarray      # int32 [n, 3], cell indices (C order: i slowest)
    Q: np.ndarray        # float64 [n], ionizing photons per second
    R: np.ndarray        # float32 [n], ray-tracing radius in cells

    def __len__(self) -> int:
        return int(self.ijk.shape[0])

    def subset(self, idx) -> "Sources":
        return Sources(np.ascontiguousarray(self.ijk[idx]),
                       np.ascontiguousarray(self.Q[idx]),
                       np.ascontiguousarray(self.R[idx]))


@dataclasses.dataclass
class Workload:
    name: str
    N: int
    cell_cm: float
    n_H: np.ndarray      # float32 [N, N, N] total hydrogen density, cm^-3
    x_HI: np.ndarray     # float32 [N, N, N] neutral fraction
    src: Sources
    seed: int
    recipe: str

    @property
    def work_sphere(self) -> float:
        """Sum over sources of (4/3) pi R^3, the paper's per-voxel normaliser."""
        R = self.src.R.astype(np.float64)
        return float(np.sum(4.0 / 3.0 * math.pi * R ** 3))


def _rngs(seed: int, n: int):
    return [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(n)]


def _kgrid(N: int):
    k1 = np.fft.fftfreq(N) * N
    k3 = np.fft.rfftfreq(N) * N
    return (k1[:, None, None] ** 2 + k1[None, :, None] ** 2 + k3[None, None, :] ** 2)


def gaussian_field(N: int, rng, slope: float = -2.0, smooth_sigma: float | None = None):
    """Unit-variance Gaussian random field with power spectrum |k|^slope.

    White noise is shaped in Fourier space by |k|^(slope/2); the k = 0 mode
    is removed.  If smooth_sigma is given, a second field smoothed with a
    Gaussian kernel of that width (in cells) is also returned.
    """
    white = rng.standard_normal((N, N, N))
    wk = np.fft.rfftn(white)
    del white
    k2 = _kgrid(N)
    with np.errstate(divide="ignore"):
        amp = np.where(k2 > 0, k2 ** (slope / 4.0), 0.0)
    gk = wk * amp
    del wk, amp
    g = np.fft.irfftn(gk, s=(N, N, N), axes=(0, 1, 2))
    g /= g.std()
    if smooth_sigma is None:
        return g
    kk = k2 * (2.0 * math.pi / N) ** 2
    gs = np.fft.irfftn(gk * np.exp(-0.5 * kk * smooth_sigma ** 2), s=(N, N, N), axes=(0, 1, 2))
    return g, gs


def lognormal_density(g: np.ndarray, mean_nH: float = 1.5e-4, ln_sigma: float = 0.5):
    """n_H = mean_nH * exp(ln_sigma * g - ln_sigma^2 / 2): lognormal with unit mean."""
    delta = np.exp(ln_sigma * g - 0.5 * ln_sigma ** 2)
    return (mean_nH * delta).astype(np.float32)


def bubble_xhi(N: int, centres: np.ndarray, rng, r_lo: float = 2.0, r_hi: float = 8.0,
               ionized: float = 1e-3) -> np.ndarray:
    """x_HI = 1 except periodic balls of radius U[r_lo, r_hi] around centres."""
    x = np.ones((N, N, N), dtype=np.float32)
    n = centres.shape[0]
    radii = rng.uniform(r_lo, r_hi, size=n)
    rmax = int(math.ceil(r_hi))
    ax = np.arange(-rmax, rmax + 1)
    oi, oj, ok = np.meshgrid(ax, ax, ax, indexing="ij")
    off = np.stack([oi.ravel(), oj.ravel(), ok.ravel()], axis=1)
    d2 = (off ** 2).sum(axis=1)
    flat = x.reshape(-1)
    chunk = max(1, 2_000_000 // off.shape[0])
    for s in range(0, n, chunk):
        c = centres[s:s + chunk].astype(np.int64)
        r2 = radii[s:s + chunk] ** 2
        inside = d2[None, :] <= r2[:, None]
        src_id, off_id = np.nonzero(inside)
        p = (c[src_id] + off[off_id]) % N
        flat[(p[:, 0] * N + p[:, 1]) * N + p[:, 2]] = ionized
    return x


def smoothed_threshold_xhi(gs: np.ndarray, ionized: float = 1e-3) -> np.ndarray:
    """x_HI = ionized where the smoothed field exceeds its median, else 1 (about half ionized)."""
    med = np.median(gs)
    return np.where(gs > med, np.float32(ionized), np.float32(1.0)).astype(np.float32)


def random_sources(N: int, n: int, rng, lgQ=(51.0, 55.0), R=(30.0, 30.0)) -> Sources:
    """Integer source cells uniform in [0, N)^3, log-uniform Q, uniform R (cells)."""
    ijk = rng.integers(0, N, size=(n, 3)).astype(np.int32)
    Q = 10.0 ** rng.uniform(lgQ[0], lgQ[1], size=n)
    if R[0] == R[1]:
        Rv = np.full(n, R[0], dtype=np.float32)
    else:
        Rv = rng.uniform(R[0], R[1], size=n).astype(np.float32)
    return Sources(ijk, Q.astype(np.float64), Rv)


# Helium as a second absorber (inputs of the two-species sweep).  The
# spectrum above 13.6 eV is split into bands at 24.59 eV (the HeI threshold),
# 35 eV and 54.42 eV (the HeII threshold, kept as a band edge only); per band
# the upper end of its table in log10 of the optical depth at its lower edge
# (its photons are absorbed to below about 1e-30 there), and the
# cross-sections of HI (the paper's law, 6.3e-18 cm^2 (E/13.6 eV)^-2.8) and
# HeI (the measured cross-section's fit 7.42e-18 cm^2 [1.66 (E/24.59 eV)^-2.05
# - 0.66 (E/24.59 eV)^-3.05]) at the band's lower edge E.  Helium by number
# n_He = 0.0789 n_H (mass fraction 0.24); x_HeI follows x_HI (helium singly
# ionized where hydrogen is ionized).
HE_BAND_EDGES_EV = (13.6, 24.59, 35.0, 54.42, math.inf)
HE_BAND_LG_HI = (2.5, 2.2, 2.3, 3.3)
HE_ABUNDANCE = 0.0789


def helium_cross_sections():
    """(sigma_HI, sigma_HeI) in cm^2 at the lower edge of every band."""
    sH, sHe = [], []
    for e in HE_BAND_EDGES_EV[:-1]:
        sH.append(6.3e-18 * (e / 13.6) ** -2.8)
        r = e / 24.59
        sHe.append(7.42e-18 * (1.66 * r ** -2.05 - 0.66 * r ** -3.05) if e >= 24.59 else 0.0)
    return np.array(sH), np.array(sHe)


# The five workloads, with their recipe.  Cell sizes: 1.4 Mpc is rounded to
# 4.3e24 cm, 1.396 Mpc (the 349 cMpc / 250 box of Section 5) to 4.308e24 cm.
CONFIGS = {
    "c1": dict(N=32, cell_cm=4.3e24, field="uniform", n_src=1, lgQ=(54.0, 54.0), R=(15.0, 15.0)),
    "c2": dict(N=128, cell_cm=4.3e24, field="lognormal+bubbles", n_src=1000, lgQ=(51.0, 55.0), R=(30.0, 30.0)),
    "c3": dict(N=250, cell_cm=4.308e24, field="lognormal+bubbles", n_src=100_000, lgQ=(50.0, 55.0), R=(5.0, 50.0)),
    "c4": dict(N=64, cell_cm=4.3e24, field="lognormal+bubbles", n_src=64, lgQ=(51.0, 55.0), R=(20.0, 20.0)),
    "c5": dict(N=250, cell_cm=4.308e24, field="lognormal+smoothed", n_src=1_000_000, lgQ=(50.0, 54.0), R=(5.0, 40.0)),
}
_CONFIG_SEED = {"c1": 1001, "c2": 1002, "c3": 1003, "c4": 1004, "c5": 1005}


def make_workload(name: str, seed: int | None = None, **override) -> Workload:
    """Build one of CONFIGS (optionally with fields overridden, e.g. N or n_src)."""
    cfg = dict(CONFIGS[name])
    cfg.update(override)
    seed = _CONFIG_SEED.get(name, 1000) if seed is None else seed
    N = int(cfg["N"])
    r_field, r_src, r_bub = _rngs(seed, 3)
    if cfg["field"] == "uniform":
        n_H = np.full((N, N, N), 1.5e-4, dtype=np.float32)
        x_HI = np.ones((N, N, N), dtype=np.float32)
        src = Sources(np.array([[N // 2] * 3], dtype=np.int32),
                      np.array([10.0 ** cfg["lgQ"][0]]), np.array([cfg["R"][0]], dtype=np.float32))
        if cfg["n_src"] != 1:
            src = random_sources(N, cfg["n_src"], r_src, cfg["lgQ"], cfg["R"])
        recipe = "uniform n_H=1.5e-4, x_HI=1"
    elif cfg["field"] == "lognormal+bubbles":
        g = gaussian_field(N, r_field)
        n_H = lognormal_density(g)
        del g
        src = random_sources(N, cfg["n_src"], r_src, cfg["lgQ"], cfg["R"])
        x_HI = bubble_xhi(N, src.ijk, r_bub)
        recipe = "lognormal(ln sigma 0.5, P(k)~k^-2) x 1.5e-4; x_HI=1e-3 in U[2,8]-cell balls around sources"
    elif cfg["field"] == "lognormal+smoothed":
        g, gs = gaussian_field(N, r_field, smooth_sigma=3.0)
        n_H = lognormal_density(g)
        del g
        x_HI = smoothed_threshold_xhi(gs)
        del gs
        src = random_sources(N, cfg["n_src"], r_src, cfg["lgQ"], cfg["R"])
        recipe = "lognormal x 1.5e-4; x_HI=1e-3 where sigma=3 smoothed field > median"
    else:
        raise ValueError(cfg["field"])
    return Workload(name, N, float(cfg["cell_cm"]), np.ascontiguousarray(n_H),
                    np.ascontiguousarray(x_HI), src, seed, recipe)
