"""Parity metric shared by the tests: relative error with a floor.

rel = max |g - o| / |o| over cells with |o| >= floor * max|o|; every other
cell must satisfy |g - o| <= tol * floor * max|o|; cells where o = 0 must be
0 (the region beyond the ray-tracing radius and beyond the table)."""
import numpy as np


def floored_rel(g, o, floor=1e-20):
    g = np.asarray(g, np.float64)
    o = np.asarray(o, np.float64)
    omax = np.abs(o).max() if o.size else 0.0
    if omax == 0:
        return 0.0, float(np.abs(g).max() if g.size else 0.0), 0
    big = np.abs(o) >= floor * omax
    rel = float((np.abs(g - o)[big] / np.abs(o[big])).max())
    small_abs = float(np.abs(g - o)[~big].max()) / (floor * omax) if (~big).any() else 0.0
    return rel, small_abs, int(big.sum())


def assert_parity(g, o, tol, floor=1e-20, what="gamma"):
    rel, small, n = floored_rel(g, o, floor)
    assert rel <= tol, f"{what}: max rel err {rel:.3e} > {tol:.1e} over {n} cells"
    assert small <= tol, f"{what}: below-floor abs err {small:.3e} (in floor units) > {tol:.1e}"
    zero = np.asarray(o) == 0
    assert np.all(np.asarray(g)[zero] == 0), f"{what}: non-zero where the oracle is exactly 0"


def assert_grad_parity(g, o, tol, floor=1e-6, what="grad"):
    """Gradient entries can be sums of large terms of both signs, so the
    relative error is taken against max(|o_i|, floor * max|o|)."""
    g = np.asarray(g, np.float64)
    o = np.asarray(o, np.float64)
    scale = np.maximum(np.abs(o), floor * np.abs(o).max())
    rel = float((np.abs(g - o) / scale).max())
    assert rel <= tol, f"{what}: max rel err {rel:.3e} > {tol:.1e}"
