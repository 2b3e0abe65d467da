"""GPU parity of the two-absorber sweep (asora_raytrace_helium: HI and HeI
columns, banded black-body spectrum) against the oracle's
(oracle.raytrace_helium), both rates at max relative error 1e-5 with the
floor of tests/parity.py; batched and plain; on a small lognormal grid with
whole-range radii (every source as layer pyramids) and on a subset of the
128^3 workload; and the refusals."""
import numpy as np
import pytest
import torch

import oracle
from tests.parity import assert_parity
from workloads import HE_ABUNDANCE, HE_BAND_EDGES_EV, HE_BAND_LG_HI, helium_cross_sections, make_workload

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module")
def asora():
    import paper_2311_01492_amd as m
    return m


@pytest.fixture(scope="module")
def bands():
    sH, sHe = helium_cross_sections()
    return [(oracle.blackbody_band_table(HE_BAND_EDGES_EV[b], HE_BAND_EDGES_EV[b + 1], lg_hi=HE_BAND_LG_HI[b]),
             sH[b], sHe[b]) for b in range(len(sH))]


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _ctx(asora, w, bands, **kw):
    bb = oracle.blackbody_table()
    ctx = asora.Asora(w.N, w.cell_cm, bb.P, bb.dP, bb.lg_lo, bb.lg_hi, **kw)
    ctx.set_helium([(t.P, t.dP, t.lg_lo, t.lg_hi, a, b) for t, a, b in bands])
    return ctx


def _fields(w):
    n_He = (HE_ABUNDANCE * w.n_H).astype(np.float32)
    return n_He, w.x_HI.copy()


def _check(asora, w, bands, **kw):
    n_He, x_He = _fields(w)
    ctx = _ctx(asora, w, bands)
    oH, oHe = oracle.raytrace_helium(w.N, w.cell_cm, bands, w.n_H, w.x_HI, n_He, x_He, w.src.ijk, w.src.Q,
                                     w.src.R)
    for plain in (False, True):
        gH, gHe = ctx.raytrace_helium(_t(w.n_H), _t(w.x_HI), _t(n_He), _t(x_He), _t(w.src.ijk), _t(w.src.Q),
                                      _t(w.src.R), plain=plain)
        ctx.check()
        assert_parity(gH.cpu().numpy(), oH, TOL, what=f"Gamma_HI (plain={plain})")
        assert_parity(gHe.cpu().numpy(), oHe, TOL, what=f"Gamma_HeI (plain={plain})")
    ctx.close()


def test_helium_small_grid_all_radii(asora, bands):
    print("case helium N=40, 20 sources R 0.5..19", flush=True)
    w = make_workload("c2", N=40, n_src=20, R=(0.5, 19.0))
    _check(asora, w, bands)


def test_helium_edges_odd_grid_wrap_and_clip(asora, bands):
    """Odd N, sources on faces and corners (periodic wrap), radii beyond half
    the box (extent clip), a duplicate source and R = 0."""
    print("case helium edges N=19", flush=True)
    w = make_workload("c2", N=19, n_src=6, R=(3.0, 17.0))
    w.src.ijk[:] = [[0, 0, 0], [18, 18, 18], [0, 9, 18], [5, 5, 5], [5, 5, 5], [12, 0, 7]]
    w.src.R[:] = [17.0, 9.5, 12.0, 4.0, 4.0, 0.0]
    _check(asora, w, bands)


@pytest.mark.parametrize("seed", range(8))
def test_helium_random_cases(asora, bands, seed):
    """Seeded random small cases: grid size (odd and even), source positions,
    radii up to beyond half the box, helium abundance and ionization drawn
    per cell (x_HeI independent of x_HI), batched and plain."""
    rng = np.random.default_rng(8000 + seed)
    N = int(rng.integers(9, 37))
    n_src = int(rng.integers(1, 7))
    w = make_workload("c2", N=N, n_src=n_src, R=(0.5, 1.0), seed=8100 + seed)
    w.src.ijk[:] = rng.integers(0, N, size=(n_src, 3)).astype(np.int32)
    w.src.R[:] = rng.uniform(0.0, 0.75 * N, size=n_src).astype(np.float32)
    n_He = (w.n_H * rng.uniform(0.05, 0.12, size=w.n_H.shape)).astype(np.float32)
    x_He = rng.uniform(1e-4, 1.0, size=w.x_HI.shape).astype(np.float32)
    print(f"case helium random seed={seed} N={N} n_src={n_src}", flush=True)
    ctx = _ctx(asora, w, bands)
    oH, oHe = oracle.raytrace_helium(w.N, w.cell_cm, bands, w.n_H, w.x_HI, n_He, x_He, w.src.ijk, w.src.Q,
                                     w.src.R)
    gH, gHe = ctx.raytrace_helium(_t(w.n_H), _t(w.x_HI), _t(n_He), _t(x_He), _t(w.src.ijk), _t(w.src.Q),
                                  _t(w.src.R), plain=bool(seed & 1))
    ctx.check()
    assert_parity(gH.cpu().numpy(), oH, TOL, what=f"Gamma_HI seed={seed}")
    assert_parity(gHe.cpu().numpy(), oHe, TOL, what=f"Gamma_HeI seed={seed}")
    ctx.close()


def test_helium_c2_subset(asora, bands):
    print("case helium 128^3 subset of 12 sources, R=30", flush=True)
    w = make_workload("c2")
    w.src = w.src.subset(np.arange(0, 1000, 84))
    _check(asora, w, bands)


def test_helium_refusals(asora, bands):
    print("case helium refusals", flush=True)
    w = make_workload("c2", N=16, n_src=2, R=(2.0, 5.0))
    bb = oracle.blackbody_table()
    ctx = asora.Asora(w.N, w.cell_cm, bb.P, bb.dP, bb.lg_lo, bb.lg_hi)
    n_He, x_He = _fields(w)
    args = (_t(w.n_H), _t(w.x_HI), _t(n_He), _t(x_He), _t(w.src.ijk), _t(w.src.Q), _t(w.src.R))
    with pytest.raises(asora.AsoraError, match="band tables"):
        ctx.raytrace_helium(*args)
    t, a, b = bands[0]
    with pytest.raises(asora.AsoraError, match="cross-sections"):
        ctx.set_helium([(t.P, t.dP, t.lg_lo, t.lg_hi, 0.0, 0.0)])
    ctx.set_helium([(t.P, t.dP, t.lg_lo, t.lg_hi, a, b) for t, a, b in bands])
    import ctypes
    lib = ctypes.CDLL(asora.lib_path())
    lib.asora_raytrace_helium.restype = ctypes.c_int32
    p = ctypes.c_void_p
    lib.asora_raytrace_helium.argtypes = [p, p, p, p, p, ctypes.c_int64, p, p, p, ctypes.c_float, p, p,
                                          ctypes.c_uint32, p]
    out = torch.zeros(w.N ** 3, dtype=torch.float32, device="cuda")
    ptrs = [x.data_ptr() for x in args]
    st = lib.asora_raytrace_helium(ctx._h, *ptrs[:4], 2, *ptrs[4:], 5.0, out.data_ptr(), out.data_ptr(),
                                   asora.STORE, None)
    assert st == -1
    ctx.close()
