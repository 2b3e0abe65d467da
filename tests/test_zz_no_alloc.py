"""The allocation-free forward (asora_raytrace_static, its scratch in the
library's fixed device array) against asora_raytrace and the oracle, through
the C ABI: two calls in a row on one context, the second with a smaller input
(fewer sources, smaller radii), then a smaller grid on a second context (both
contexts use the device's one array), the plain and early-exit forms, and
the refusal of sizes beyond the array."""
import ctypes

import numpy as np
import pytest
import torch

import oracle
from tests.parity import assert_parity
from workloads import make_workload

pytestmark = pytest.mark.gpu
TOL = 1e-5


@pytest.fixture(scope="module")
def asora():
    import paper_2311_01492_amd as m
    return m


@pytest.fixture(scope="module")
def bb():
    return oracle.blackbody_table()


def _t(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _both(ctx, w, src, **kw):
    nH, xH, ijk, Q, R = _t(w.n_H), _t(w.x_HI), _t(src.ijk), _t(src.Q), _t(src.R)
    out = torch.full((w.N ** 3,), float("nan"), dtype=torch.float32, device="cuda")
    gs = ctx.raytrace_static(nH, xH, ijk, Q, R, out=out, **kw)
    gr = ctx.raytrace(nH, xH, ijk, Q, R, **kw)
    ctx.check()
    return gs.cpu().numpy().astype(np.float64), gr.cpu().numpy().astype(np.float64)


def test_static_forward_two_calls_then_smaller_grid(asora, bb):
    print("case static forward, N=64 then fewer sources, then N=40", flush=True)
    w = make_workload("c2", N=64, n_src=40, R=(3.0, 30.0))
    ctx = asora.Asora(w.N, w.cell_cm, bb.P, bb.dP, bb.lg_lo, bb.lg_hi)
    # whole sources, octants and layer pyramids in one call
    gs, gr = _both(ctx, w, w.src)
    o = oracle.raytrace(w.N, w.cell_cm, bb, w.n_H, w.x_HI, w.src.ijk, w.src.Q, w.src.R)
    assert_parity(gs, o, TOL, what="static, call 1")
    assert_parity(gs, gr, TOL, what="static vs raytrace, call 1")
    # the second call, smaller: whatever the first left in the array is cleared
    sub = w.src.subset(np.arange(8))
    sub.R[:] = np.minimum(sub.R, 14.0)
    gs, gr = _both(ctx, w, sub)
    o = oracle.raytrace(w.N, w.cell_cm, bb, w.n_H, w.x_HI, sub.ijk, sub.Q, sub.R)
    assert_parity(gs, o, TOL, what="static, call 2")
    assert_parity(gs, gr, TOL, what="static vs raytrace, call 2")
    for kw in (dict(plain=True), dict(early_exit=True)):
        gs, gr = _both(ctx, w, w.src, **kw)
        assert_parity(gs, gr, TOL, what=f"static vs raytrace {kw}")
    ctx.close()
    # a smaller grid on another context, the same array
    w2 = make_workload("c2", N=40, n_src=12, R=(4.0, 19.0))
    ctx2 = asora.Asora(w2.N, w2.cell_cm, bb.P, bb.dP, bb.lg_lo, bb.lg_hi)
    gs, gr = _both(ctx2, w2, w2.src)
    o = oracle.raytrace(w2.N, w2.cell_cm, bb, w2.n_H, w2.x_HI, w2.src.ijk, w2.src.Q, w2.src.R)
    assert_parity(gs, o, TOL, what="static, N=40")
    assert_parity(gs, gr, TOL, what="static vs raytrace, N=40")
    ctx2.close()


def test_static_forward_refuses_sizes_beyond_the_array(asora, bb):
    print("case static forward limits", flush=True)
    w = make_workload("c2", N=66, n_src=2, R=(3.0, 5.0))
    ctx = asora.Asora(w.N, w.cell_cm, bb.P, bb.dP, bb.lg_lo, bb.lg_hi)
    nH, xH = _t(w.n_H), _t(w.x_HI)
    out = torch.zeros(w.N ** 3, dtype=torch.float32, device="cuda")
    with pytest.raises(asora.AsoraError, match="N=66"):
        ctx.raytrace_static(nH, xH, _t(w.src.ijk), _t(w.src.Q), _t(w.src.R), out=out)
    ctx.close()
    w = make_workload("c2", N=16, n_src=2, R=(3.0, 5.0))
    ctx = asora.Asora(w.N, w.cell_cm, bb.P, bb.dP, bb.lg_lo, bb.lg_hi)
    n = (1 << 16) + 1
    ijk = torch.zeros((n, 3), dtype=torch.int32, device="cuda")
    Q = torch.ones(n, dtype=torch.float64, device="cuda")
    R = torch.ones(n, dtype=torch.float32, device="cuda")
    out = torch.zeros(w.N ** 3, dtype=torch.float32, device="cuda")
    with pytest.raises(asora.AsoraError, match="n_src=65537"):
        ctx.raytrace_static(_t(w.n_H), _t(w.x_HI), ijk, Q, R, out=out)
    # ASORA_STORE (kept records need memory) is refused before anything is enqueued
    lib = ctypes.CDLL(asora.lib_path())
    lib.asora_raytrace_static.restype = ctypes.c_int32
    p = ctypes.c_void_p
    lib.asora_raytrace_static.argtypes = [p, p, p, ctypes.c_int64, p, p, p, ctypes.c_float, p, p,
                                          ctypes.c_uint32, p]
    lib.asora_last_error.restype = ctypes.c_char_p
    lib.asora_last_error.argtypes = [p]
    st = lib.asora_raytrace_static(ctx._h, _t(w.n_H).data_ptr(), _t(w.x_HI).data_ptr(), 2, ijk.data_ptr(),
                                   Q.data_ptr(), R.data_ptr(), 1.0, out.data_ptr(), None, asora.STORE, None)
    assert st == -1 and b"flags" in lib.asora_last_error(ctx._h)
    ctx.close()
