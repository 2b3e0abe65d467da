"""GPU adjoint (asora_raytrace_backward) against the FP64 oracle's reverse
mode and against central finite differences of the oracle forward, for the
loss L = sum_p w_p log10(Gamma_p + 1e-20) with w ~ N(0,1) per cell."""
import math

import numpy as np
import pytest
import torch

import oracle
from tests.parity import assert_grad_parity
from workloads import make_workload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def asora():
    import paper_2311_01492_amd as m
    return m


@pytest.fixture(scope="module")
def bb():
    return oracle.blackbody_table()


def _loss_grad(g, wt):
    return wt / ((g + 1e-20) * math.log(10))


# large sources as layer pyramids, their adjoint's rate terms split between
# the gathering and the reverse pass (the default) or all gathered; or as
# shell pyramids
SWEEPS = [(3, 2), (3, 1), (2, 0)]
SWEEP_IDS = ["layers", "layers-gathered", "shells"]


def _gpu_backward(asora, w, table, gbar, sweep=(3, 2), **kw):
    ctx = asora.Asora(w.N, w.cell_cm, table.P, table.dP, table.lg_lo, table.lg_hi, **kw)
    ctx.set_tuning(pyramid_sweep=sweep[0], adj_rate=sweep[1])
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    dn, dx, dq = ctx.backward(t(w.n_H), t(w.x_HI), t(w.src.ijk), t(w.src.Q), t(w.src.R), t(gbar))
    ctx.check()
    return (dn.cpu().numpy().astype(np.float64), dx.cpu().numpy().astype(np.float64),
            dq.cpu().numpy())


def _case(name, **kw):
    w = make_workload(name, **kw)
    bb = oracle.blackbody_table()
    g = oracle.raytrace(w.N, w.cell_cm, bb, w.n_H, w.x_HI, w.src.ijk, w.src.Q, w.src.R)
    wt = np.random.default_rng(4).standard_normal(g.shape)
    return w, g, wt


@pytest.mark.parametrize("sweep", SWEEPS, ids=SWEEP_IDS)
def test_c4_against_oracle_reverse(asora, bb, sweep):
    print("case c4 adjoint vs oracle sweep", sweep, flush=True)
    w, g, wt = _case("c4")
    gbar = _loss_grad(g, wt)
    on, ox, oq = oracle.raytrace_grad(w.N, w.cell_cm, bb, w.n_H, w.x_HI, w.src.ijk, w.src.Q,
                                      w.src.R, gbar)
    gn, gx, gq = _gpu_backward(asora, w, bb, gbar, sweep=sweep)
    assert_grad_parity(gn, on, 1e-5, what="dL/dn_H")
    assert_grad_parity(gx, ox, 1e-5, what="dL/dx_HI")
    np.testing.assert_allclose(gq, oq, rtol=1e-5)


@pytest.mark.parametrize("sweep", SWEEPS, ids=SWEEP_IDS)
@pytest.mark.parametrize("tau_w,scalar", [(math.inf, False), (0.6, True)])
def test_uneven_radii_all_piece_kinds(asora, bb, tau_w, scalar, sweep):
    print("case adjoint uneven", tau_w, scalar, "sweep", sweep, flush=True)
    w, g, wt = _case("c2", N=40, n_src=24, R=(2.0, 38.0))
    g = oracle.raytrace(w.N, w.cell_cm, bb, w.n_H, w.x_HI, w.src.ijk, w.src.Q, w.src.R,
                        tau_w=tau_w, reading=1 if scalar else 0)
    gbar = _loss_grad(g, wt)
    on, ox, oq = oracle.raytrace_grad(w.N, w.cell_cm, bb, w.n_H, w.x_HI, w.src.ijk, w.src.Q,
                                      w.src.R, gbar, tau_w=tau_w, reading=1 if scalar else 0)
    gn, gx, gq = _gpu_backward(asora, w, bb, gbar, sweep=sweep, tau_w=tau_w, halfpath_scalar=scalar)
    assert_grad_parity(gn, on, 1e-5, what="dL/dn_H")
    assert_grad_parity(gx, ox, 1e-5, what="dL/dx_HI")
    np.testing.assert_allclose(gq, oq, rtol=1e-5)


@pytest.mark.parametrize("sweep", SWEEPS, ids=SWEEP_IDS)
def test_edges_odd_grid_wrap_clip_and_empty(asora, bb, sweep):
    """The adjoint on the forward's edge cases: odd N with sources on faces and
    corners (periodic wrap), radii beyond half the box (extent clip), a
    duplicate source and R = 0; an even grid with a radius beyond the box;
    and an empty source list (all gradients zero)."""
    print("case adjoint edges sweep", sweep, flush=True)
    for N, ijk, R in ((19, [[0, 0, 0], [18, 18, 18], [0, 9, 18], [5, 5, 5], [5, 5, 5], [12, 0, 7]],
                       [17.0, 9.5, 12.0, 4.0, 4.0, 0.0]),
                      (20, [[19, 0, 19], [3, 12, 8], [10, 10, 10]], [26.0, 12.0, 30.0])):
        w, _, wt = _case("c2", N=N, n_src=len(R), R=(1.0, 2.0))
        w.src.ijk[:] = ijk
        w.src.R[:] = R
        g = oracle.raytrace(w.N, w.cell_cm, bb, w.n_H, w.x_HI, w.src.ijk, w.src.Q, w.src.R)
        gbar = _loss_grad(g, wt)
        on, ox, oq = oracle.raytrace_grad(w.N, w.cell_cm, bb, w.n_H, w.x_HI, w.src.ijk, w.src.Q,
                                          w.src.R, gbar)
        gn, gx, gq = _gpu_backward(asora, w, bb, gbar, sweep=sweep)
        assert_grad_parity(gn, on, 1e-5, what=f"dL/dn_H N={N}")
        assert_grad_parity(gx, ox, 1e-5, what=f"dL/dx_HI N={N}")
        np.testing.assert_allclose(gq, oq, rtol=1e-5)
    ctx = asora.Asora(w.N, w.cell_cm, bb.P, bb.dP, bb.lg_lo, bb.lg_hi)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    dn, dx, dq = ctx.backward(t(w.n_H), t(w.x_HI), torch.empty(0, 3, dtype=torch.int32, device="cuda"),
                              torch.empty(0, dtype=torch.float64, device="cuda"),
                              torch.empty(0, dtype=torch.float32, device="cuda"), t(gbar), R_max=0.0)
    ctx.check()
    assert float(dn.abs().max()) == 0.0 and float(dx.abs().max()) == 0.0 and dq.numel() == 0


def _covering(w, c):
    d = (np.asarray(c)[None, :] - w.src.ijk + w.N // 2) % w.N - w.N // 2
    return np.nonzero((d ** 2).sum(axis=1) <= w.src.R.astype(np.float64) ** 2)[0]


def test_c4_against_finite_differences(asora, bb):
    """Central differences (step 1e-4 relative) of the FP64 oracle forward on
    100 seeded entries: 40 of n_H, 40 of x_HI, 20 of Q.  Only the sources whose
    ball holds the perturbed cell are re-run (the others do not change)."""
    print("case c4 adjoint vs FD", flush=True)
    w, g, wt = _case("c4")
    gbar = _loss_grad(g, wt)
    gn, gx, gq = _gpu_backward(asora, w, bb, gbar)
    rng = np.random.default_rng(9)
    nH = w.n_H.astype(np.float64)
    xH = w.x_HI.astype(np.float64)
    dl = lambda gp, gm: float(np.sum(wt * (np.log10(gp + 1e-20) - np.log10(gm + 1e-20))))
    cells = np.argwhere(g > 1e-6 * g.max())
    errs = []
    for field, grad, name in ((nH, gn, "n_H"), (xH, gx, "x_HI")):
        for c in map(tuple, cells[rng.choice(len(cells), 40, replace=False)]):
            S = _covering(w, c)
            sub = w.src.subset(S)
            base = oracle.raytrace(w.N, w.cell_cm, bb, nH, xH, sub.ijk, sub.Q, sub.R)
            h = 1e-4 * field[c]
            fp, fm = field.copy(), field.copy()
            fp[c] += h
            fm[c] -= h
            args = (lambda f: (f, xH)) if field is nH else (lambda f: (nH, f))
            gp = g - base + oracle.raytrace(w.N, w.cell_cm, bb, *args(fp), sub.ijk, sub.Q, sub.R)
            gm = g - base + oracle.raytrace(w.N, w.cell_cm, bb, *args(fm), sub.ijk, sub.Q, sub.R)
            fd = dl(gp, gm) / (2 * h)
            scale = max(abs(fd), 1e-6 * np.abs(grad).max())
            errs.append(abs(grad[c] - fd) / scale)
            assert abs(grad[c] - fd) <= 1e-4 * scale, (name, c, grad[c], fd)
    for s in rng.choice(len(w.src), 20, replace=False):
        sub = w.src.subset([s])
        base = oracle.raytrace(w.N, w.cell_cm, bb, nH, xH, sub.ijk, sub.Q, sub.R)
        h = 1e-4 * w.src.Q[s]
        gp = g - base + oracle.raytrace(w.N, w.cell_cm, bb, nH, xH, sub.ijk, sub.Q + h, sub.R)
        gm = g - base + oracle.raytrace(w.N, w.cell_cm, bb, nH, xH, sub.ijk, sub.Q - h, sub.R)
        fd = dl(gp, gm) / (2 * h)
        errs.append(abs(gq[s] - fd) / abs(fd))
        assert gq[s] == pytest.approx(fd, rel=1e-4)
    print("max rel err vs FD", max(errs), flush=True)


def test_autograd_function(asora, bb):
    """torch.autograd through asora.raytrace gives the adjoint kernels' gradients."""
    w = make_workload("c2", N=32, n_src=10, R=(3.0, 14.0))
    ctx = asora.Asora(w.N, w.cell_cm, bb.P, bb.dP, bb.lg_lo, bb.lg_hi)
    dev = torch.device("cuda")
    nH = torch.from_numpy(w.n_H).to(dev).requires_grad_(True)
    xH = torch.from_numpy(w.x_HI).to(dev).requires_grad_(True)
    Q = torch.from_numpy(w.src.Q).to(dev).requires_grad_(True)
    ijk = torch.from_numpy(w.src.ijk).to(dev)
    R = torch.from_numpy(w.src.R).to(dev)
    wt = torch.from_numpy(np.random.default_rng(2).standard_normal((w.N,) * 3)).to(dev)
    gam = asora.raytrace(ctx, nH, xH, ijk, Q, R)
    loss = (wt * torch.log10(gam.double() + 1e-20)).sum()
    loss.backward()
    gbar = (wt / ((gam.detach().double() + 1e-20) * math.log(10)))
    dn, dx, dq = ctx.backward(nH.detach(), xH.detach(), ijk, Q.detach(), R, gbar)
    torch.testing.assert_close(nH.grad, dn, rtol=1e-5, atol=1e-6 * float(dn.abs().max()))
    torch.testing.assert_close(xH.grad, dx, rtol=1e-5, atol=1e-6 * float(dx.abs().max()))
    torch.testing.assert_close(Q.grad, dq, rtol=1e-6, atol=0)
    # the same through the recomputing backward
    for t_ in (nH, xH, Q):
        t_.grad = None
    gam = asora.raytrace(ctx, nH, xH, ijk, Q, R, store=False)
    (wt * torch.log10(gam.double() + 1e-20)).sum().backward()
    torch.testing.assert_close(nH.grad, dn, rtol=1e-5, atol=1e-6 * float(dn.abs().max()))
    torch.testing.assert_close(Q.grad, dq, rtol=1e-6, atol=0)


@pytest.mark.parametrize("adj_rate", [2, 1], ids=["split", "gathered"])
def test_kept_records_match_recompute_and_oracle(asora, bb, adj_rate):
    """Forward with ASORA_STORE keeps the pyramids' column records; the
    backward that reads them gives the recomputing backward's gradients and
    the oracle's.  Uneven radii cover whole-source and octant pieces (always
    recomputed) next to the pyramids."""
    print("case kept records c4 adj_rate", adj_rate, flush=True)
    w, g, wt = _case("c4")
    gbar = _loss_grad(g, wt)
    on, ox, oq = oracle.raytrace_grad(w.N, w.cell_cm, bb, w.n_H, w.x_HI, w.src.ijk, w.src.Q,
                                      w.src.R, gbar)
    ctx = asora.Asora(w.N, w.cell_cm, bb.P, bb.dP, bb.lg_lo, bb.lg_hi)
    ctx.set_tuning(adj_rate=adj_rate)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    nH, xH, ijk, Q, R, gb = t(w.n_H), t(w.x_HI), t(w.src.ijk), t(w.src.Q), t(w.src.R), t(gbar)
    ctx.raytrace(nH, xH, ijk, Q, R, store=True)
    kept, need, alloc = ctx.store_info()
    assert kept and 0 < need <= alloc
    ks = ctx.backward(nH, xH, ijk, Q, R, gb, store=True)
    rc = ctx.backward(nH, xH, ijk, Q, R, gb)
    ctx.check()
    for a, b, o, name in zip(ks, rc, (on, ox, oq), ("dL/dn_H", "dL/dx_HI", "dL/dQ")):
        a, b = a.cpu().numpy(), b.cpu().numpy()
        np.testing.assert_allclose(a, b, rtol=1e-9, atol=1e-12 * np.abs(b).max(), err_msg=name)
        if name == "dL/dQ":
            np.testing.assert_allclose(a, o, rtol=1e-5)
        else:
            assert_grad_parity(a, o, 1e-5, what=name)
    # uneven radii: whole-source, octant and pyramid pieces in one call
    print("case kept records uneven", flush=True)
    w, g, wt = _case("c2", N=40, n_src=24, R=(2.0, 38.0))
    gbar = _loss_grad(g, wt)
    on, ox, oq = oracle.raytrace_grad(w.N, w.cell_cm, bb, w.n_H, w.x_HI, w.src.ijk, w.src.Q,
                                      w.src.R, gbar)
    ctx = asora.Asora(w.N, w.cell_cm, bb.P, bb.dP, bb.lg_lo, bb.lg_hi)
    ctx.set_tuning(adj_rate=adj_rate, adj_waves=12 if adj_rate == 1 else 2)
    nH, xH, ijk, Q, R, gb = t(w.n_H), t(w.x_HI), t(w.src.ijk), t(w.src.Q), t(w.src.R), t(gbar)
    ctx.raytrace(nH, xH, ijk, Q, R, store=True)
    assert ctx.store_info()[0]
    gn, gx, gq = (a.cpu().numpy() for a in ctx.backward(nH, xH, ijk, Q, R, gb, store=True))
    ctx.check()
    assert_grad_parity(gn, on, 1e-5, what="dL/dn_H")
    assert_grad_parity(gx, ox, 1e-5, what="dL/dx_HI")
    np.testing.assert_allclose(gq, oq, rtol=1e-5)


@pytest.mark.parametrize("adj_rate", [1, 2])
def test_wide_work_groups(asora, bb, adj_rate):
    """The layer adjoint's 16-wave build (held to four waves per SIMD) in all
    three forms: recomputed columns with gathered or split rate terms, and
    kept records; uneven radii, so every piece kind runs."""
    print(f"case wide adjoint adj_rate={adj_rate}", flush=True)
    w, g, wt = _case("c2", N=40, n_src=24, R=(2.0, 38.0))
    gbar = _loss_grad(g, wt)
    on, ox, oq = oracle.raytrace_grad(w.N, w.cell_cm, bb, w.n_H, w.x_HI, w.src.ijk, w.src.Q,
                                      w.src.R, gbar)
    ctx = asora.Asora(w.N, w.cell_cm, bb.P, bb.dP, bb.lg_lo, bb.lg_hi)
    ctx.set_tuning(adj_rate=adj_rate, adj_waves=16)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    nH, xH, ijk, Q, R, gb = t(w.n_H), t(w.x_HI), t(w.src.ijk), t(w.src.Q), t(w.src.R), t(gbar)
    for store in (False, True):
        if store:
            ctx.raytrace(nH, xH, ijk, Q, R, store=True)
            assert ctx.store_info()[0]
        gn, gx, gq = (a.cpu().numpy() for a in ctx.backward(nH, xH, ijk, Q, R, gb, store=store))
        ctx.check()
        assert_grad_parity(gn, on, 1e-5, what=f"dL/dn_H (store={store})")
        assert_grad_parity(gx, ox, 1e-5, what=f"dL/dx_HI (store={store})")
        np.testing.assert_allclose(gq, oq, rtol=1e-5)
    ctx.close()


def test_kept_records_fall_back_to_recompute(asora, bb):
    """Records that do not fit the budget are not kept; records kept for other
    input buffers are not used: both backwards recompute."""
    print("case kept records fallback", flush=True)
    w, g, wt = _case("c2", N=32, n_src=6, R=(16.0, 20.0))
    gbar = _loss_grad(g, wt)
    ctx = asora.Asora(w.N, w.cell_cm, bb.P, bb.dP, bb.lg_lo, bb.lg_hi)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    nH, xH, ijk, Q, R, gb = t(w.n_H), t(w.x_HI), t(w.src.ijk), t(w.src.Q), t(w.src.R), t(gbar)
    on, ox, oq = oracle.raytrace_grad(w.N, w.cell_cm, bb, w.n_H, w.x_HI, w.src.ijk, w.src.Q,
                                      w.src.R, gbar)
    ctx.set_store_budget(1024)
    ctx.raytrace(nH, xH, ijk, Q, R, store=True)
    kept, need, _ = ctx.store_info()
    assert not kept and need > 1024
    gn, gx, gq = (a.cpu().numpy() for a in ctx.backward(nH, xH, ijk, Q, R, gb, store=True))
    assert_grad_parity(gn, on, 1e-5, what="dL/dn_H")
    np.testing.assert_allclose(gq, oq, rtol=1e-5)
    # records kept for a fully neutral x_HI; the backward is asked about the real one
    ctx.set_store_budget(0)
    x_other = torch.ones_like(xH)
    ctx.raytrace(nH, x_other, ijk, Q, R, store=True)
    assert ctx.store_info()[0]
    gn, gx, gq = (a.cpu().numpy() for a in ctx.backward(nH, xH, ijk, Q, R, gb, store=True))
    ctx.check()
    assert_grad_parity(gn, on, 1e-5, what="dL/dn_H")
    assert_grad_parity(gx, ox, 1e-5, what="dL/dx_HI")
    np.testing.assert_allclose(gq, oq, rtol=1e-5)


def test_kept_records_of_an_early_exit_forward(asora, bb):
    """A forward with ASORA_EARLY_EXIT and ASORA_STORE keeps records up to each
    pyramid's first opaque layer; the early-exit backward that reads them, the
    early-exit backward that recomputes and the full backward (every layer)
    give the same gradients, and the oracle's.  A backward without the flag
    does not read those records (it recomputes every layer)."""
    print("case kept records early exit", flush=True)
    w, g, wt = _case("c2", N=48, n_src=24, R=(10.0, 22.0))
    gbar = _loss_grad(g, wt)
    on, ox, oq = oracle.raytrace_grad(w.N, w.cell_cm, bb, w.n_H, w.x_HI, w.src.ijk, w.src.Q,
                                      w.src.R, gbar)
    ctx = asora.Asora(w.N, w.cell_cm, bb.P, bb.dP, bb.lg_lo, bb.lg_hi)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    nH, xH, ijk, Q, R, gb = t(w.n_H), t(w.x_HI), t(w.src.ijk), t(w.src.Q), t(w.src.R), t(gbar)
    ctx.raytrace(nH, xH, ijk, Q, R, store=True, early_exit=True)
    assert ctx.store_info()[0]
    ks = ctx.backward(nH, xH, ijk, Q, R, gb, store=True, early_exit=True)
    re = ctx.backward(nH, xH, ijk, Q, R, gb, early_exit=True)
    rc = ctx.backward(nH, xH, ijk, Q, R, gb)
    rs = ctx.backward(nH, xH, ijk, Q, R, gb, store=True)   # flags differ: recomputes
    ctx.check()
    for a, b, c, d, o, name in zip(ks, re, rc, rs, (on, ox, oq), ("dL/dn_H", "dL/dx_HI", "dL/dQ")):
        a, b, c, d = a.cpu().numpy(), b.cpu().numpy(), c.cpu().numpy(), d.cpu().numpy()
        for x in (b, c, d):
            np.testing.assert_allclose(a, x, rtol=1e-9, atol=1e-12 * np.abs(x).max(), err_msg=name)
        if name == "dL/dQ":
            np.testing.assert_allclose(a, o, rtol=1e-5)
        else:
            assert_grad_parity(a, o, 1e-5, what=name)
