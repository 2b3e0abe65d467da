"""Full-size checks in the benchmark's launch configuration: every source of
the 128^3 workload (1000 sources, R = 30), the 250^3 one (1e5 sources) and the
million-source one in one forward and one adjoint call, with the scheduling
the autotuner picks on them.

dL/dQ_s depends only on source s and on dL/dGamma (Gamma is a sum over
sources, each linear in its Q), so sampled sources of the full call are
checked one by one against the oracle's reverse mode run on those sources
alone.  Over all sources the linear-response identity
sum_s Q_s dL/dQ_s = sum_p dL/dGamma_p Gamma_p ties the adjoint to the
forward.  On the 128^3 workload, whose column records fit in memory, the
adjoint that reads them is also checked against the one that recomputes."""
import numpy as np
import pytest
import torch

import oracle
from tests.parity import assert_grad_parity
from workloads import make_workload

pytestmark = pytest.mark.gpu

# what the autotuner chose on these workloads in benchmark runs
TUNING = {
    "c2": dict(R_whole=6.0, R_oct=15.0, max_waves=16, pyramid_sweep=3, table_place=1, adj_waves=4,
               adj_rate=1),
    "c3": dict(R_whole=6.0, R_oct=10.0, max_waves=16, pyramid_sweep=3, table_place=2, adj_waves=4,
               adj_rate=2),
    "c5": dict(R_whole=8.0, R_oct=8.0, max_waves=16, pyramid_sweep=3, table_place=2, adj_waves=4,
               adj_rate=1),
}


@pytest.fixture(scope="module")
def asora():
    import paper_2311_01492_amd as m
    return m


@pytest.fixture(scope="module")
def bb():
    return oracle.blackbody_table()


@pytest.mark.parametrize("name", ["c2", "c3", "c5"])
def test_full_workload_adjoint(asora, bb, name):
    w = make_workload(name)
    print("case full workload", name, len(w.src), "sources", flush=True)
    ctx = asora.Asora(w.N, w.cell_cm, bb.P, bb.dP, bb.lg_lo, bb.lg_hi)
    ctx.set_tuning(**TUNING[name])
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    nH, xH, ijk, Q, R = t(w.n_H), t(w.x_HI), t(w.src.ijk), t(w.src.Q), t(w.src.R)
    rng = np.random.default_rng(17)
    gbar = rng.uniform(0.0, 1.0, w.N ** 3)
    gamma = ctx.raytrace(nH, xH, ijk, Q, R, store=True)
    kept = ctx.store_info()[0]
    assert kept == (name == "c2")   # the records of the 250^3 workloads need terabytes
    dn, dx, dq = ctx.backward(nH, xH, ijk, Q, R, t(gbar), store=kept)
    ctx.check()
    g = gamma.cpu().numpy().astype(np.float64).ravel()
    dq = dq.cpu().numpy()
    # linear response: Gamma from the FP32 forward, dL/dQ from the FP64 adjoint
    lhs, rhs = float(np.dot(w.src.Q, dq)), float(np.dot(gbar, g))
    assert lhs == pytest.approx(rhs, rel=1e-5), (lhs, rhs)
    if kept:
        rc = [a.cpu().numpy() for a in ctx.backward(nH, xH, ijk, Q, R, t(gbar), store=False)]
        ctx.check()
        for a, b, what in zip((dn.cpu().numpy(), dx.cpu().numpy(), dq), rc, ("dL/dn_H", "dL/dx_HI", "dL/dQ")):
            np.testing.assert_allclose(a, b, rtol=1e-9, atol=1e-12 * np.abs(b).max(), err_msg=what)
    # sampled sources (radius <= 30 to bound the oracle's time) against the oracle
    cand = np.nonzero(w.src.R <= 30.0)[0]
    idx = np.sort(rng.choice(cand, size=4, replace=False))
    sub = w.src.subset(idx)
    _, _, oq = oracle.raytrace_grad(w.N, w.cell_cm, bb, w.n_H, w.x_HI, sub.ijk, sub.Q, sub.R, gbar)
    np.testing.assert_allclose(dq[idx], oq, rtol=1e-5)
    assert np.all(oq > 0)
