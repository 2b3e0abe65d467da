"""Benchmark of the ASORA ray-tracing step on one MI355X.

A step is one asora_raytrace call over the whole source list of the
workload (n_HI and accumulator set-up, scheduling sort, persistent sweep,
FP32 conversion), inputs resident in HBM.  The metric is the paper's
time per source per voxel, t / sum_s (4/3) pi R_s^3 (Section 4.2), in ns.

Default workload: 128^3 grid, 1.4 Mpc cells, lognormal density with
ionized bubbles, 1000 sources, R = 30 cells (FP32 in, FP64 columns).
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ns per source-voxel (ASORA fwd, fwd+adjoint), batched vs plain, at 1e-5 rel err"
HBM_PEAK_GBS = 8000.0
ALG_BYTES_PER_SV = 16.0   # n_H + x_HI gather (2 x FP32) + rate read-modify-write (2 x FP32)
KERNEL_SOURCES = ["paper_2311_01492_amd/csrc/asora_dev.h", "paper_2311_01492_amd/csrc/asora_fwd.hip"]
PMC_FILE = os.path.join(ROOT, "profiles", "fwd_persistent_c2_pmc.json")

WORKLOADS = {
    "c2": dict(name="c2", kw={}, plain_src=1000,
               desc="128^3, cell 4.3e24 cm, lognormal n_H (ln sigma 0.5, P(k)~k^-2) x 1.5e-4, "
                    "x_HI 1e-3 in U[2,8]-cell bubbles, 1000 sources, Q 10^U[51,55], R=30"),
    "c3": dict(name="c3", kw={}, plain_src=1000,
               desc="250^3, cell 4.308e24 cm, lognormal + bubbles, 1e5 sources, Q 10^U[50,55], R U[5,50]"),
    "c5": dict(name="c5", kw={}, plain_src=1000,
               desc="250^3, cell 4.308e24 cm, lognormal, x_HI from smoothed threshold, 1e6 sources, "
                    "Q 10^U[50,54], R U[5,40]"),
}


def kernel_sha() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(open(os.path.join(ROOT, f), "rb").read())
    return h.hexdigest()[:16]


def cpu_baseline(w, budget_s: float = 12.0):
    """The FP64 oracle as it stands, single-threaded, on the first sources of
    the same workload until about budget_s of CPU time."""
    import numpy as np

    import oracle
    tb = oracle.blackbody_table()
    oracle.raytrace(w.N, w.cell_cm, tb, w.n_H, w.x_HI, w.src.ijk[:1], w.src.Q[:1], w.src.R[:1])
    done, work, t = 0, 0.0, 0.0
    chunk = 8
    while t < budget_s and done < len(w.src):
        sl = slice(done, min(done + chunk, len(w.src)))
        t0 = time.perf_counter()
        oracle.raytrace(w.N, w.cell_cm, tb, w.n_H, w.x_HI, w.src.ijk[sl], w.src.Q[sl], w.src.R[sl])
        t += time.perf_counter() - t0
        work += float(np.sum(4.0 / 3.0 * math.pi * w.src.R[sl].astype(np.float64) ** 3))
        done = sl.stop
    return {"value": t / work * 1e9, "unit": "ns per source-voxel", "cores": 1, "kind": "oracle",
            "sample": f"first {done} of {len(w.src)} sources of the same workload "
                      f"({t:.1f} s, one thread, FP64)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-plain", action="store_true", help="skip the one-launch-per-source form")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported "
              f"(sources would shard over GPUs with one all-reduce of Gamma, not built here)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration:
        n = 1 << 28
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read_per_launch": 4 * n, "copy_bytes_written_per_launch": 4 * n}))
        return

    import paper_2311_01492_amd as asora
    from workloads import make_workload

    spec = WORKLOADS[args.workload]
    print(f"[bench] building workload {args.workload}", file=sys.stderr, flush=True)
    w = make_workload(spec["name"], **spec["kw"])
    P, dP = asora.table_blackbody(5e4, 2.8, 2000, -20.0, 4.0)
    ctx = asora.Asora(w.N, w.cell_cm, P, dP, -20.0, 4.0, tau_w=0.6)
    dev = torch.device("cuda", 0)
    nH = torch.from_numpy(w.n_H).to(dev)
    xH = torch.from_numpy(w.x_HI).to(dev)
    ijk = torch.from_numpy(w.src.ijk).to(dev)
    Q = torch.from_numpy(w.src.Q).to(dev)
    R = torch.from_numpy(w.src.R).to(dev)
    R_max = float(w.src.R.max())
    work = w.work_sphere
    gamma = torch.empty(w.N ** 3, dtype=torch.float32, device=dev)

    def step(plain=False, n=None, profile=False):
        s = slice(0, n)
        ctx.raytrace(nH, xH, ijk[s], Q[s], R[s], R_max=R_max, out=gamma, plain=plain, profile=profile)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    print(f"[bench] warmup done, timing {args.steps} steps", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) / args.steps * 1e3
    ctx.check()
    ns_sv = ms * 1e6 / work

    # the dominant kernel (the persistent sweep), timed with HIP events on the
    # stream it runs on, over the same number of steps
    sweep = []
    for _ in range(args.steps):
        step(profile=True)
        sweep.append(ctx.profile()[0])
    sweep_ms = float(np.mean(sweep))
    achieved = ALG_BYTES_PER_SV * work / (sweep_ms * 1e-3) / 1e9

    traffic = None
    if os.path.exists(PMC_FILE):
        pmc = json.load(open(PMC_FILE))
        if pmc.get("kernel_sha") == kernel_sha() and pmc.get("workload") == args.workload:
            traffic = pmc.get("hbm_bytes_per_launch")

    out = {
        "metric": METRIC, "value": ns_sv, "unit": "ns per source-voxel", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64/f32", "data": "synthetic",
        "config": {"workload": f"{args.workload}: {spec['desc']}", "grid": w.N,
                   "n_sources": len(w.src), "source_voxels": work, "seed": w.seed,
                   "mode": "batched persistent"},
        "sweep_ms": sweep_ms,
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "kernel": "fwd_persistent", "alg_bytes_per_source_voxel": ALG_BYTES_PER_SV},
    }

    if not args.no_plain:
        n = min(spec["plain_src"], len(w.src))
        sub_work = float(np.sum(4.0 / 3.0 * math.pi * w.src.R[:n].astype(np.float64) ** 3))
        step(plain=True, n=n)
        torch.cuda.synchronize()
        reps = 2
        t0 = time.perf_counter()
        for _ in range(reps):
            step(plain=True, n=n)
        torch.cuda.synchronize()
        pms = (time.perf_counter() - t0) / reps * 1e3
        out["plain"] = {"ns_per_source_voxel": pms * 1e6 / sub_work, "sources": n,
                        "ms_per_call": pms, "plain_over_batched": (pms * 1e6 / sub_work) / ns_sv}
    out["paper_context"] = {"value": 3.156, "unit": "ns per source-voxel",
                            "hardware": "1x NVIDIA Tesla P100, FP64 grid data",
                            "workload": "250^3, R in {10,30,50,100}, up to 1e6 sources (asymptote)"}
    if not args.no_cpu:
        print("[bench] CPU oracle baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
