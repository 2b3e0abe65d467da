"""Benchmark of the ASORA ray-tracing step (forward and adjoint) on one MI355X.

A step is one pass of the whole hot path over the workload's source list:
the forward sweep (asora_raytrace: n_HI and accumulator set-up, scheduling
sort, persistent sweep over all source pieces, FP32 conversion of Gamma)
followed by the adjoint (asora_raytrace_backward: the same set-up, the
columns from the records the forward kept when they fit in memory, else
recomputed per piece, reverse sweep, dL/dn_H and dL/dx_HI conversion) for a
fixed dL/dGamma, all inputs resident in HBM.  The metric
is the paper's time per source per voxel, t / sum_s (4/3) pi R_s^3
(Section 4.2), in ns: `value` is the forward+adjoint step; the batched
forward alone and the plain form (one launch per source) are reported beside
it.

Default workload: 128^3 grid, 1.4 Mpc cells, lognormal density with ionized
bubbles, 1000 sources, R = 30 cells.  Prints one JSON line.

`--reduce-pmc DIR` turns rocprofv3 counter runs (CSV output) of this script
into the per-launch HBM traffic file read here, and `--reduce-sq DIR` the SQ
instruction counters into the VALU-issue file (the commands that made them
head the summaries under profiles/).
"""
from __future__ import annotations

import argparse
import csv
import glob
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
# VALU issue: each SIMD issues one wave64 instruction per 4 cycles (16 lanes);
# 256 CUs x 4 SIMDs at 2.4 GHz
VALU_PEAK_PER_S = 256 * 4 * 2.4e9 / 4
# algorithmic HBM bytes per source-voxel
FWD_BYTES_PER_SV = 16.0   # n_H + x_HI reads (2 x FP32), Gamma read-modify-write (2 x FP32)
ADJ_BYTES_PER_SV = 32.0   # n_H + x_HI (2 x FP32), dL/dGamma (FP64), dL/dn_HI read-modify-write (2 x FP64)
KEEP_FWD_BYTES_PER_SV = FWD_BYTES_PER_SV + 8.0   # and the kept entry column of every cell (FP64)
KERNEL_SOURCES = ["paper_2311_01492_amd/csrc/asora_dev.h", "paper_2311_01492_amd/csrc/asora_fwd.hip",
                  "paper_2311_01492_amd/csrc/asora_adj.hip"]
# sweep kernels of each pass (one dispatch per piece kind up to the largest
# radius; the kinds without sources return at once)
KERNELS = {"fwd": ("fwd_wave", "fwd_layer"), "adj": ("adj_wave", "adj_layer")}

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


def pmc_file(workload: str) -> str:
    return os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.json")


def valu_file(workload: str) -> str:
    return os.path.join(ROOT, "profiles", f"valu_issue_{workload}.json")


# ---------------------------------------------------------------------------
def _read_counter_csv(path):
    """{kernel name: {counter: [value per dispatch]}} from a rocprofv3
    counter_collection.csv."""
    out = {}
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            name = row.get("Kernel_Name", "")
            ctr = row.get("Counter_Name", "")
            val = float(row.get("Counter_Value", "nan"))
            out.setdefault(name, {}).setdefault(ctr, []).append(val)
    return out


def _per_dispatch(table, kernel_substr, counter):
    vals = [v for name, c in table.items() if kernel_substr in name for v in c.get(counter, [])]
    return sum(vals) / len(vals) if vals else None


def reduce_pmc(directory: str, workload: str):
    """Combine four rocprofv3 --pmc runs (CSV) found under `directory`:
    fetch/ and write/ (FETCH_SIZE, WRITE_SIZE of this benchmark), and
    copy_fetch/ and copy_write/ (the same counters for `--copy-calibration`,
    a 1 GiB device copy).  Each counter is scaled by known bytes / counted
    bytes of the copy; the result is the mean per dispatch of every sweep
    kernel (each is launched once per call)."""
    def load(sub):
        files = glob.glob(os.path.join(directory, sub, "**", "*counter_collection.csv"), recursive=True)
        if not files:
            raise SystemExit(f"no counter_collection.csv under {directory}/{sub}")
        t = {}
        for p in files:
            for k, v in _read_counter_csv(p).items():
                for c, vals in v.items():
                    t.setdefault(k, {}).setdefault(c, []).extend(vals)
        return t
    fetch, write, cf, cw = load("fetch"), load("write"), load("copy_fetch"), load("copy_write")
    copy_bytes = float(1 << 30)
    # the copy kernel is the largest single dispatch of the calibration run
    cf_kib = max(sum(v) / len(v) for k in cf.values() for c, v in k.items() if c == "FETCH_SIZE")
    cw_kib = max(sum(v) / len(v) for k in cw.values() for c, v in k.items() if c == "WRITE_SIZE")
    f_read = copy_bytes / (cf_kib * 1024.0)
    f_write = copy_bytes / (cw_kib * 1024.0)
    res = {"kernel_sha": kernel_sha(), "workload": workload,
           "calibration": {"copy_bytes": copy_bytes, "fetch_kib": cf_kib, "write_kib": cw_kib,
                           "read_factor": f_read, "write_factor": f_write},
           "kernels": {}}

    def short(name):
        n = name.split("(")[0].replace("void ", "").replace("asora::", "")
        return n

    for name, c in fetch.items():
        k = short(name)
        if not any(k.startswith(sub) for subs in KERNELS.values() for sub in subs):
            continue
        wname = [n for n in write if short(n) == k]
        if not wname:
            continue
        fv, wv = c.get("FETCH_SIZE", []), write[wname[0]].get("WRITE_SIZE", [])
        if not fv or not wv:
            continue
        fb = sum(fv) / len(fv) * 1024.0 * f_read
        wb = sum(wv) / len(wv) * 1024.0 * f_write
        res["kernels"][k] = {"fetch_bytes_per_dispatch": fb, "write_bytes_per_dispatch": wb,
                             "hbm_bytes_per_dispatch": fb + wb, "dispatches": len(fv)}
    os.makedirs(os.path.dirname(pmc_file(workload)), exist_ok=True)
    with open(pmc_file(workload), "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res))


def reduce_sq(directory: str, workload: str):
    """Mean SQ_INSTS_VALU (wave instructions) and SQ_WAVES per dispatch of
    every sweep kernel, from rocprofv3 --pmc runs (CSV) found under
    `directory` (any run that collected SQ_INSTS_VALU)."""
    files = glob.glob(os.path.join(directory, "**", "*counter_collection.csv"), recursive=True)
    table = {}
    for p in files:
        for k, v in _read_counter_csv(p).items():
            for c, vals in v.items():
                table.setdefault(k, {}).setdefault(c, []).extend(vals)
    res = {"kernel_sha": kernel_sha(), "workload": workload, "valu_peak_per_s": VALU_PEAK_PER_S,
           "kernels": {}}
    for name, c in table.items():
        k = name.split("(")[0].replace("void ", "").replace("asora::", "")
        if not any(k.startswith(sub) for subs in KERNELS.values() for sub in subs):
            continue
        if "SQ_INSTS_VALU" not in c:
            continue
        v = c["SQ_INSTS_VALU"]
        res["kernels"][k] = {"valu_insts_per_dispatch": sum(v) / len(v), "dispatches": len(v)}
        if "SQ_WAVES" in c:
            res["kernels"][k]["waves_per_dispatch"] = sum(c["SQ_WAVES"]) / len(c["SQ_WAVES"])
    if not res["kernels"]:
        raise SystemExit(f"no SQ_INSTS_VALU of a sweep kernel under {directory}")
    os.makedirs(os.path.dirname(valu_file(workload)), exist_ok=True)
    with open(valu_file(workload), "w") as f:
        json.dump(res, f, indent=1)
    print(json.dumps(res))


# ---------------------------------------------------------------------------
def lattice_voxels(R, N: int) -> int:
    """The cells the sweep visits, summed over sources: lattice offsets with
    i^2 + j^2 + k^2 <= floor(R^2) inside the periodic extent (N/2 cells on the
    negative side, N/2 - 1 on the positive one for even N, (N - 1)/2 on both
    for odd N).  The exact count beside the paper's (4/3) pi R^3."""
    import numpy as np
    R = np.asarray(R, np.float64)
    if R.size == 0:
        return 0
    neg, pos = (N // 2, N // 2 - 1) if N % 2 == 0 else ((N - 1) // 2, (N - 1) // 2)
    rmax = int(math.ceil(float(R.max())))
    d = np.arange(-min(rmax, neg), min(rmax, pos) + 1, dtype=np.int64)
    r2 = (d[:, None, None] ** 2 + d[None, :, None] ** 2 + d[None, None, :] ** 2).ravel()
    cum = np.cumsum(np.bincount(r2))
    rsq = np.minimum(np.floor(R * R).astype(np.int64), len(cum) - 1)
    return int(cum[rsq].sum())


def cpu_baseline(w, budget_s: float = 12.0):
    """The FP64 oracle as it stands (forward, then reverse for
    L = sum w log10(Gamma + 1e-20)), single-threaded, on the first sources of
    the same workload until about budget_s of CPU time."""
    import numpy as np

    import oracle
    tb = oracle.blackbody_table()
    rng = np.random.default_rng(7)
    oracle.raytrace(w.N, w.cell_cm, tb, w.n_H, w.x_HI, w.src.ijk[:1], w.src.Q[:1], w.src.R[:1])
    done, work, t = 0, 0.0, 0.0
    chunk = 4
    while t < budget_s and done < len(w.src):
        sl = slice(done, min(done + chunk, len(w.src)))
        ijk, Q, R = w.src.ijk[sl], w.src.Q[sl], w.src.R[sl]
        t0 = time.perf_counter()
        g = oracle.raytrace(w.N, w.cell_cm, tb, w.n_H, w.x_HI, ijk, Q, R)
        t += time.perf_counter() - t0
        gbar = rng.standard_normal(g.shape) / ((g + 1e-20) * math.log(10))
        t0 = time.perf_counter()
        oracle.raytrace_grad(w.N, w.cell_cm, tb, w.n_H, w.x_HI, ijk, Q, R, gbar)
        t += time.perf_counter() - t0
        work += float(np.sum(4.0 / 3.0 * math.pi * R.astype(np.float64) ** 3))
        done = sl.stop
    return {"value": t / work * 1e9, "unit": "ns per source-voxel", "cores": 1, "kind": "oracle",
            "sample": f"forward + reverse of the first {done} of {len(w.src)} sources of the same "
                      f"workload ({t:.1f} s, one thread, FP64)"}


def test1_time_steps(asora, torch):
    """Test 1 of Section 4.1 with the library's time step (asora_time_step):
    one source of 1e48 photons/s in uniform gas (n_H = 1e-3 cm^-3, T = 1e4 K,
    case-B alpha = 2.59e-13 cm^3/s, grey opacity) at the centre of a
    (10 kpc)^3 box on 128^3 cells, ten coarse steps of 50 Myr, each iterated
    to convergence.  Wall time per step and the I-front radius along x over
    the analytic r_S (1 - exp(-t/t_rec))^(1/3)."""
    import numpy as np
    N, kpc, myr = 128, 3.0856775814913673e21, 3.15576e13
    ndot, nh0, alpha = 1e48, 1e-3, 2.59e-13
    cell = 10.0 * kpc / N
    c = N // 2
    P, dP = asora.table_grey()
    ctx = asora.Asora(N, cell, P, dP, -20.0, math.log10(80.0))
    dev = torch.device("cuda")
    nH = torch.full((N ** 3,), nh0, dtype=torch.float32, device=dev)
    ijk = torch.tensor([[c, c, c]], dtype=torch.int32, device=dev)
    Q = torch.tensor([ndot], dtype=torch.float64, device=dev)
    R = torch.tensor([N / 2 - 0.5], dtype=torch.float32, device=dev)
    y = torch.ones(N ** 3, dtype=torch.float64, device=dev)
    r_s = (3.0 * ndot / (4.0 * math.pi * alpha * nh0 ** 2)) ** (1.0 / 3.0)
    t_rec = 1.0 / (alpha * nh0)
    dt = 50.0 * myr
    ms, passes, ratio = [], [], []
    for k in range(10):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ye, ya, g, p = ctx.time_step(nH, y, ijk, Q, R, dt, alpha)
        torch.cuda.synchronize()
        ms.append((time.perf_counter() - t0) * 1e3)
        passes.append(p)
        y = ye.reshape(-1).contiguous()
        line = ye[c, c, c:].double().cpu().numpy()
        k2 = int(np.argmax(line >= 0.5)) if (line >= 0.5).any() else len(line)
        r_i = cell * ((k2 - 1) + (0.5 - line[k2 - 1]) / (line[k2] - line[k2 - 1])) if 0 < k2 < len(line) else 0.0
        ratio.append(r_i / (r_s * (1.0 - math.exp(-(k + 1) * dt / t_rec)) ** (1.0 / 3.0)))
    ctx.close()
    return {"grid": N, "steps": 10, "dt_Myr": 50.0, "ms_per_step": ms, "passes": passes,
            "rI_over_analytic": ratio}


def parse_tuning(text):
    """'R_oct=10,table_place=lds,adj_rate=gathered' -> keyword arguments of
    Asora.set_tuning (the named values are those the JSON line prints)."""
    named = {"table_place": {"lds": 1, "caches": 2}, "adj_rate": {"gathered": 1, "split": 2}}
    out = {}
    for item in filter(None, text.split(",")):
        k, v = item.split("=")
        k = k.strip()
        if k in named and v in named[k]:
            out[k] = named[k][v]
        else:
            out[k] = float(v) if k in ("R_whole", "R_oct") else int(v)
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-plain", action="store_true", help="skip the one-launch-per-source form")
    ap.add_argument("--no-tune", action="store_true", help="keep the default scheduling parameters")
    ap.add_argument("--no-test1", action="store_true", help="skip the Test 1 time steps (chemistry)")
    ap.add_argument("--no-graph", action="store_true",
                    help="skip the recorded-graph timing (its sweeps share kernel names with the eager ones)")
    ap.add_argument("--no-early-exit", action="store_true",
                    help="skip the early-exit timings (their sweeps share kernel names with the full ones)")
    ap.add_argument("--tuning", metavar="K=V,...",
                    help="set these scheduling parameters instead of autotuning (keys as in the "
                         "JSON line's tuning object, e.g. R_oct=10,adj_rate=gathered)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--reduce-pmc", metavar="DIR", help="reduce rocprofv3 counter CSVs and exit")
    ap.add_argument("--reduce-sq", metavar="DIR",
                    help="reduce rocprofv3 SQ counter CSVs (VALU instructions) and exit")
    args = ap.parse_args()
    if args.reduce_pmc:
        reduce_pmc(args.reduce_pmc, args.workload)
        return
    if args.reduce_sq:
        reduce_sq(args.reduce_sq, args.workload)
        return
    if args.gpus != 1:
        print(f"bench.py: one GPU only; --gpus {args.gpus} is not supported (sources would shard "
              f"over GPUs with one all-reduce of Gamma, which is not built)", file=sys.stderr)
        sys.exit(2)
    args.steps = max(1, min(args.steps, 32))   # the library keeps events of the last 64 calls

    import numpy as np
    import torch

    if args.copy_calibration:
        n = 1 << 28
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
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
    lattice = lattice_voxels(w.src.R, w.N)
    n3 = w.N ** 3
    gamma = torch.empty(n3, dtype=torch.float32, device=dev)
    dn = torch.empty(n3, dtype=torch.float32, device=dev)
    dx = torch.empty(n3, dtype=torch.float32, device=dev)
    dq = torch.empty(len(w.src), dtype=torch.float64, device=dev)

    # dL/dGamma of L = sum w log10(Gamma + 1e-20), w ~ N(0,1) seeded, at this Gamma
    ctx.raytrace(nH, xH, ijk, Q, R, R_max=R_max, out=gamma)
    wt = torch.from_numpy(np.random.default_rng(w.seed + 1).standard_normal(n3)).to(dev)
    gbar = (wt / ((gamma.double() + 1e-20) * math.log(10))).contiguous()

    def fwd(profile=False, plain=False, n=None, store=False):
        s = slice(0, n)
        ctx.raytrace(nH, xH, ijk[s], Q[s], R[s], R_max=R_max, out=gamma, plain=plain, profile=profile,
                     store=store)

    def adj(profile=False, store=False):
        ctx.backward(nH, xH, ijk, Q, R, gbar, R_max=R_max, profile=profile, out=(dn, dx, dq), store=store)

    # ---- scheduling parameters: the library's autotuner on this workload
    # (forward with kept records + adjoint), before anything is timed
    tuning = {"autotuned": False}
    if args.tuning:
        ctx.set_tuning(**parse_tuning(args.tuning))
    elif not args.no_tune:
        print("[bench] autotune", file=sys.stderr, flush=True)
        best, rep = ctx.autotune(nH, xH, ijk, Q, R, R_max=R_max, passes=2)
        tuning = {"autotuned": True, "candidates": len(rep), "best_ms": best}
    tun = dict(zip(asora.TUNING_KEYS, ctx.get_tuning()))
    tun["table_place"] = "lds" if tun["table_place"] == 1 else "caches"
    tun["adj_rate"] = "split" if tun["adj_rate"] == 2 else "gathered"
    tuning.update(tun)

    def timed_step(store):
        """Mean wall ms per step over args.steps steps (warm-up first), and the
        HIP-event durations of the sweep kernels and of the whole calls."""
        for _ in range(args.warmup):
            fwd(store=store)
            adj(store=store)
        torch.cuda.synchronize()
        ctx.profile_read()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fwd(profile=True, store=store)
            adj(profile=True, store=store)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / args.steps * 1e3
        ctx.check()
        prof = ctx.profile_read()
        assert len(prof) == 2 * args.steps, len(prof)
        return {"ms": ms, "fwd_sweep_ms": float(np.mean([p[0] for p in prof[0::2]])),
                "adj_sweep_ms": float(np.mean([p[0] for p in prof[1::2]])),
                "fwd_call_ms": float(np.mean([p[1] for p in prof[0::2]])),
                "adj_call_ms": float(np.mean([p[1] for p in prof[1::2]]))}

    # ---- the step: forward + adjoint, sweep kernels timed with HIP events.
    # With the column records kept by the forward when they fit in memory
    # (what the differentiable path does), else recomputed by the adjoint.
    print(f"[bench] timing {args.steps} steps (kept column records)", file=sys.stderr, flush=True)
    step_kept = timed_step(True)
    kept, keep_bytes, _ = ctx.store_info()
    print(f"[bench] timing {args.steps} steps (recompute)", file=sys.stderr, flush=True)
    step_rc = timed_step(False)
    step = step_kept if kept else step_rc
    ms = step["ms"]
    fwd_sweep_ms, adj_sweep_ms = step["fwd_sweep_ms"], step["adj_sweep_ms"]
    fwd_call_ms, adj_call_ms = step["fwd_call_ms"], step["adj_call_ms"]

    # ---- the same step recorded once as a HIP graph and replayed
    graph_ms = None
    if not args.no_graph:
        print("[bench] recorded step", file=sys.stderr, flush=True)
        graph = ctx.record_step(nH, xH, ijk, Q, R, gamma, dL_dgamma=gbar, grads=(dn, dx, dq), R_max=R_max,
                                store=kept)
        for _ in range(args.warmup):
            graph.launch()
        # wall clock bracketed by synchronizations, as the eager step is timed
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            graph.launch()
        torch.cuda.synchronize()
        graph_ms = (time.perf_counter() - t0) / args.steps * 1e3
        ctx.check()
        graph.close()

    # ---- batched forward alone
    print("[bench] batched forward", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        fwd()
    torch.cuda.synchronize()
    fwd_ms = (time.perf_counter() - t0) / args.steps * 1e3

    # ---- the exact early exit (ASORA_EARLY_EXIT): each pyramid stops after its
    # first opaque layer.  Same Gamma, fewer cells swept: not the graded
    # metric, which counts every cell of every ball.
    ee_fwd_ms = ee_step_ms = None
    if not args.no_early_exit:
        print("[bench] early-exit forward and step", file=sys.stderr, flush=True)

        def fwd_early(store=False):
            ctx.raytrace(nH, xH, ijk, Q, R, R_max=R_max, out=gamma, store=store, early_exit=True)

        for _ in range(args.warmup):
            fwd_early()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fwd_early()
        torch.cuda.synchronize()
        ee_fwd_ms = (time.perf_counter() - t0) / args.steps * 1e3
        for _ in range(args.warmup):
            fwd_early(store=True)
            adj(store=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            fwd_early(store=True)
            adj(store=True)
        torch.cuda.synchronize()
        ee_step_ms = (time.perf_counter() - t0) / args.steps * 1e3

    # ---- the photo-heating sweep (asora_raytrace_heating): the rate and the
    # heating of the same black body from one sweep, two table lookups per cell
    print("[bench] heating forward", file=sys.stderr, flush=True)
    Hh, dHh = asora.table_blackbody_heat(5e4, 2.8, 2000, -20.0, 4.0)
    ctx.set_heating_table(Hh, dHh)
    heat = torch.empty_like(gamma)

    def fwd_heat():
        ctx.raytrace_heating(nH, xH, ijk, Q, R, R_max=R_max, out=gamma, heating_out=heat)

    for _ in range(args.warmup):
        fwd_heat()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        fwd_heat()
    torch.cuda.synchronize()
    heat_ms = (time.perf_counter() - t0) / args.steps * 1e3

    traffic = {}
    if os.path.exists(pmc_file(args.workload)):
        pmc = json.load(open(pmc_file(args.workload)))
        if pmc.get("kernel_sha") == kernel_sha() and pmc.get("workload") == args.workload:
            traffic = {k: v.get("hbm_bytes_per_dispatch") for k, v in pmc.get("kernels", {}).items()}
    valu = {}
    if os.path.exists(valu_file(args.workload)):
        vj = json.load(open(valu_file(args.workload)))
        if vj.get("kernel_sha") == kernel_sha() and vj.get("workload") == args.workload:
            valu = {k: v.get("valu_insts_per_dispatch") for k, v in vj.get("kernels", {}).items()}

    # the dominant sweep kernels: layer pyramids (sweep 3) or shell pyramids;
    # the step's adjoint reads kept records or recomputes; the forward alone
    # keeps nothing
    tun = dict(zip(asora.TUNING_KEYS, ctx.get_tuning()))
    big = R_max > tun["R_oct"]
    layer = big and tun["pyramid_sweep"] == 3
    tl = "true" if tun["table_place"] == 1 else "false"
    sp = "true" if tun["adj_rate"] == 2 else "false"
    kname = {"fwd": f"fwd_layer<false, {tl}>" if layer else "fwd_wave<2>",
             "adj": ("adj_layer<true, false>" if kept else f"adj_layer<false, {sp}>") if layer
             else "adj_wave<2>"}
    if not big:
        kname = {"fwd": "fwd_wave<1>", "adj": "adj_wave<1>"}
    # the step's forward keeps the records when they fit (layer pieces only)
    kname["fwd_step"] = f"fwd_layer<true, {tl}>" if (kept and layer) else kname["fwd"]
    fwd_step_bytes = KEEP_FWD_BYTES_PER_SV if (kept and layer) else FWD_BYTES_PER_SV

    def roof(bytes_per_sv, sweep_ms, kernel, key):
        achieved = bytes_per_sv * work / (sweep_ms * 1e-3) / 1e9
        r = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
             "frac": achieved / HBM_PEAK_GBS, "traffic": traffic.get(kernel),
             "kernel": kernel, "launch_ms": sweep_ms,
             "alg_bytes_per_source_voxel": bytes_per_sv, "source_voxels_per_launch": work}
        # the limit that binds: VALU issue, from the kernel's counted wave
        # instructions per dispatch (null when the counters are stale)
        vi = valu.get(kernel)
        r["valu_issue"] = None if vi is None else {
            "insts_per_launch": vi, "achieved_per_s": vi / (sweep_ms * 1e-3), "peak_per_s": VALU_PEAK_PER_S,
            "frac": vi / (sweep_ms * 1e-3) / VALU_PEAK_PER_S}
        return r

    out = {
        "metric": METRIC, "value": ms * 1e6 / work, "unit": "ns per source-voxel", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64/f32", "data": "synthetic",
        "ns_per_lattice_voxel": ms * 1e6 / lattice,
        "config": {"workload": f"{args.workload}: {spec['desc']}", "grid": w.N, "lattice_voxels": lattice,
                   "n_sources": len(w.src), "source_voxels": work, "seed": w.seed,
                   "step": "batched forward + adjoint" + (" (columns kept by the forward)" if kept
                                                          else " (columns recomputed by the adjoint)")},
        # the step's longer sweep kernel (forward or adjoint)
        "roofline": (roof(fwd_step_bytes, fwd_sweep_ms, kname["fwd_step"], "fwd") if fwd_sweep_ms >= adj_sweep_ms
                     else roof(ADJ_BYTES_PER_SV, adj_sweep_ms, kname["adj"], "adj")),
        "step_sweeps": {"fwd": roof(fwd_step_bytes, fwd_sweep_ms, kname["fwd_step"], "fwd"),
                        "adj": roof(ADJ_BYTES_PER_SV, adj_sweep_ms, kname["adj"], "adj")},
        "fwd": {"ns_per_source_voxel": fwd_ms * 1e6 / work, "ms_per_call": fwd_ms,
                "roofline": roof(FWD_BYTES_PER_SV, step_rc["fwd_sweep_ms"], kname["fwd"], "fwd")},
        "adjoint": {"ns_per_source_voxel": (ms - fwd_ms) * 1e6 / work,
                    "sweep_ms": adj_sweep_ms, "call_ms": adj_call_ms},
        "fwd_call_ms_in_step": fwd_call_ms,
        "tuning": tuning,
        "graph_step": (None if graph_ms is None else
                       {"ms_per_step": graph_ms, "ns_per_source_voxel": graph_ms * 1e6 / work}),
        "steps_by_mode": {
            "kept": {"ns_per_source_voxel": step_kept["ms"] * 1e6 / work, "ms_per_step": step_kept["ms"],
                     "adj_sweep_ms": step_kept["adj_sweep_ms"], "fwd_sweep_ms": step_kept["fwd_sweep_ms"],
                     "records_kept": kept, "record_bytes": keep_bytes},
            "recompute": {"ns_per_source_voxel": step_rc["ms"] * 1e6 / work, "ms_per_step": step_rc["ms"],
                          "adj_sweep_ms": step_rc["adj_sweep_ms"], "fwd_sweep_ms": step_rc["fwd_sweep_ms"]}},
    }

    if not args.no_plain:
        n = min(spec["plain_src"], len(w.src))
        sub_work = float(np.sum(4.0 / 3.0 * math.pi * w.src.R[:n].astype(np.float64) ** 3))
        print(f"[bench] plain forward, {n} launches", file=sys.stderr, flush=True)
        fwd(plain=True, n=n)
        torch.cuda.synchronize()
        reps = 2
        t0 = time.perf_counter()
        for _ in range(reps):
            fwd(plain=True, n=n)
        torch.cuda.synchronize()
        pms = (time.perf_counter() - t0) / reps * 1e3
        out["plain"] = {"ns_per_source_voxel": pms * 1e6 / sub_work, "sources": n,
                        "ms_per_call": pms,
                        "plain_over_batched_fwd": (pms * 1e6 / sub_work) / out["fwd"]["ns_per_source_voxel"]}
    if ee_fwd_ms is not None:
        out["early_exit"] = {
            "note": "ASORA_EARLY_EXIT: same Gamma, fewer cells swept; ns are per source-voxel of the full "
                    "balls, so not comparable with value",
            "fwd_ms_per_call": ee_fwd_ms, "fwd_speedup": fwd_ms / ee_fwd_ms,
            "step_ms": ee_step_ms, "step_speedup": ms / ee_step_ms}
    out["heating"] = {
        "note": "asora_raytrace_heating: Gamma and the photo-heating rate from one sweep (two table "
                "lookups per cell); ns per source-voxel of the same balls",
        "fwd_ms_per_call": heat_ms, "ns_per_source_voxel": heat_ms * 1e6 / work,
        "over_fwd_alone": heat_ms / fwd_ms}
    # ---- the chemistry step on the same grid (asora_chemistry): elementwise,
    # HBM-bound; 44 algorithmic bytes per cell (Gamma, n_H FP32, x_HI and the
    # previous <x_HI> FP64 in; <x_HI>, x_HI(dt) FP64 and <x_HI> FP32 out)
    print("[bench] chemistry step", file=sys.stderr, flush=True)
    ctx.raytrace(nH, xH, ijk, Q, R, R_max=R_max, out=gamma)
    y0 = xH.double()
    n3 = w.N ** 3
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(args.warmup):
        ctx.chemistry(gamma, nH, y0, 1.6e15, 2.59e-13, xHI_avg_prev=y0)
    torch.cuda.synchronize()
    reps = 20
    ev0.record()
    for _ in range(reps):
        ctx.chemistry(gamma, nH, y0, 1.6e15, 2.59e-13)
    ev1.record()
    torch.cuda.synchronize()
    chem_ms = ev0.elapsed_time(ev1) / reps
    chem_gbs = 44.0 * n3 / (chem_ms * 1e-3) / 1e9
    out["chemistry"] = {"ms_per_call": chem_ms, "cells": n3, "alg_bytes_per_cell": 44,
                        "roofline": {"bound": "hbm", "achieved": chem_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                     "frac": chem_gbs / HBM_PEAK_GBS}}
    if not args.no_test1:
        out["test1_time_steps"] = test1_time_steps(asora, torch)
    out["paper_context"] = {"value": 3.156, "unit": "ns per source-voxel (forward)",
                            "hardware": "1x NVIDIA Tesla P100, FP64 grid data",
                            "workload": "250^3, R in {10,30,50,100}, up to 1e6 sources (asymptote)"}
    if not args.no_cpu:
        print("[bench] CPU oracle baseline", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
