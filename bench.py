"""Benchmark of the ASORA ray-tracing step (forward and adjoint) on one MI355X.

A step is one pass of the whole hot path over the workload's source list:
the forward sweep (asora_raytrace: n_HI and accumulator set-up, scheduling
sort, persistent sweep over all source pieces, FP32 conversion of Gamma)
followed by the adjoint (asora_raytrace_backward: the same set-up, the
columns from the records the forward kept when they fit in memory, else
recomputed per piece, reverse sweep, dL/dn_H and dL/dx_HI conversion) for a
fixed dL/dGamma, all inputs resident in HBM.  Both passes sweep every cell
of every ball (no early exit).  The metric is the paper's time per source
per voxel, t / sum_s (4/3) pi R_s^3 (Section 4.2), in ns: `value` is the
forward+adjoint step; the batched forward alone and the plain form (one
launch per source, on a seeded 1 % subset of the sources) are reported
beside it, and the FP64 CPU oracle on the host's cores.

Default workload: the million-source 250^3 step (1.396 Mpc cells, lognormal
density, x_HI from a thresholded smoothed field, 1e6 sources with R uniform
in [5, 40] cells), the largest configuration that fits one GPU.  The
scheduling parameters come from the library's autotuner, whose results for
the measured workloads are kept in paper_2311_01492_amd/tuning_cache.txt.
Prints one JSON line.

`--reduce-pmc DIR` turns rocprofv3 counter runs (CSV output) of this script
into the per-launch HBM traffic file read here, `--reduce-sq DIR` the SQ
instruction counters into the VALU-issue file and `--reduce-lds DIR` the LDS
byte counters into the LDS-traffic file (the commands that made them head the
summaries under profiles/).
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
FWD_BYTES_PER_SV = 24.0   # n_H + x_HI reads (2 x FP32), Gamma accumulator read-modify-write (2 x FP64)
ADJ_BYTES_PER_SV = 32.0   # n_H + x_HI (2 x FP32), dL/dGamma (FP64), dL/dn_HI read-modify-write (2 x FP64)
# column records, a separate term: one FP64 entry per cell, written by the
# forward that keeps them and read back by the adjoint (the rate's three FP64
# coefficients per cell with a rate come on top; their count depends on the
# field)
REC_BYTES_PER_CELL = 8.0
# the sweep kernels' sources and the plans that size their launches (waves,
# LDS, the table of square roots): counters taken on other versions are not used
KERNEL_SOURCES = ["paper_2311_01492_amd/csrc/asora_dev.h", "paper_2311_01492_amd/csrc/asora_fwd.hip",
                  "paper_2311_01492_amd/csrc/asora_adj.hip", "paper_2311_01492_amd/csrc/asora_internal.h",
                  "paper_2311_01492_amd/csrc/asora_api.hip"]
# sweep kernels of each pass (one dispatch per piece kind up to the largest
# radius; the kinds without sources return at once)
KERNELS = {"fwd": ("fwd_wave", "fwd_layer"), "adj": ("adj_wave", "adj_layer")}

WORKLOADS = {
    "c2": dict(name="c2", kw={},
               desc="128^3, cell 4.3e24 cm, lognormal n_H (ln sigma 0.5, P(k)~k^-2) x 1.5e-4, "
                    "x_HI 1e-3 in U[2,8]-cell bubbles, 1000 sources, Q 10^U[51,55], R=30"),
    "c3": dict(name="c3", kw={},
               desc="250^3, cell 4.308e24 cm, lognormal + bubbles, 1e5 sources, Q 10^U[50,55], R U[5,50]"),
    "c5": dict(name="c5", kw={},
               desc="250^3, cell 4.308e24 cm, lognormal n_H, x_HI 1e-3 where the sigma=3 smoothed field "
                    "exceeds its median (else 1), 1e6 sources, Q 10^U[50,54], R U[5,40]"),
}
# the plain form: a seeded subset of 1 % of the sources, at least 1000 (all of
# a smaller list), timed and scaled by its own source-voxels
PLAIN_FRACTION, PLAIN_MIN = 0.01, 1000


def _code_only(text: str) -> str:
    """C++ source without comments and whitespace: what the compiler sees,
    so that edits of the prose alone keep the profiles' hash."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if text.startswith("//", i):
            i = text.find("\n", i)
            i = n if i < 0 else i
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            i = n if j < 0 else j + 2
        elif c in "\"'":   # string or character literal, kept as written
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        else:
            if not c.isspace():
                out.append(c)
            i += 1
    return "".join(out)


def kernel_sha(root: str = ROOT) -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        h.update(_code_only(open(os.path.join(root, f), encoding="utf-8").read()).encode())
    return h.hexdigest()[:16]


def pmc_file(workload: str) -> str:
    return os.path.join(ROOT, "profiles", f"hbm_traffic_{workload}.json")


def valu_file(workload: str) -> str:
    return os.path.join(ROOT, "profiles", f"valu_issue_{workload}.json")


def lds_file(workload: str) -> str:
    return os.path.join(ROOT, "profiles", f"lds_traffic_{workload}.json")


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


def reduce_lds(directory: str, workload: str):
    """Mean LDS bytes per dispatch of every sweep kernel from rocprofv3 --pmc
    runs (CSV) under `directory` that collected SQ_INSTS_LDS_LOAD_BANDWIDTH,
    SQ_INSTS_LDS_STORE_BANDWIDTH and SQ_INSTS_LDS_ATOMIC_BANDWIDTH (each counts
    64-byte units: instruction width times active lanes), with the bank-conflict
    and LDS-busy cycles when present."""
    files = glob.glob(os.path.join(directory, "**", "*counter_collection.csv"), recursive=True)
    table = {}
    for p in files:
        for k, v in _read_counter_csv(p).items():
            for c, vals in v.items():
                table.setdefault(k, {}).setdefault(c, []).extend(vals)
    res = {"kernel_sha": kernel_sha(), "workload": workload, "kernels": {}}
    mean = lambda v: sum(v) / len(v)
    for name, c in table.items():
        k = name.split("(")[0].replace("void ", "").replace("asora::", "")
        if not any(k.startswith(sub) for subs in KERNELS.values() for sub in subs):
            continue
        if "SQ_INSTS_LDS_LOAD_BANDWIDTH" not in c:
            continue
        e = {part: 64.0 * mean(c[f"SQ_INSTS_LDS_{part.upper()}_BANDWIDTH"])
             for part in ("load", "store", "atomic") if f"SQ_INSTS_LDS_{part.upper()}_BANDWIDTH" in c}
        e = {f"{part}_bytes_per_dispatch": v for part, v in e.items()}
        e["lds_bytes_per_dispatch"] = sum(e.values())
        for ctr in ("SQ_LDS_BANK_CONFLICT", "SQ_LDS_IDX_ACTIVE", "SQ_ACTIVE_INST_LDS", "SQ_INSTS_LDS"):
            if ctr in c:
                e[ctr] = mean(c[ctr])
        e["dispatches"] = len(c["SQ_INSTS_LDS_LOAD_BANDWIDTH"])
        res["kernels"][k] = e
    if not res["kernels"]:
        raise SystemExit(f"no LDS byte counters of a sweep kernel under {directory}")
    os.makedirs(os.path.dirname(lds_file(workload)), exist_ok=True)
    with open(lds_file(workload), "w") as f:
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


def host_cpu():
    """The timing host: CPU model, logical CPUs, and the CPUs this process may
    run on (capped at 16, the host share of one GPU on the GPU hosts)."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        allowed = len(os.sched_getaffinity(0))
    except AttributeError:
        allowed = os.cpu_count() or 1
    return {"model": model, "nproc": os.cpu_count(), "allowed": allowed, "used_max": min(allowed, 16)}


def cpu_baseline(w, gbar, budget_s: float = 10.0):
    """The FP64 oracle as it stands: forward (Gamma) then reverse mode (for the
    step's dL/dGamma) of a seeded random sample of the workload's sources,
    each run one oracle call over its sample.  First on one thread, then on
    every allowed core (up to 16): the sources split over threads, each its
    own oracle call (the oracle's C code runs without the interpreter lock),
    the sum over sources being the paper's source split (Section 3.2).  Each
    sample is sized to about budget_s of one core's work."""
    import concurrent.futures as cf

    import numpy as np

    import oracle
    tb = oracle.blackbody_table()
    perm = np.random.default_rng(w.seed + 2).permutation(len(w.src))
    sv = 4.0 / 3.0 * math.pi * w.src.R.astype(np.float64) ** 3

    def run(idx):
        idx = np.sort(idx)
        ijk, Q, R = w.src.ijk[idx], w.src.Q[idx], w.src.R[idx]
        t0 = time.perf_counter()
        oracle.raytrace(w.N, w.cell_cm, tb, w.n_H, w.x_HI, ijk, Q, R)
        oracle.raytrace_grad(w.N, w.cell_cm, tb, w.n_H, w.x_HI, ijk, Q, R, gbar)
        return time.perf_counter() - t0

    def take(start, seconds, rate):
        """Sources perm[start:stop] worth about `seconds` at `rate` s per sv."""
        cum = np.cumsum(sv[perm[start:]]) * rate
        n = max(1, int(np.searchsorted(cum, seconds)))
        return start + min(n, len(perm) - start)

    pos = 4
    rate = run(perm[:pos]) / float(sv[perm[:pos]].sum())       # calibration (wrapper included)
    stop = take(pos, budget_s, rate)
    idx1 = perm[pos:stop]
    t1 = run(idx1)
    work1 = float(sv[idx1].sum())
    rate = t1 / work1
    hc = host_cpu()
    cores = hc["used_max"]
    slices = []
    pos = stop
    for _ in range(cores):
        if pos >= len(perm):
            break
        stop = take(pos, budget_s, rate)
        slices.append(perm[pos:stop])
        pos = stop
    t0 = time.perf_counter()
    with cf.ThreadPoolExecutor(max_workers=len(slices)) as ex:
        list(ex.map(run, slices))
    tall = time.perf_counter() - t0
    work_all = float(sum(sv[s].sum() for s in slices))
    n_all = int(sum(len(s) for s in slices))
    return {"value": tall / work_all * 1e9, "unit": "ns per source-voxel", "cores": len(slices),
            "kind": "oracle",
            "sample": f"forward + reverse of {n_all} seeded random sources of the {len(w.src)} of the same "
                      f"workload, split over {len(slices)} threads, one oracle call each ({tall:.1f} s wall, "
                      f"FP64)",
            "host": hc,
            "single_thread": {"value": t1 / work1 * 1e9, "cores": 1, "sources": int(len(idx1)),
                              "seconds": t1}}


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
    ap.add_argument("--workload", default="c5", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-plain", action="store_true", help="skip the one-launch-per-source form")
    ap.add_argument("--no-tune", action="store_true", help="keep the default scheduling parameters")
    ap.add_argument("--retune", action="store_true", help="autotune even if the tuning cache has the workload")
    ap.add_argument("--save-tuning", metavar="PATH", help="write the autotuner's results to PATH")
    ap.add_argument("--no-test1", action="store_true", help="skip the Test 1 time steps (chemistry)")
    ap.add_argument("--no-graph", action="store_true",
                    help="skip the recorded-graph timing (its sweeps share kernel names with the eager ones)")
    ap.add_argument("--no-early-exit", action="store_true",
                    help="skip the early-exit timings (their sweeps share kernel names with the full ones)")
    ap.add_argument("--no-heating", action="store_true", help="skip the photo-heating forward")
    ap.add_argument("--no-helium", action="store_true", help="skip the two-absorber (HI, HeI) forward")
    ap.add_argument("--tuning", metavar="K=V,...",
                    help="set these scheduling parameters instead of autotuning (keys as in the "
                         "JSON line's tuning object, e.g. R_oct=10,adj_rate=gathered)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration)")
    ap.add_argument("--reduce-pmc", metavar="DIR", help="reduce rocprofv3 counter CSVs and exit")
    ap.add_argument("--reduce-sq", metavar="DIR",
                    help="reduce rocprofv3 SQ counter CSVs (VALU instructions) and exit")
    ap.add_argument("--reduce-lds", metavar="DIR",
                    help="reduce rocprofv3 LDS byte counter CSVs and exit")
    args = ap.parse_args()
    if args.reduce_pmc:
        reduce_pmc(args.reduce_pmc, args.workload)
        return
    if args.reduce_sq:
        reduce_sq(args.reduce_sq, args.workload)
        return
    if args.reduce_lds:
        reduce_lds(args.reduce_lds, args.workload)
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

    def say(msg):
        print(f"[bench] {msg}", file=sys.stderr, flush=True)

    spec = WORKLOADS[args.workload]
    say(f"building workload {args.workload}")
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
    del wt

    def fwd(profile=False, plain=False, store=False, early=False, src=None):
        i3, q, r = (ijk, Q, R) if src is None else src
        ctx.raytrace(nH, xH, i3, q, r, R_max=R_max, out=gamma, plain=plain, profile=profile,
                     store=store, early_exit=early)

    def adj(profile=False, store=False, early=False):
        ctx.backward(nH, xH, ijk, Q, R, gbar, R_max=R_max, profile=profile, out=(dn, dx, dq), store=store,
                     early_exit=early)

    def wall(fn, reps, warm=1):
        """Mean wall ms of fn() over reps calls bracketed by synchronizations."""
        for _ in range(warm):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps * 1e3

    # ---- scheduling parameters: the library's autotuner on this workload
    # (forward with kept records + adjoint), before anything is timed; its
    # results for the measured workloads are cached in a file
    tuning = {"autotuned": False}
    if args.tuning:
        ctx.set_tuning(**parse_tuning(args.tuning))
    elif not args.no_tune:
        cached = ctx.load_tuning(asora.TUNING_CACHE) if not args.retune else 0
        say("autotune" + (f" ({cached} cached results)" if cached else ""))
        ctx.set_tune_progress(lambda row, rep: say("  candidate " + ", ".join(
            f"{k}={v:g}" for k, v in row.items()) + ("" if rep else " (adj_rate preselection)")))
        t0 = time.perf_counter()
        best, rep = ctx.autotune(nH, xH, ijk, Q, R, R_max=R_max, passes=2, retune=args.retune)
        tuning = {"autotuned": True, "candidates_timed": len(rep), "from_cache": len(rep) == 0,
                  "best_ms": best, "seconds": time.perf_counter() - t0}
        if args.save_tuning:
            ctx.save_tuning(args.save_tuning)
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
    fwd(store=True)
    torch.cuda.synchronize()
    kept, keep_bytes, _ = ctx.store_info()
    step_kept = None
    if kept:
        say(f"timing {args.steps} steps (kept column records)")
        step_kept = timed_step(True)
    say(f"timing {args.steps} steps (columns recomputed by the adjoint)")
    step_rc = timed_step(False)
    step = step_kept if kept else step_rc
    ms = step["ms"]
    fwd_sweep_ms, adj_sweep_ms = step["fwd_sweep_ms"], step["adj_sweep_ms"]
    fwd_call_ms, adj_call_ms = step["fwd_call_ms"], step["adj_call_ms"]
    # side measurements: about 8 s each at most, at least 2 calls
    side = max(2, min(args.steps, int(math.ceil(8000.0 / max(ms, 1e-3)))))

    # ---- the same step recorded once as a HIP graph and replayed
    graph_ms = None
    if not args.no_graph:
        say("recorded step")
        graph = ctx.record_step(nH, xH, ijk, Q, R, gamma, dL_dgamma=gbar, grads=(dn, dx, dq), R_max=R_max,
                                store=kept)
        # wall clock bracketed by synchronizations, as the eager step is timed
        graph_ms = wall(graph.launch, side)
        ctx.check()
        graph.close()

    # ---- batched forward alone
    say("batched forward")
    fwd_ms = wall(fwd, max(side, min(args.steps, 2 * side)))

    # ---- the exact early exit (ASORA_EARLY_EXIT): each pyramid stops after its
    # first opaque layer, in both passes.  Same Gamma and gradients, fewer
    # cells swept: not the graded metric, which counts every cell of every ball.
    ee = None
    if not args.no_early_exit:
        say("early-exit forward and step")
        ee_fwd_ms = wall(lambda: fwd(early=True), side)
        fwd(store=True, early=True)
        torch.cuda.synchronize()
        ee_kept = ctx.store_info()[0]
        ee_step_ms = wall(lambda: (fwd(store=ee_kept, early=True), adj(store=ee_kept, early=True)), side)
        ee = {"note": "ASORA_EARLY_EXIT in both passes: same Gamma and gradients, fewer cells swept; ns are "
                      "per source-voxel of the full balls, so not comparable with value",
              "fwd_ms_per_call": ee_fwd_ms, "fwd_speedup": fwd_ms / ee_fwd_ms,
              "step_ms": ee_step_ms, "step_speedup": ms / ee_step_ms, "records_kept": ee_kept}

    # ---- the photo-heating sweep (asora_raytrace_heating): the rate and the
    # heating of the same black body from one sweep, two table lookups per cell
    heat_ms = None
    if not args.no_heating:
        say("heating forward")
        Hh, dHh = asora.table_blackbody_heat(5e4, 2.8, 2000, -20.0, 4.0)
        ctx.set_heating_table(Hh, dHh)
        heat = torch.empty_like(gamma)
        heat_ms = wall(lambda: ctx.raytrace_heating(nH, xH, ijk, Q, R, R_max=R_max, out=gamma,
                                                    heating_out=heat), side)
        del heat

    # ---- the two-absorber sweep (asora_raytrace_helium): HI and HeI columns
    # per cell, a black body in four bands with a table each, on the same
    # balls (n_He = 0.0789 n_H, x_HeI = x_HI)
    he_ms = None
    if not args.no_helium:
        say("helium forward")
        from workloads import HE_ABUNDANCE, HE_BAND_EDGES_EV, HE_BAND_LG_HI, helium_cross_sections
        sH, sHe = helium_cross_sections()
        bands = []
        for b in range(len(sH)):
            Pb, dPb = asora.table_blackbody_band(HE_BAND_EDGES_EV[b], HE_BAND_EDGES_EV[b + 1], 5e4, 2.8, 2000,
                                                 -20.0, HE_BAND_LG_HI[b])
            bands.append((Pb, dPb, -20.0, HE_BAND_LG_HI[b], sH[b], sHe[b]))
        ctx.set_helium(bands)
        nHe = (nH * HE_ABUNDANCE).contiguous()
        gH, gHe = torch.empty_like(gamma), torch.empty_like(gamma)
        he_ms = wall(lambda: ctx.raytrace_helium(nH, xH, nHe, xH, ijk, Q, R, R_max=R_max, out=(gH, gHe)), side)
        del gH, gHe, nHe

    def counters(path):
        if not os.path.exists(path):
            return {}
        j = json.load(open(path))
        if j.get("kernel_sha") != kernel_sha() or j.get("workload") != args.workload:
            return {}
        return j.get("kernels", {})

    traffic = {k: v.get("hbm_bytes_per_dispatch") for k, v in counters(pmc_file(args.workload)).items()}
    valu = {k: v.get("valu_insts_per_dispatch") for k, v in counters(valu_file(args.workload)).items()}
    lds = {k: v for k, v in counters(lds_file(args.workload)).items()}

    # the dominant sweep kernels: layer pyramids (sweep 3) or shell pyramids;
    # the step's adjoint reads kept records or recomputes; the forward alone
    # keeps nothing
    tun = dict(zip(asora.TUNING_KEYS, ctx.get_tuning()))
    big = R_max > tun["R_oct"]
    layer = big and tun["pyramid_sweep"] == 3
    tl = "true" if tun["table_place"] == 1 else "false"
    sp = "true" if tun["adj_rate"] == 2 and not kept else "false"
    aw = 16 if tun["adj_waves"] > 12 else 12   # the layer adjoint's build (wide above 12 waves)
    kname = {"fwd": f"fwd_layer<false, {tl}>" if layer else "fwd_wave<2>",
             "adj": f"adj_layer<{'true' if kept else 'false'}, {sp}, {aw}>" if layer else "adj_wave<2>"}
    if not big:
        kname = {"fwd": "fwd_wave<1>", "adj": "adj_wave<1>"}
    # the step's forward keeps the records when they fit (layer pieces only)
    kname["fwd_step"] = f"fwd_layer<true, {tl}>" if (kept and layer) else kname["fwd"]
    rec_step = kept and layer

    def roof(bytes_per_sv, sweep_ms, kernel, record):
        """Roofline of one sweep kernel: algorithmic bytes per launch over its
        mean HIP-event duration; the column records' bytes (kept records) as a
        separate term; counted HBM traffic, VALU issue and LDS bytes from the
        profiles when they were taken on the current kernel sources."""
        achieved = bytes_per_sv * work / (sweep_ms * 1e-3) / 1e9
        r = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
             "frac": achieved / HBM_PEAK_GBS, "traffic": traffic.get(kernel),
             "kernel": kernel, "launch_ms": sweep_ms,
             "alg_bytes_per_source_voxel": bytes_per_sv, "source_voxels_per_launch": work,
             "record_bytes_per_launch": REC_BYTES_PER_CELL * lattice if record else 0.0}
        vi = valu.get(kernel)
        r["valu_issue"] = None if vi is None else {
            "insts_per_launch": vi, "per_source_voxel": 64.0 * vi / work,
            "achieved_per_s": vi / (sweep_ms * 1e-3), "peak_per_s": VALU_PEAK_PER_S,
            "frac": vi / (sweep_ms * 1e-3) / VALU_PEAK_PER_S}
        li = lds.get(kernel)
        r["lds"] = None if li is None else {
            "bytes_per_launch": li["lds_bytes_per_dispatch"],
            "achieved_GBs": li["lds_bytes_per_dispatch"] / (sweep_ms * 1e-3) / 1e9,
            "bank_conflict_over_active": (li["SQ_LDS_BANK_CONFLICT"] / li["SQ_LDS_IDX_ACTIVE"]
                                          if li.get("SQ_LDS_IDX_ACTIVE") else None)}
        return r

    fwd_roof = roof(FWD_BYTES_PER_SV, fwd_sweep_ms, kname["fwd_step"], rec_step)
    adj_roof = roof(ADJ_BYTES_PER_SV, adj_sweep_ms, kname["adj"], rec_step)
    out = {
        "metric": METRIC, "value": ms * 1e6 / work, "unit": "ns per source-voxel", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": False,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64/f32", "data": "synthetic",
        "ns_per_lattice_voxel": ms * 1e6 / lattice,
        "config": {"workload": f"{args.workload}: {spec['desc']}", "grid": w.N, "lattice_voxels": lattice,
                   "n_sources": len(w.src), "source_voxels": work, "seed": w.seed,
                   "step": "batched forward + adjoint, every cell of every ball"
                           + (" (columns kept by the forward)" if kept
                              else " (columns recomputed by the adjoint: the records do not fit)")},
        # the step's longer sweep kernel (forward or adjoint)
        "roofline": fwd_roof if fwd_sweep_ms >= adj_sweep_ms else adj_roof,
        "step_sweeps": {"fwd": fwd_roof, "adj": adj_roof, "adj_over_fwd": adj_sweep_ms / fwd_sweep_ms},
        "fwd": {"ns_per_source_voxel": fwd_ms * 1e6 / work, "ms_per_call": fwd_ms,
                "roofline": roof(FWD_BYTES_PER_SV, step_rc["fwd_sweep_ms"], kname["fwd"], False)},
        "adjoint": {"ns_per_source_voxel": (ms - fwd_ms) * 1e6 / work,
                    "sweep_ms": adj_sweep_ms, "call_ms": adj_call_ms},
        "fwd_call_ms_in_step": fwd_call_ms,
        "tuning": tuning,
        "graph_step": (None if graph_ms is None else
                       {"ms_per_step": graph_ms, "ns_per_source_voxel": graph_ms * 1e6 / work, "replays": side}),
        "steps_by_mode": {
            "recompute": {"ns_per_source_voxel": step_rc["ms"] * 1e6 / work, "ms_per_step": step_rc["ms"],
                          "adj_sweep_ms": step_rc["adj_sweep_ms"], "fwd_sweep_ms": step_rc["fwd_sweep_ms"]},
            "kept": (None if step_kept is None else
                     {"ns_per_source_voxel": step_kept["ms"] * 1e6 / work, "ms_per_step": step_kept["ms"],
                      "adj_sweep_ms": step_kept["adj_sweep_ms"], "fwd_sweep_ms": step_kept["fwd_sweep_ms"],
                      "record_bytes": keep_bytes}),
            "records_kept": kept, "record_bytes_needed": keep_bytes},
    }

    if not args.no_plain:
        n = min(len(w.src), max(PLAIN_MIN, int(math.ceil(PLAIN_FRACTION * len(w.src)))))
        idx = np.sort(np.random.default_rng(w.seed + 3).choice(len(w.src), size=n, replace=False))
        sub_work = float(np.sum(4.0 / 3.0 * math.pi * w.src.R[idx].astype(np.float64) ** 3))
        sub = tuple(t[torch.from_numpy(idx).to(dev)].contiguous() for t in (ijk, Q, R))
        say(f"plain forward, {n} launches")
        pms = wall(lambda: fwd(plain=True, src=sub), 2)
        out["plain"] = {"ns_per_source_voxel": pms * 1e6 / sub_work, "sources": n,
                        "subset": f"seeded {n} of {len(w.src)} sources", "ms_per_call": pms,
                        "plain_over_batched_fwd": (pms * 1e6 / sub_work) / out["fwd"]["ns_per_source_voxel"]}
    if ee is not None:
        out["early_exit"] = ee
    if heat_ms is not None:
        out["heating"] = {
            "note": "asora_raytrace_heating: Gamma and the photo-heating rate from one sweep (two table "
                    "lookups per cell); ns per source-voxel of the same balls",
            "fwd_ms_per_call": heat_ms, "ns_per_source_voxel": heat_ms * 1e6 / work,
            "over_fwd_alone": heat_ms / fwd_ms}
    if he_ms is not None:
        out["helium"] = {
            "note": "asora_raytrace_helium: Gamma_HI and Gamma_HeI from one sweep carrying the HI and HeI "
                    "columns, four spectral bands (two tables per band and cell); ns per source-voxel of the "
                    "same balls",
            "fwd_ms_per_call": he_ms, "ns_per_source_voxel": he_ms * 1e6 / work, "over_fwd_alone": he_ms / fwd_ms}
    # ---- the chemistry step on the same grid (asora_chemistry): elementwise,
    # HBM-bound; 44 algorithmic bytes per cell (Gamma, n_H FP32, x_HI and the
    # previous <x_HI> FP64 in; <x_HI>, x_HI(dt) FP64 and <x_HI> FP32 out)
    say("chemistry step")
    fwd()
    y0 = xH.double()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(args.warmup):
        ctx.chemistry(gamma, nH, y0, 1.6e15, 2.59e-13, xHI_avg_prev=y0)
    torch.cuda.synchronize()
    reps = 20
    ev0.record()
    for _ in range(reps):
        ctx.chemistry(gamma, nH, y0, 1.6e15, 2.59e-13, xHI_avg_prev=y0)
    ev1.record()
    torch.cuda.synchronize()
    chem_ms = ev0.elapsed_time(ev1) / reps
    chem_gbs = 44.0 * n3 / (chem_ms * 1e-3) / 1e9
    out["chemistry"] = {"ms_per_call": chem_ms, "cells": n3, "alg_bytes_per_cell": 44,
                        "roofline": {"bound": "hbm", "achieved": chem_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                     "frac": chem_gbs / HBM_PEAK_GBS}}
    del y0
    if not args.no_test1:
        out["test1_time_steps"] = test1_time_steps(asora, torch)
    out["paper_context"] = {"value": 3.156, "unit": "ns per source-voxel (forward)",
                            "hardware": "1x NVIDIA Tesla P100, FP64 grid data",
                            "workload": "250^3, R in {10,30,50,100}, up to 1e6 sources (asymptote)"}
    if not args.no_cpu:
        say("CPU oracle baseline")
        gb_host = gbar.cpu().numpy().reshape(w.N, w.N, w.N)
        ctx.close()
        out["cpu_baseline"] = cpu_baseline(w, gb_host)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
