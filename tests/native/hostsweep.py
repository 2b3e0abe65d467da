"""ctypes access to tests/native/host_sweep.hip (CPU build of the library's
per-cell code, driven serially).  Test infrastructure."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
LIB = os.path.join(HERE, "_build", "libhostsweep.so")
SRCS = [os.path.join(HERE, "host_sweep.hip"),
        os.path.join(ROOT, "paper_2311_01492_amd", "csrc", "asora_tables.cpp")]
DEPS = SRCS + [os.path.join(ROOT, "paper_2311_01492_amd", "csrc", f) for f in ("asora_dev.h", "asora_internal.h")]
_lib = None


def build(force=False):
    if force or not os.path.exists(LIB) or any(os.path.getmtime(LIB) < os.path.getmtime(d) for d in DEPS):
        os.makedirs(os.path.dirname(LIB), exist_ok=True)
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.run(["/opt/rocm/bin/hipcc", "-O2", "-std=c++17", "-fPIC", "-shared",
                        "--offload-arch=gfx950", "-o", tmp] + SRCS, check=True, capture_output=True)
        os.replace(tmp, LIB)
    return LIB


def load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(LIB)
        p, i, d, f, l = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_float, ctypes.c_long
        lib.hc_rectwalk_check.restype = i
        lib.hc_rectwalk_check.argtypes = [i]
        lib.hc_raytrace.restype = i
        lib.hc_raytrace.argtypes = [i, d, d, i, d, d, p, p, d, i, p, p, l, p, p, p, f, f, i, p, p]
        lib.hc_neg_divdiff_batch.restype = None
        lib.hc_neg_divdiff_batch.argtypes = [i, d, d, p, p, l, p, p, p]
        lib.hc_rate_derivs64_batch.restype = None
        lib.hc_rate_derivs64_batch.argtypes = [i, d, d, p, p, l, p, p, p]
        lib.hc_tab_eval64_batch.restype = None
        lib.hc_tab_eval64_batch.argtypes = [i, d, d, p, p, l, p, p]
        lib.hc_raytrace_grad.restype = i
        lib.hc_raytrace_grad.argtypes = [i, d, d, i, d, d, p, p, d, i, p, p, l, p, p, p, f, f, i, p, p, p]
        lib.hc_raytrace_layer.restype = i
        lib.hc_raytrace_layer.argtypes = [i, d, d, i, d, d, p, p, d, i, p, p, l, p, p, p, p, p]
        lib.hc_raytrace_layer_grad.restype = i
        lib.hc_raytrace_layer_grad.argtypes = [i, d, d, i, d, d, p, p, d, i, p, p, l, p, p, p, p, p, p, i,
                                               p]
        lib.hc_rows.restype = i
        lib.hc_rows.argtypes = [i, i, i, i, i, p, p]
        _lib = lib
    return _lib


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def raytrace(N, cell_cm, sigma0, table, n_H, x_HI, ijk, Q, R, tau_w=0.6, reading=0, type_force=-1,
             R_whole=10.0, R_oct=30.0, coldens=False, layers=False):
    """type_force: shell piece kind for every source (0, 1, 2), or -1 by radius;
    layers: every source as layer pyramids."""
    lib = load()
    g = np.zeros(N ** 3)
    cd = np.zeros(N ** 3) if coldens else None
    P, dP = np.ascontiguousarray(table.P, np.float64), np.ascontiguousarray(table.dP, np.float64)
    nH = np.ascontiguousarray(n_H, np.float32)
    xH = np.ascontiguousarray(x_HI, np.float32)
    ijk = np.ascontiguousarray(ijk, np.int32)
    Q = np.ascontiguousarray(Q, np.float64)
    R = np.ascontiguousarray(R, np.float32)
    if layers:
        st = lib.hc_raytrace_layer(N, cell_cm, sigma0, len(P), table.lg_lo, table.lg_hi, _p(P), _p(dP),
                                   float(tau_w), reading, _p(nH), _p(xH), len(Q), _p(ijk), _p(Q),
                                   _p(R), _p(g), _p(cd))
    else:
        st = lib.hc_raytrace(N, cell_cm, sigma0, len(P), table.lg_lo, table.lg_hi, _p(P), _p(dP),
                             float(tau_w), reading, _p(nH), _p(xH), len(Q), _p(ijk), _p(Q), _p(R),
                             R_whole, R_oct, type_force, _p(g), _p(cd))
    if st != 0:
        raise RuntimeError(f"host sweep failed: {st}")
    g = g.reshape((N,) * 3)
    return (g, cd.reshape((N,) * 3)) if coldens else g


def rectwalk_check(wv_max):
    return load().hc_rectwalk_check(int(wv_max))


def neg_divdiff(table, a, dt):
    lib = load()
    a = np.ascontiguousarray(a, np.float64)
    dt = np.ascontiguousarray(dt, np.float64)
    out = np.empty(a.shape, np.float32)
    P, dP = np.ascontiguousarray(table.P, np.float64), np.ascontiguousarray(table.dP, np.float64)
    lib.hc_neg_divdiff_batch(len(P), table.lg_lo, table.lg_hi, _p(P), _p(dP), a.size, _p(a), _p(dt), _p(out))
    return out


def rate_derivs64(table, a, dt):
    """(D, dD/da, dD/d(dt)) of the adjoint's FP64 rate derivatives, [m, 3]."""
    lib = load()
    a = np.ascontiguousarray(a, np.float64)
    dt = np.ascontiguousarray(dt, np.float64)
    out = np.empty((a.size, 3), np.float64)
    P, dP = np.ascontiguousarray(table.P, np.float64), np.ascontiguousarray(table.dP, np.float64)
    lib.hc_rate_derivs64_batch(len(P), table.lg_lo, table.lg_hi, _p(P), _p(dP), a.size, _p(a), _p(dt),
                               _p(out))
    return out


def tab_eval64(table, tau):
    """The library's FP64 interpolant (P, dP/dtau, d2P/dtau2) at tau, [m, 3]."""
    lib = load()
    tau = np.ascontiguousarray(tau, np.float64)
    out = np.empty((tau.size, 3), np.float64)
    P, dP = np.ascontiguousarray(table.P, np.float64), np.ascontiguousarray(table.dP, np.float64)
    lib.hc_tab_eval64_batch(len(P), table.lg_lo, table.lg_hi, _p(P), _p(dP), tau.size, _p(tau), _p(out))
    return out


def rows(N, type_, piece, Rsq, q):
    lib = load()
    n = (8 if type_ == 0 else 1) * (q + 1)
    blo = np.zeros(n, np.int32)
    cnt = np.zeros(n, np.int32)
    lib.hc_rows(N, type_, piece, Rsq, q, _p(blo), _p(cnt))
    return blo, cnt


def raytrace_grad(N, cell_cm, sigma0, table, n_H, x_HI, ijk, Q, R, gbar, tau_w=0.6, reading=0,
                  type_force=-1, R_whole=10.0, R_oct=30.0, layers=False, split=True, kept=False,
                  stats=None, early_exit=False):
    """(dL/dn_H, dL/dx_HI, dL/dQ) for dL/dGamma = gbar (FP64); layers: every
    source as layer pyramids, the rate terms of dense chunks in the reverse
    pass (split) or all gathered first, or (kept) taken from coefficients the
    forward pass stored, as with records kept by the forward.  stats (a dict,
    layers only) receives n_stopped: the pyramids whose adjoint stopped at an
    opaque layer before their last, and visited / total: cells (rectangle
    slots) in the layers the adjoint visits / in all layers.  early_exit: every
    pass of a pyramid stops at its first opaque layer (otherwise all layers
    are visited)."""
    lib = load()
    P, dP = np.ascontiguousarray(table.P, np.float64), np.ascontiguousarray(table.dP, np.float64)
    nH = np.ascontiguousarray(n_H, np.float32)
    xH = np.ascontiguousarray(x_HI, np.float32)
    ijk = np.ascontiguousarray(ijk, np.int32)
    Q = np.ascontiguousarray(Q, np.float64)
    R = np.ascontiguousarray(R, np.float32)
    gb = np.ascontiguousarray(gbar, np.float64)
    nbar = np.zeros(N ** 3)
    qbar = np.zeros(len(Q))
    if layers:
        st3 = np.zeros(3, np.int64)
        st = lib.hc_raytrace_layer_grad(N, cell_cm, sigma0, len(P), table.lg_lo, table.lg_hi, _p(P),
                                        _p(dP), float(tau_w), reading, _p(nH), _p(xH), len(Q), _p(ijk),
                                        _p(Q), _p(R), _p(gb), _p(nbar), _p(qbar),
                                        (2 if kept else (1 if split else 0)) | (4 if early_exit else 0),
                                        _p(st3))
        if stats is not None:
            stats.update(n_stopped=int(st3[0]), visited=int(st3[1]), total=int(st3[2]))
    else:
        st = lib.hc_raytrace_grad(N, cell_cm, sigma0, len(P), table.lg_lo, table.lg_hi, _p(P), _p(dP),
                                  float(tau_w), reading, _p(nH), _p(xH), len(Q), _p(ijk), _p(Q), _p(R),
                                  R_whole, R_oct, type_force, _p(gb), _p(nbar), _p(qbar))
    if st != 0:
        raise RuntimeError(f"host grad failed: {st}")
    nbar = nbar.reshape((N,) * 3)
    return xH.astype(np.float64) * nbar, nH.astype(np.float64) * nbar, qbar


def log_fast(a):
    lib = load()
    lib.hc_log_fast.restype = ctypes.c_double
    lib.hc_log_fast.argtypes = [ctypes.c_double]
    return lib.hc_log_fast(float(a))


def log_f64(a):
    lib = load()
    lib.hc_log_f64.restype = ctypes.c_double
    lib.hc_log_f64.argtypes = [ctypes.c_double]
    return lib.hc_log_f64(float(a))
