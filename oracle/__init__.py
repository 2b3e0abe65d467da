"""FP64 CPU oracle of the ASORA ray-tracing step -- TEST INFRASTRUCTURE ONLY.

Only the tests, the smoke check and the CPU-baseline leg of the benchmark may
import this package.  It shares no code with the HIP library
(paper_2311_01492_amd): the sweep is plain sequential C (asora_oracle.c,
FP64, built with -O2 -ffp-contract=off), the tables come from SciPy quadrature
(tables.py) and the long-characteristics brute force is numpy (lc.py).

Every function follows the paper's statement of the method; see the header
of asora_oracle.c for the passages and the readings of unstated points.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from .tables import (SIGMA0, Table, blackbody_band_table, blackbody_heat_table,  # noqa: F401
                     blackbody_table, grey_table)

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "asora_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

ORC_OK, ORC_EINVAL, ORC_ENOMEM, ORC_ECAUSAL, ORC_EZERO = 0, -1, -2, -5, -6


def build(force: bool = False) -> str:
    """Compile asora_oracle.c with gcc (FP64, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-std=gnu11",
                               "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB)
        d, i, l, p = ctypes.c_double, ctypes.c_int, ctypes.c_long, ctypes.c_void_p
        lib.oracle_raytrace.restype = i
        lib.oracle_raytrace.argtypes = [i, d, d, i, d, d, p, p, d, i, p, l, p, p, p, p, p]
        lib.oracle_raytrace_grad.restype = i
        lib.oracle_raytrace_grad.argtypes = [i, d, d, i, d, d, p, p, d, i, p, l, p, p, p, p, p, p]
        lib.oracle_table_eval.restype = d
        lib.oracle_table_eval.argtypes = [i, d, d, p, p, d, p, p]
        lib.oracle_interp.restype = d
        lib.oracle_interp.argtypes = [p, p, d, d, p]
        lib.oracle_shell_order.restype = l
        lib.oracle_shell_order.argtypes = [i, d, p, p, l]
        lib.oracle_neighbours.restype = i
        lib.oracle_neighbours.argtypes = [p, p, p]
        lib.oracle_raytrace_he.restype = i
        lib.oracle_raytrace_he.argtypes = [i, d, d, i, i, p, p, p, p, p, p, d, i, p, p, l, p, p, p, p, p, p,
                                           p]
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p) if a is not None else None


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


class OracleError(RuntimeError):
    pass


def _check(st):
    if st != ORC_OK:
        raise OracleError({ORC_EINVAL: "invalid argument", ORC_ENOMEM: "out of memory",
                           ORC_ECAUSAL: "causality violated", ORC_EZERO: "n_HI = 0 in reverse mode"}
                          .get(st, str(st)))


def n_HI(n_H, x_HI):
    """Neutral hydrogen density n_HI = n_H x_HI, formed in FP64."""
    return _f64(n_H) * _f64(x_HI)


def raytrace(N, cell_cm, table: Table, n_H, x_HI, ijk, Q, R, sigma0=SIGMA0, tau_w=0.6,
             reading=0, coldens=False):
    """Photoionization rate Gamma (FP64, N^3) summed over sources; with
    coldens=True (single source only) also the entry column N_in (cm^-2)."""
    lib = _load()
    nhi = n_HI(n_H, x_HI).reshape(-1)
    assert nhi.size == N ** 3
    ijk = np.ascontiguousarray(ijk, dtype=np.int32).reshape(-1, 3)
    Qa, Ra = _f64(Q).reshape(-1), _f64(R).reshape(-1)
    gam = np.zeros(N ** 3)
    cd = np.zeros(N ** 3) if coldens else None
    st = lib.oracle_raytrace(N, cell_cm, sigma0, table.n, table.lg_lo, table.lg_hi,
                             _ptr(_f64(table.P)), _ptr(_f64(table.dP)), float(tau_w), int(reading),
                             _ptr(nhi), ijk.shape[0], _ptr(ijk), _ptr(Qa), _ptr(Ra), _ptr(gam), _ptr(cd))
    _check(st)
    gam = gam.reshape(N, N, N)
    return (gam, cd.reshape(N, N, N)) if coldens else gam


def raytrace_helium(N, cell_cm, bands, n_H, x_HI, n_He, x_HeI, ijk, Q, R, sigma0=SIGMA0, tau_w=0.6,
                    reading=0, coldens=False):
    """Photoionization rates of HI and HeI (FP64, N^3 each) summed over
    sources, for a spectrum in bands: `bands` is a sequence of (Table,
    sigma_HI, sigma_HeI), each band's table P_b on its own nodes (the
    photons of the band that survive an optical depth measured at its lower
    edge) and the two cross-sections (cm^2) there.  n_HI = n_H x_HI and
    n_HeI = n_He x_HeI are formed in FP64.  With coldens=True (single source)
    also the entry columns of HI and HeI.  The readings are those listed in
    asora_oracle.c above oracle_raytrace_he."""
    lib = _load()
    nhi = n_HI(n_H, x_HI).reshape(-1)
    nhe = (_f64(n_He) * _f64(x_HeI)).reshape(-1)
    assert nhi.size == N ** 3 and nhe.size == N ** 3
    nb = len(bands)
    ntab = bands[0][0].n
    assert all(t.n == ntab for t, _, _ in bands)
    lg_lo = _f64([t.lg_lo for t, _, _ in bands])
    lg_hi = _f64([t.lg_hi for t, _, _ in bands])
    P = _f64(np.concatenate([t.P for t, _, _ in bands]))
    dP = _f64(np.concatenate([t.dP for t, _, _ in bands]))
    sH = _f64([b[1] for b in bands])
    sHe = _f64([b[2] for b in bands])
    ijk = np.ascontiguousarray(ijk, dtype=np.int32).reshape(-1, 3)
    Qa, Ra = _f64(Q).reshape(-1), _f64(R).reshape(-1)
    gH, gHe = np.zeros(N ** 3), np.zeros(N ** 3)
    cH = np.zeros(N ** 3) if coldens else None
    cHe = np.zeros(N ** 3) if coldens else None
    st = lib.oracle_raytrace_he(N, cell_cm, sigma0, nb, ntab, _ptr(lg_lo), _ptr(lg_hi), _ptr(P), _ptr(dP),
                                _ptr(sH), _ptr(sHe), float(tau_w), int(reading), _ptr(nhi), _ptr(nhe),
                                ijk.shape[0], _ptr(ijk), _ptr(Qa), _ptr(Ra), _ptr(gH), _ptr(gHe), _ptr(cH),
                                _ptr(cHe))
    _check(st)
    shape = (N, N, N)
    if coldens:
        return gH.reshape(shape), gHe.reshape(shape), cH.reshape(shape), cHe.reshape(shape)
    return gH.reshape(shape), gHe.reshape(shape)


def raytrace_heating(N, cell_cm, heat_table: Table, n_H, x_HI, ijk, Q, R, sigma0=SIGMA0, tau_w=0.6,
                     reading=0):
    """Photo-heating rate per HI atom (eV/s, FP64, N^3) summed over sources,
    for the heating table H of the sources' spectrum (tables.blackbody_H).

    The heating of a cell is the energy its HI absorbs, Q [H(tau_in) -
    H(tau_out)], over n_HI V, as the rate is the photons it absorbs, Q
    [P(tau_in) - P(tau_out)], over n_HI V (eq. sugg): the same sweep and the
    same columns with H in place of P.  Both are linear in the table, so
    this is the rate computation given the heating table."""
    return raytrace(N, cell_cm, heat_table, n_H, x_HI, ijk, Q, R, sigma0=sigma0, tau_w=tau_w,
                    reading=reading)


def raytrace_grad(N, cell_cm, table: Table, n_H, x_HI, ijk, Q, R, gbar, sigma0=SIGMA0,
                  tau_w=0.6, reading=0):
    """Reverse mode: returns (dL/dn_H, dL/dx_HI, dL/dQ) for dL/dGamma = gbar."""
    lib = _load()
    nH, xH = _f64(n_H).reshape(-1), _f64(x_HI).reshape(-1)
    nhi = nH * xH
    ijk = np.ascontiguousarray(ijk, dtype=np.int32).reshape(-1, 3)
    Qa, Ra = _f64(Q).reshape(-1), _f64(R).reshape(-1)
    nbar = np.zeros(N ** 3)
    qbar = np.zeros(ijk.shape[0])
    st = lib.oracle_raytrace_grad(N, cell_cm, sigma0, table.n, table.lg_lo, table.lg_hi,
                                  _ptr(_f64(table.P)), _ptr(_f64(table.dP)), float(tau_w), int(reading),
                                  _ptr(nhi), ijk.shape[0], _ptr(ijk), _ptr(Qa), _ptr(Ra),
                                  _ptr(_f64(gbar).reshape(-1)), _ptr(nbar), _ptr(qbar))
    _check(st)
    return ((xH * nbar).reshape(N, N, N), (nH * nbar).reshape(N, N, N), qbar)


def table_eval(table: Table, tau):
    """Interpolant P^(tau) and its first two derivatives (vectorised)."""
    lib = _load()
    tau = np.atleast_1d(np.asarray(tau, dtype=np.float64))
    P, d1, d2 = np.empty_like(tau), np.empty_like(tau), np.empty_like(tau)
    a, b = ctypes.c_double(), ctypes.c_double()
    Pp, dPp = _ptr(_f64(table.P)), _ptr(_f64(table.dP))
    for k, t in enumerate(tau):
        P[k] = lib.oracle_table_eval(table.n, table.lg_lo, table.lg_hi, Pp, dPp, float(t),
                                     ctypes.byref(a), ctypes.byref(b))
        d1[k], d2[k] = a.value, b.value
    return P, d1, d2


def interp(d, M4, sigma0=SIGMA0, tau_w=0.6):
    """N_in of the cell at offset d from neighbour columns M4 (e1..e4 order)."""
    lib = _load()
    dd = np.ascontiguousarray(d, dtype=np.int32)
    M = _f64(M4)
    s4 = np.zeros(4)
    v = lib.oracle_interp(_ptr(dd), _ptr(M), float(sigma0), float(tau_w), _ptr(s4))
    return v, s4


def neighbours(d):
    """Offsets (k x 3) and geometric weights (k) of the non-zero-weight neighbours."""
    lib = _load()
    dd = np.ascontiguousarray(d, dtype=np.int32)
    off = np.zeros(12, dtype=np.int32)
    s = np.zeros(4)
    n = lib.oracle_neighbours(_ptr(dd), _ptr(off), _ptr(s))
    return off[:3 * n].reshape(n, 3), s[:n]


def shell_order(N, R):
    """Cells of one source in visiting order: offsets [n, 3] and shell index [n]."""
    lib = _load()
    n = lib.oracle_shell_order(int(N), float(R), None, None, 0)
    out = np.zeros((n, 3), dtype=np.int32)
    sh = np.zeros(n, dtype=np.int32)
    lib.oracle_shell_order(int(N), float(R), _ptr(out), _ptr(sh), n)
    return out, sh
