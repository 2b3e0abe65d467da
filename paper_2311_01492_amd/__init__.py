"""ASORA ray tracing on MI355X (gfx950): Python binding of libasora.so.

The binding only marshals arguments: every step of the ray-tracing step runs
in the HIP kernels of libasora.so, behind the C ABI of include/asora.h.
PyTorch supplies device memory and streams.  If the library is missing the
import fails; there is no CPU fallback.

    import paper_2311_01492_amd as asora
    P, dP = asora.table_blackbody(5e4)                 # host float64 arrays
    ctx = asora.Asora(N, cell_cm, P, dP)
    gamma = ctx.raytrace(n_H, x_HI, ijk, Q, R)         # torch tensors on cuda
    gamma = asora.raytrace(ctx, n_H, x_HI, ijk, Q, R)  # differentiable version
"""
from __future__ import annotations

import ctypes
import math
import os

import numpy as np
import torch  # loads the HIP runtime that libasora.so binds to

__all__ = ["Asora", "AsoraError", "raytrace", "table_blackbody", "table_grey", "lib_path",
           "SIGMA0", "ACCUMULATE", "PLAIN", "STORE", "HALFPATH_SCALAR"]

SIGMA0 = 6.3e-18          # HI cross-section at 13.6 eV, cm^2
ACCUMULATE, PLAIN, PROFILE, STORE, EARLY_EXIT = 0x1, 0x2, 0x4, 0x8, 0x10
HALFPATH_SCALAR = 0x1
# scheduling parameters, in the order asora_get_tuning returns them
TUNING_KEYS = ("R_whole", "R_oct", "max_waves", "pyramid_sweep", "table_place", "adj_waves", "adj_rate")

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libasora.so")
# autotuner results of the workloads measured here (asora_tuning_save format)
TUNING_CACHE = os.path.join(_HERE, "tuning_cache.txt")

if not os.path.exists(_LIB_PATH):
    raise ImportError(f"{_LIB_PATH} is not built; run `python __graft_entry__.py` or "
                      f"`python paper_2311_01492_amd/build.py` first (there is no CPU fallback)")
_lib = ctypes.CDLL(_LIB_PATH)

_c_int, _c_i64, _c_u32 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32
_c_d, _c_f, _p = ctypes.c_double, ctypes.c_float, ctypes.c_void_p

_lib.asora_init.restype = _c_int
_lib.asora_init.argtypes = [ctypes.POINTER(_p), _c_int, _c_d, _c_d, _c_d, _c_d, _c_int, _p, _p,
                            _c_d, _c_u32, _c_int]
_lib.asora_raytrace.restype = _c_int
_lib.asora_raytrace.argtypes = [_p, _p, _p, _c_i64, _p, _p, _p, _c_f, _p, _p, _c_u32, _p]
_lib.asora_raytrace_static.restype = _c_int
_lib.asora_raytrace_static.argtypes = [_p, _p, _p, _c_i64, _p, _p, _p, _c_f, _p, _p, _c_u32, _p]
_lib.asora_chemistry.restype = _c_int
_lib.asora_chemistry.argtypes = [_p, _p, _p, _p, _p, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, _p, _p, _p, ctypes.POINTER(ctypes.c_uint64), _p]
_lib.asora_time_step.restype = _c_int
_lib.asora_time_step.argtypes = [_p, _p, _p, _c_i64, _p, _p, _p, _c_f, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, ctypes.c_double, ctypes.c_double, _c_int, _c_int, _p, _p, _p,
                                 ctypes.POINTER(_c_int), _p]
_lib.asora_raytrace_backward.restype = _c_int
_lib.asora_raytrace_backward.argtypes = [_p, _p, _p, _c_i64, _p, _p, _p, _c_f, _p, _p, _p, _p,
                                         _c_u32, _p]
_lib.asora_table_blackbody.restype = _c_int
_lib.asora_table_blackbody.argtypes = [_c_d, _c_d, _c_int, _c_d, _c_d, _p, _p]
_lib.asora_table_blackbody_heat.restype = _c_int
_lib.asora_table_blackbody_heat.argtypes = [_c_d, _c_d, _c_int, _c_d, _c_d, _p, _p]
_lib.asora_set_heating_table.restype = _c_int
_lib.asora_set_heating_table.argtypes = [_p, _p, _p]
_lib.asora_raytrace_heating.restype = _c_int
_lib.asora_raytrace_heating.argtypes = [_p, _p, _p, _c_i64, _p, _p, _p, _c_f, _p, _p, _c_u32, _p]
_lib.asora_table_blackbody_band.restype = _c_int
_lib.asora_table_blackbody_band.argtypes = [_c_d, _c_d, _c_d, _c_d, _c_int, _c_d, _c_d, _p, _p]
_lib.asora_set_helium.restype = _c_int
_lib.asora_set_helium.argtypes = [_p, _c_int, _c_int, _p, _p, _p, _p, _p, _p]
_lib.asora_raytrace_helium.restype = _c_int
_lib.asora_raytrace_helium.argtypes = [_p, _p, _p, _p, _p, _c_i64, _p, _p, _p, _c_f, _p, _p, _c_u32, _p]
_lib.asora_table_grey.restype = _c_int
_lib.asora_table_grey.argtypes = [_c_int, _c_d, _c_d, _p, _p]
_lib.asora_check.restype = _c_int
_lib.asora_check.argtypes = [_p, _p]
_lib.asora_profile.restype = _c_int
_lib.asora_profile.argtypes = [_p, ctypes.POINTER(_c_d), ctypes.POINTER(_c_d)]
_lib.asora_profile_read.restype = _c_int
_lib.asora_profile_read.argtypes = [_p, _c_int, ctypes.POINTER(_c_int), _p, _p]
_lib.asora_set_tuning.restype = _c_int
_lib.asora_set_tuning.argtypes = [_p, _c_f, _c_f, _c_int, _c_int, _c_int, _c_int, _c_int]
_lib.asora_get_tuning.restype = _c_int
_lib.asora_get_tuning.argtypes = [_p, ctypes.POINTER(_c_f), ctypes.POINTER(_c_f)] + \
    [ctypes.POINTER(_c_int)] * 5
_lib.asora_store_info.restype = _c_int
_lib.asora_store_info.argtypes = [_p, ctypes.POINTER(_c_int), ctypes.POINTER(ctypes.c_uint64),
                                  ctypes.POINTER(ctypes.c_uint64)]
_lib.asora_set_store_budget.restype = _c_int
_lib.asora_set_store_budget.argtypes = [_p, ctypes.c_uint64]
_lib.asora_autotune.restype = _c_int
_lib.asora_autotune.argtypes = [_p, _p, _p, _c_i64, _p, _p, _p, _c_f, _c_int, _c_u32, _p,
                                ctypes.POINTER(_c_f), _c_int, ctypes.POINTER(_c_int), _p]
_lib.asora_graph_create.restype = _c_int
_lib.asora_graph_create.argtypes = [_p, _p, _p, _c_i64, _p, _p, _p, _c_f, _p, _p, _p, _p, _p, _c_u32,
                                    ctypes.POINTER(_p)]
_lib.asora_graph_launch.restype = _c_int
_lib.asora_graph_launch.argtypes = [_p, _p]
_lib.asora_graph_free.restype = _c_int
_lib.asora_graph_free.argtypes = [_p]
_lib.asora_last_error.restype = ctypes.c_char_p
_lib.asora_last_error.argtypes = [_p]
_lib.asora_free.restype = _c_int
_lib.asora_free.argtypes = [_p]
_lib.asora_max_sources.restype = _c_i64
_lib.asora_max_sources.argtypes = []
_lib.asora_tuning_save.restype = _c_int
_lib.asora_tuning_save.argtypes = [_p, ctypes.c_char_p]
_lib.asora_tuning_load.restype = _c_int
_lib.asora_tuning_load.argtypes = [_p, ctypes.c_char_p, ctypes.POINTER(_c_int)]
_TUNE_CB = ctypes.CFUNCTYPE(None, ctypes.POINTER(_c_f), _c_int, _p)
_lib.asora_set_tune_progress.restype = _c_int
_lib.asora_set_tune_progress.argtypes = [_p, _TUNE_CB, _p]

_STATUS = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ESTATE", -5: "ERANGE",
           -6: "ENOSYS"}


class AsoraError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


def max_sources() -> int:
    """The largest number of sources one call accepts (asora_max_sources)."""
    return int(_lib.asora_max_sources())


def lib_path() -> str:
    return _LIB_PATH


def _raise(st: int, ctx_ptr=None):
    if st != 0:
        msg = _lib.asora_last_error(ctx_ptr)
        raise AsoraError(st, msg.decode() if msg else "")


def _np_ptr(a: np.ndarray):
    return a.ctypes.data_as(_p)


def _dptr(t):
    return None if t is None else _p(t.data_ptr())


def table_blackbody(T_bb: float = 5e4, index: float = 2.8, n: int = 2000, lg_lo: float = -20.0,
                    lg_hi: float = 4.0):
    """(P, dP/dtau) as float64 numpy arrays for a black body behind a power-law
    cross-section; built by the library on the host."""
    P, dP = np.empty(n), np.empty(n)
    _raise(_lib.asora_table_blackbody(T_bb, index, n, lg_lo, lg_hi, _np_ptr(P), _np_ptr(dP)))
    return P, dP


def table_blackbody_heat(T_bb: float = 5e4, index: float = 2.8, n: int = 2000, lg_lo: float = -20.0,
                         lg_hi: float = 4.0):
    """(H, dH/dtau) in eV: the photo-heating table of the same black body, on
    the nodes of table_blackbody with the same arguments; built on the host."""
    H, dH = np.empty(n), np.empty(n)
    _raise(_lib.asora_table_blackbody_heat(T_bb, index, n, lg_lo, lg_hi, _np_ptr(H), _np_ptr(dH)))
    return H, dH


def table_blackbody_band(e_lo_eV: float, e_hi_eV: float, T_bb: float = 5e4, index: float = 2.8, n: int = 2000,
                         lg_lo: float = -20.0, lg_hi: float = 2.5):
    """(P_b, dP_b/dtau) of one band [e_lo_eV, e_hi_eV) of the black body
    (asora_table_blackbody_band; e_hi_eV = inf for an open band)."""
    P = np.empty(n)
    dP = np.empty(n)
    _raise(_lib.asora_table_blackbody_band(T_bb, index, e_lo_eV, e_hi_eV, n, lg_lo, lg_hi, _np_ptr(P), _np_ptr(dP)))
    return P, dP


def table_grey(n: int = 2000, lg_lo: float = -20.0, lg_hi: float = math.log10(80.0)):
    P, dP = np.empty(n), np.empty(n)
    _raise(_lib.asora_table_grey(n, lg_lo, lg_hi, _np_ptr(P), _np_ptr(dP)))
    return P, dP


def _stream_ptr(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return _p(s.cuda_stream)


class Asora:
    """One grid (N, cell size) and one photoionization table on one device."""

    def __init__(self, N: int, cell_cm: float, P, dPdtau, lg_lo: float = -20.0, lg_hi: float = 4.0,
                 sigma0: float = SIGMA0, tau_w: float = 0.6, halfpath_scalar: bool = False,
                 device: int | None = None):
        if not torch.cuda.is_available():
            raise AsoraError(-4, "no HIP device available (the library has no CPU path)")
        self.device = torch.cuda.current_device() if device is None else int(device)
        P = np.ascontiguousarray(P, dtype=np.float64)
        dP = np.ascontiguousarray(dPdtau, dtype=np.float64)
        self.N, self.cell_cm, self.sigma0 = int(N), float(cell_cm), float(sigma0)
        self.n_tab = int(P.size)
        h = _p()
        st = _lib.asora_init(ctypes.byref(h), self.N, self.cell_cm, self.sigma0, float(lg_lo),
                             float(lg_hi), int(P.size), _np_ptr(P), _np_ptr(dP), float(tau_w),
                             HALFPATH_SCALAR if halfpath_scalar else 0, self.device)
        _raise(st)
        self._h = h

    def close(self):
        """Release the context (not while a StepGraph of it is open)."""
        if getattr(self, "_h", None):
            _raise(_lib.asora_free(self._h), self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- argument checks shared by forward and backward ----------------------
    def _check(self, name, t, dtype, numel=None):
        """A tensor handed to the library as a raw pointer: its dtype, device,
        layout and size must be what the entry point reads or writes."""
        numel = self.N ** 3 if numel is None else numel
        if (not torch.is_tensor(t) or t.dtype != dtype or t.device != torch.device("cuda", self.device)
                or not t.is_contiguous() or t.numel() != numel):
            raise AsoraError(-1, f"{name} must be a contiguous {dtype} tensor of {numel} elements "
                                 f"on cuda:{self.device}")
        return t

    def _prep(self, n_H, x_HI, ijk, Q, R, R_max):
        dev = torch.device("cuda", self.device)
        for name, t, dt in (("n_H", n_H, torch.float32), ("x_HI", x_HI, torch.float32)):
            if t.dtype != dt or t.device != dev or not t.is_contiguous() or t.numel() != self.N ** 3:
                raise AsoraError(-1, f"{name} must be a contiguous float32 cuda tensor of N^3 cells")
        ijk = ijk.to(dev, torch.int32).contiguous()
        Q = Q.to(dev, torch.float64).contiguous()
        if R is not None and not torch.is_tensor(R):
            R = torch.full((ijk.shape[0],), float(R), dtype=torch.float32, device=dev)
        if R is not None:
            R = R.to(dev, torch.float32).contiguous()
        if R_max is None:
            R_max = float(R.max().item()) if (R is not None and R.numel()) else 0.0
        n = ijk.shape[0] if ijk.dim() == 2 else 0
        if ijk.numel() != 3 * n or Q.numel() != n or (R is not None and R.numel() != n):
            raise AsoraError(-1, "ijk must be [n,3], Q and R [n]")
        return ijk, Q, R, float(R_max), n

    def raytrace(self, n_H, x_HI, ijk, Q, R=None, R_max=None, plain=False, coldens=False,
                 out=None, accumulate=False, profile=False, store=False, early_exit=False, stream=None):
        """Gamma (float32 cuda, N^3) for the sources; with coldens=True (one
        source) also the entry column N_in (float64, N^3).  store=True keeps the
        pyramids' column records for a following backward(store=True).
        early_exit=True stops each pyramid after its first opaque layer (the
        same Gamma; fewer cells swept)."""
        ijk, Q, R, R_max, n = self._prep(n_H, x_HI, ijk, Q, R, R_max)
        dev = n_H.device
        gamma = (self._check("out", out, torch.float32) if out is not None
                 else torch.empty(self.N ** 3, dtype=torch.float32, device=dev))
        cd = torch.empty(self.N ** 3, dtype=torch.float64, device=dev) if coldens else None
        flags = (PLAIN if plain else 0) | (ACCUMULATE if accumulate else 0) | (PROFILE if profile else 0)
        flags |= (STORE if store else 0) | (EARLY_EXIT if early_exit else 0)
        st = _lib.asora_raytrace(self._h, _dptr(n_H), _dptr(x_HI), n, _dptr(ijk), _dptr(Q),
                                 _dptr(R), R_max, _dptr(gamma), _dptr(cd), flags,
                                 _stream_ptr(stream))
        _raise(st, self._h)
        shape = (self.N,) * 3
        return (gamma.view(shape), cd.view(shape)) if coldens else gamma.view(shape)

    def raytrace_static(self, n_H, x_HI, ijk, Q, R=None, R_max=None, out=None, coldens=None,
                        plain=False, accumulate=False, early_exit=False, stream=None):
        """Gamma into `out` (float32 cuda, N^3) through asora_raytrace_static,
        the entry point that allocates no device memory (N <= 64, up to 65536
        sources); `coldens` (float64 cuda N^3, one source) receives the entry
        column.  The caller provides every buffer."""
        ijk, Q, R, R_max, n = self._prep(n_H, x_HI, ijk, Q, R, R_max)
        if out is None:
            raise AsoraError(-1, "raytrace_static needs the output buffer `out`")
        self._check("out", out, torch.float32)
        if coldens is not None:
            self._check("coldens", coldens, torch.float64)
        flags = (PLAIN if plain else 0) | (ACCUMULATE if accumulate else 0) | (EARLY_EXIT if early_exit else 0)
        st = _lib.asora_raytrace_static(self._h, _dptr(n_H), _dptr(x_HI), n, _dptr(ijk), _dptr(Q), _dptr(R),
                                        R_max, _dptr(out), _dptr(coldens), flags, _stream_ptr(stream))
        _raise(st, self._h)
        return out.view((self.N,) * 3)

    def set_helium(self, bands):
        """Band tables of the two-absorber sweep (asora_set_helium): `bands` is a
        sequence of (P, dP/dtau, lg_lo, lg_hi, sigma_HI, sigma_HeI), every
        band's table on n nodes uniform in log10 tau from lg_lo to lg_hi."""
        nb = len(bands)
        n = len(bands[0][0])
        P = np.ascontiguousarray(np.concatenate([b[0] for b in bands]), dtype=np.float64)
        dP = np.ascontiguousarray(np.concatenate([b[1] for b in bands]), dtype=np.float64)
        if P.size != nb * n or dP.size != nb * n:
            raise AsoraError(-1, "every band's table must have the same number of nodes")
        col = lambda k: np.ascontiguousarray([float(b[k]) for b in bands], dtype=np.float64)
        lo, hi, sH, sHe = col(2), col(3), col(4), col(5)
        _raise(_lib.asora_set_helium(self._h, nb, n, _np_ptr(lo), _np_ptr(hi), _np_ptr(P), _np_ptr(dP),
                                     _np_ptr(sH), _np_ptr(sHe)), self._h)

    def raytrace_helium(self, n_H, x_HI, n_He, x_HeI, ijk, Q, R=None, R_max=None, plain=False, out=None,
                        accumulate=False, profile=False, stream=None):
        """(Gamma_HI, Gamma_HeI), float32 cuda N^3 each, from one two-absorber
        sweep (asora_raytrace_helium); out = (gamma_HI, gamma_HeI) to fill."""
        ijk, Q, R, R_max, n = self._prep(n_H, x_HI, ijk, Q, R, R_max)
        for name, t in (("n_He", n_He), ("x_HeI", x_HeI)):
            self._check(name, t, torch.float32)
        dev = n_H.device
        if out is not None:
            gH, gHe = out
            self._check("gamma_HI", gH, torch.float32)
            self._check("gamma_HeI", gHe, torch.float32)
        else:
            gH = torch.empty(self.N ** 3, dtype=torch.float32, device=dev)
            gHe = torch.empty_like(gH)
        flags = (PLAIN if plain else 0) | (ACCUMULATE if accumulate else 0) | (PROFILE if profile else 0)
        st = _lib.asora_raytrace_helium(self._h, _dptr(n_H), _dptr(x_HI), _dptr(n_He), _dptr(x_HeI), n, _dptr(ijk),
                                        _dptr(Q), _dptr(R), R_max, _dptr(gH), _dptr(gHe), flags,
                                        _stream_ptr(stream))
        _raise(st, self._h)
        shape = (self.N,) * 3
        return gH.view(shape), gHe.view(shape)

    def set_heating_table(self, H, dHdtau):
        """Photo-heating table (host arrays on this context's table nodes)."""
        H = np.ascontiguousarray(H, dtype=np.float64)
        dH = np.ascontiguousarray(dHdtau, dtype=np.float64)
        if H.shape != (self.n_tab,) or dH.shape != (self.n_tab,):
            raise AsoraError(-1, f"H and dH/dtau must be 1-d arrays of the table's {self.n_tab} nodes")
        _raise(_lib.asora_set_heating_table(self._h, _np_ptr(H), _np_ptr(dH)), self._h)

    def raytrace_heating(self, n_H, x_HI, ijk, Q, R=None, R_max=None, plain=False, out=None,
                         heating_out=None, accumulate=False, profile=False, store=False,
                         early_exit=False, stream=None):
        """(Gamma, heating) from one sweep: float32 cuda N^3 each, heating in
        the heating table's energy unit per second per HI atom."""
        ijk, Q, R, R_max, n = self._prep(n_H, x_HI, ijk, Q, R, R_max)
        dev = n_H.device
        gamma = (self._check("out", out, torch.float32) if out is not None
                 else torch.empty(self.N ** 3, dtype=torch.float32, device=dev))
        heat = (self._check("heating_out", heating_out, torch.float32) if heating_out is not None
                else torch.empty_like(gamma))
        flags = (PLAIN if plain else 0) | (ACCUMULATE if accumulate else 0) | (PROFILE if profile else 0)
        flags |= (STORE if store else 0) | (EARLY_EXIT if early_exit else 0)
        st = _lib.asora_raytrace_heating(self._h, _dptr(n_H), _dptr(x_HI), n, _dptr(ijk), _dptr(Q),
                                         _dptr(R), R_max, _dptr(gamma), _dptr(heat), flags,
                                         _stream_ptr(stream))
        _raise(st, self._h)
        shape = (self.N,) * 3
        return gamma.view(shape), heat.view(shape)

    def backward(self, n_H, x_HI, ijk, Q, R, dL_dgamma, R_max=None, profile=False, stream=None,
                 out=None, store=False, early_exit=False):
        """(dL/dn_H, dL/dx_HI, dL/dQ) for the given dL/dgamma (converted to FP64).
        out: optional (dn [N^3 float32], dx [N^3 float32], dq [n float64]) to fill.
        store=True: use the column records kept by raytrace(store=True) with the
        same tensors (which must not have changed since), else recompute.
        early_exit=True stops each pyramid at its first opaque layer (kept
        records are used only if their forward made the same choice)."""
        ijk, Q, R, R_max, n = self._prep(n_H, x_HI, ijk, Q, R, R_max)
        dev = n_H.device
        g = dL_dgamma.to(dev, torch.float64).contiguous()
        if out is not None:
            dn, dx, dq = out
            for t, dt, m in ((dn, torch.float32, self.N ** 3), (dx, torch.float32, self.N ** 3),
                             (dq, torch.float64, n)):
                if t.dtype != dt or t.device != dev or not t.is_contiguous() or t.numel() != m:
                    raise AsoraError(-1, "backward out buffers: contiguous cuda (N^3 f32, N^3 f32, n f64)")
        else:
            dn = torch.empty(self.N ** 3, dtype=torch.float32, device=dev)
            dx = torch.empty_like(dn)
            dq = torch.empty(n, dtype=torch.float64, device=dev)
        st = _lib.asora_raytrace_backward(self._h, _dptr(n_H), _dptr(x_HI), n, _dptr(ijk),
                                          _dptr(Q), _dptr(R), R_max, _dptr(g), _dptr(dn),
                                          _dptr(dx), _dptr(dq),
                                          (PROFILE if profile else 0) | (STORE if store else 0) |
                                          (EARLY_EXIT if early_exit else 0),
                                          _stream_ptr(stream))
        _raise(st, self._h)
        shape = (self.N,) * 3
        return dn.view(shape), dx.view(shape), dq

    def profile(self):
        """(sweep_ms, total_ms) of the last call made with profile=True."""
        a, b = _c_d(), _c_d()
        _raise(_lib.asora_profile(self._h, ctypes.byref(a), ctypes.byref(b)), self._h)
        return a.value, b.value

    def profile_read(self, max_calls: int = 64):
        """[(sweep_ms, total_ms), ...] of the profiled calls since the previous
        read, oldest first (at most the last 64)."""
        a = np.zeros(max_calls)
        b = np.zeros(max_calls)
        n = _c_int()
        _raise(_lib.asora_profile_read(self._h, int(max_calls), ctypes.byref(n), _np_ptr(a),
                                       _np_ptr(b)), self._h)
        return list(zip(a[:n.value].tolist(), b[:n.value].tolist()))

    def autotune(self, n_H, x_HI, ijk, Q, R=None, R_max=None, passes=1, retune=False, stream=None):
        """Time candidate scheduling parameters on these inputs (library's
        asora_autotune) and keep the fastest.  Returns (best_ms, report) with one
        dict per timed candidate."""
        ijk, Q, R, R_max, n = self._prep(n_H, x_HI, ijk, Q, R, R_max)
        rep = np.zeros((64, 8), np.float32)
        best, nrep = _c_f(), _c_int()
        _raise(_lib.asora_autotune(self._h, _dptr(n_H), _dptr(x_HI), n, _dptr(ijk), _dptr(Q), _dptr(R),
                                   R_max, int(passes), 1 if retune else 0, _stream_ptr(stream),
                                   ctypes.byref(best), 64, ctypes.byref(nrep),
                                   rep.ctypes.data_as(_p)), self._h)
        keys = TUNING_KEYS + ("ms",)
        return best.value, [dict(zip(keys, map(float, r))) for r in rep[:nrep.value]]

    def set_tune_progress(self, fn):
        """fn(row: dict, in_report: bool) is called after every candidate the
        autotuner times (asora_set_tune_progress); None removes it."""
        if fn is None:
            self._tune_cb = None
            _raise(_lib.asora_set_tune_progress(self._h, ctypes.cast(None, _TUNE_CB), None), self._h)
            return
        keys = TUNING_KEYS + ("ms",)

        def cb(row, in_report, user):
            fn(dict(zip(keys, (float(row[i]) for i in range(8)))), bool(in_report))

        self._tune_cb = _TUNE_CB(cb)   # kept alive with the context
        _raise(_lib.asora_set_tune_progress(self._h, self._tune_cb, None), self._h)

    def save_tuning(self, path):
        """Write the autotuner results of this context to `path` (asora_tuning_save)."""
        _raise(_lib.asora_tuning_save(self._h, os.fsencode(path)), self._h)

    def load_tuning(self, path) -> int:
        """Add the autotuner results stored in `path` to this context's cache
        (asora_tuning_load); returns how many were read."""
        n = _c_int(0)
        _raise(_lib.asora_tuning_load(self._h, os.fsencode(path), ctypes.byref(n)), self._h)
        return n.value

    def record_step(self, n_H, x_HI, ijk, Q, R, gamma, dL_dgamma=None, grads=None, R_max=None,
                    store=False, accumulate=False, plain=False):
        """Record the step (forward into gamma; with dL_dgamma also the adjoint
        into grads = (dn, dx, dq)) as a HIP graph: StepGraph.launch() replays it
        on the tensors' current contents.  Runs the step once while recording."""
        ijk, Q, R, R_max, n = self._prep(n_H, x_HI, ijk, Q, R, R_max)
        self._check("gamma", gamma, torch.float32)
        dn = dx = dq = g = None
        if dL_dgamma is not None:
            g = self._check("dL_dgamma", dL_dgamma, torch.float64)
            if grads is None:
                raise AsoraError(-1, "grads = (dL/dn_H, dL/dx_HI, dL/dQ) buffers are needed with dL_dgamma")
            dn, dx, dq = grads
            self._check("dL/dn_H", dn, torch.float32)
            self._check("dL/dx_HI", dx, torch.float32)
            self._check("dL/dQ", dq, torch.float64, n)
        flags = (STORE if store else 0) | (ACCUMULATE if accumulate else 0) | (PLAIN if plain else 0)
        h = _p()
        _raise(_lib.asora_graph_create(self._h, _dptr(n_H), _dptr(x_HI), n, _dptr(ijk), _dptr(Q),
                                       _dptr(R), R_max, _dptr(gamma), _dptr(g), _dptr(dn), _dptr(dx),
                                       _dptr(dq), flags, ctypes.byref(h)), self._h)
        return StepGraph(self, h, (n_H, x_HI, ijk, Q, R, gamma, g, dn, dx, dq))

    def chemistry(self, gamma, n_H, xHI_0, dt, alpha_H, C_H=0.0, xHI_avg_prev=None, conv_rtol=1e-3,
                  stream=None):
        """Hydrogen chemistry step (library's asora_chemistry): returns
        (<x_HI>, x_HI(dt), <x_HI> as float32, n_changed or None) for the
        time-averaged rate gamma (float32) over dt seconds."""
        dev = n_H.device
        n3 = self.N ** 3
        for name, t_, dt_ in (("gamma", gamma, torch.float32), ("n_H", n_H, torch.float32),
                              ("xHI_0", xHI_0, torch.float64)):
            self._check(name, t_, dt_)
        if xHI_avg_prev is not None:
            self._check("xHI_avg_prev", xHI_avg_prev, torch.float64)
        y_avg = torch.empty(n3, dtype=torch.float64, device=dev)
        y_end = torch.empty_like(y_avg)
        y32 = torch.empty(n3, dtype=torch.float32, device=dev)
        cnt = ctypes.c_uint64(0)
        _raise(_lib.asora_chemistry(self._h, _dptr(gamma), _dptr(n_H), _dptr(xHI_0), _dptr(xHI_avg_prev),
                                    float(dt), float(alpha_H), float(C_H), float(conv_rtol), _dptr(y_avg),
                                    _dptr(y_end), _dptr(y32),
                                    ctypes.byref(cnt) if xHI_avg_prev is not None else None,
                                    _stream_ptr(stream)), self._h)
        shape = (self.N,) * 3
        return (y_avg.view(shape), y_end.view(shape), y32.view(shape),
                cnt.value if xHI_avg_prev is not None else None)

    def time_step(self, n_H, xHI_0, ijk, Q, R, dt, alpha_H, C_H=0.0, R_max=None, conv_rtol=1e-3,
                  conv_frac=1e-4, max_passes=50, fixed_passes=0, stream=None):
        """One time step of the ray-tracing <-> chemistry iteration (library's
        asora_time_step): returns (x_HI(dt), <x_HI>, gamma, passes)."""
        ijk, Q, R, R_max, n = self._prep(n_H, n_H, ijk, Q, R, R_max)
        n3 = self.N ** 3
        self._check("xHI_0", xHI_0, torch.float64)
        dev = n_H.device
        y_end = torch.empty(n3, dtype=torch.float64, device=dev)
        y_avg = torch.empty_like(y_end)
        gamma = torch.empty(n3, dtype=torch.float32, device=dev)
        passes = _c_int(0)
        _raise(_lib.asora_time_step(self._h, _dptr(n_H), _dptr(xHI_0), n, _dptr(ijk), _dptr(Q), _dptr(R), R_max,
                                    float(dt), float(alpha_H), float(C_H), float(conv_rtol), float(conv_frac),
                                    int(max_passes), int(fixed_passes), _dptr(y_end), _dptr(y_avg),
                                    _dptr(gamma), ctypes.byref(passes), _stream_ptr(stream)), self._h)
        shape = (self.N,) * 3
        return y_end.view(shape), y_avg.view(shape), gamma.view(shape), passes.value

    def store_info(self):
        """(kept, bytes_needed, bytes_allocated) of the column records."""
        v, need, alloc = _c_int(), ctypes.c_uint64(), ctypes.c_uint64()
        _raise(_lib.asora_store_info(self._h, ctypes.byref(v), ctypes.byref(need), ctypes.byref(alloc)),
               self._h)
        return bool(v.value), need.value, alloc.value

    def set_store_budget(self, nbytes: int):
        """Largest device memory for kept column records (0: half the free memory)."""
        _raise(_lib.asora_set_store_budget(self._h, int(nbytes)), self._h)

    def set_tuning(self, R_whole=0.0, R_oct=0.0, max_waves=0, pyramid_sweep=0, table_place=0,
                   adj_waves=0, adj_rate=0):
        """Scheduling parameters (0 keeps a value): pyramid_sweep 2 = shells,
        3 = layers; table_place 1 = LDS, 2 = through the caches; adj_waves
        waves per work-group of the layer adjoint; adj_rate 1 = its rate terms
        all gathered into full waves, 2 = dense chunks' in the reverse pass."""
        _raise(_lib.asora_set_tuning(self._h, float(R_whole), float(R_oct), int(max_waves),
                                     int(pyramid_sweep), int(table_place), int(adj_waves),
                                     int(adj_rate)), self._h)

    def get_tuning(self):
        """The scheduling parameters, in the order of TUNING_KEYS."""
        a, b = _c_f(), _c_f()
        ints = [_c_int() for _ in range(5)]
        _raise(_lib.asora_get_tuning(self._h, ctypes.byref(a), ctypes.byref(b),
                                     *[ctypes.byref(x) for x in ints]), self._h)
        return (a.value, b.value) + tuple(x.value for x in ints)

    def check(self, stream=None):
        """Wait for the stream; raise if a kernel flagged a source."""
        _raise(_lib.asora_check(self._h, _stream_ptr(stream)), self._h)


class StepGraph:
    """A recorded step (asora_graph_create); holds the tensors it uses."""

    def __init__(self, ctx: Asora, handle, tensors):
        self._ctx, self._h, self._tensors = ctx, handle, tensors

    def launch(self, stream=None):
        _raise(_lib.asora_graph_launch(self._h, _stream_ptr(stream)), self._ctx._h)

    def close(self):
        if getattr(self, "_h", None):
            _lib.asora_graph_free(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class _RaytraceFn(torch.autograd.Function):
    @staticmethod
    def forward(fctx, ctx: Asora, n_H, x_HI, ijk, Q, R, R_max, store):
        # the library reads the device buffers as given: pass the very tensors
        # that backward will pass, so that kept column records match them
        ijk, Qc, Rc, R_max, _ = ctx._prep(n_H, x_HI, ijk, Q.detach(), R, R_max)
        fctx.save_for_backward(n_H, x_HI, ijk, Qc, Rc if Rc is not None else torch.empty(0))
        fctx.asora, fctx.R_max, fctx.has_R = ctx, R_max, Rc is not None
        fctx.q_dtype = Q.dtype
        out = ctx.raytrace(n_H.detach(), x_HI.detach(), ijk, Qc, Rc, R_max=R_max, store=store)
        # kept records belong to this call until another forward keeps its own
        fctx.keep_gen = -1
        if store:
            ctx._keep_gen = getattr(ctx, "_keep_gen", 0) + 1
            fctx.keep_gen = ctx._keep_gen
        return out

    @staticmethod
    def backward(fctx, g):
        n_H, x_HI, ijk, Q, R = fctx.saved_tensors
        R = R if fctx.has_R else None
        kept = fctx.keep_gen == getattr(fctx.asora, "_keep_gen", 0)
        dn, dx, dq = fctx.asora.backward(n_H.detach(), x_HI.detach(), ijk, Q, R,
                                         g.double().contiguous(), R_max=fctx.R_max, store=kept)
        return None, dn, dx, None, dq.to(fctx.q_dtype), None, None, None


def raytrace(ctx: Asora, n_H, x_HI, ijk, Q, R=None, R_max=None, store=True):
    """Differentiable Gamma(n_H, x_HI, Q): backward runs the adjoint kernels.
    store=True keeps the forward's column records for the backward when they
    fit the store budget (otherwise the backward recomputes them)."""
    return _RaytraceFn.apply(ctx, n_H, x_HI, ijk, Q, R, R_max, store)
