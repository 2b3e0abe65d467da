"""The C-ABI library: loads, exports every entry point of include/asora.h,
validates arguments before touching a device, and builds tables on the host
that agree with the oracle's independent quadrature.  No GPU needed."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "asora.h")).read()
    return sorted(set(re.findall(r"^(?:asora_status|const char \*|int64_t)\s*(asora_\w+)\(", txt, re.M)))


@pytest.fixture(scope="module")
def pkg():
    import paper_2311_01492_amd as asora
    return asora


def test_exports_every_declared_symbol(pkg):
    names = _declared()
    assert len(names) >= 8
    lib = ctypes.CDLL(pkg.lib_path())
    for n in names:
        assert hasattr(lib, n), n


def test_max_sources_fits_the_work_item_numbering(pkg):
    """The kernels number (source, piece) work items in 32-bit integers, up to
    24 pieces per source: the accepted source count keeps them in range."""
    n = pkg.max_sources()
    assert n * 24 <= 2 ** 31 - 1 < (n + 1) * 24
    assert n >= 1_000_000   # the million-source workload fits one call
    assert "asora_max_sources" in _declared()


def test_table_blackbody_matches_oracle(pkg):
    P, dP = pkg.table_blackbody(5e4, 2.8, 2000, -20.0, 4.0)
    tb = oracle.blackbody_table()
    np.testing.assert_allclose(P, tb.P, rtol=1e-10, atol=0)
    np.testing.assert_allclose(dP, tb.dP, rtol=1e-10, atol=0)


def test_table_blackbody_heat_matches_oracle(pkg):
    """The photo-heating table (eV) against the oracle's quadrature, on a
    coarser node grid (the oracle's adaptive quadrature takes ~0.3 s per
    hundred nodes)."""
    H, dH = pkg.table_blackbody_heat(5e4, 2.8, 200, -20.0, 4.0)
    th = oracle.blackbody_heat_table(n=200)
    np.testing.assert_allclose(H, th.P, rtol=1e-10, atol=0)
    np.testing.assert_allclose(dH, th.dP, rtol=1e-10, atol=0)
    with pytest.raises(pkg.AsoraError):
        pkg.table_blackbody_heat(0.0)


def test_table_blackbody_band_matches_oracle(pkg):
    """The band tables of the two-absorber sweep against the oracle's
    quadrature (coarse node grids: the oracle's adaptive quadrature is slow)."""
    for lo, hi, lg_hi in ((13.6, 24.59, 2.5), (35.0, 54.42, 2.3), (54.42, math.inf, 3.3)):
        P, dP = pkg.table_blackbody_band(lo, hi, n=120, lg_hi=lg_hi)
        t = oracle.blackbody_band_table(lo, hi, n=120, lg_hi=lg_hi)
        np.testing.assert_allclose(P, t.P, rtol=1e-10, atol=0)
        np.testing.assert_allclose(dP, t.dP, rtol=1e-10, atol=0)
    with pytest.raises(pkg.AsoraError):
        pkg.table_blackbody_band(10.0, 20.0)


def test_table_grey(pkg):
    P, dP = pkg.table_grey(500, -20.0, math.log10(80.0))
    tau = 10 ** np.linspace(-20, math.log10(80.0), 500)
    # node positions agree to a few ulp of log10 tau, i.e. ~tau*1e-15 in ln P
    np.testing.assert_allclose(P, np.exp(-tau), rtol=1e-12)
    np.testing.assert_allclose(dP, -np.exp(-tau), rtol=1e-12)


def test_table_argument_errors(pkg):
    with pytest.raises(pkg.AsoraError) as e:
        pkg.table_blackbody(-1.0)
    assert e.value.status == -1


def _init(pkg, **kw):
    lib = ctypes.CDLL(pkg.lib_path())
    lib.asora_init.restype = ctypes.c_int
    lib.asora_init.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int, ctypes.c_double,
                               ctypes.c_double, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double, ctypes.c_uint32,
                               ctypes.c_int]
    lib.asora_last_error.restype = ctypes.c_char_p
    P, dP = pkg.table_blackbody(5e4, 2.8, 64, -20.0, 4.0)
    a = dict(N=16, cell=4.3e24, sig=6.3e-18, lo=-20.0, hi=4.0, n=64, P=P, dP=dP, tw=0.6, flags=0, dev=0)
    a.update(kw)
    h = ctypes.c_void_p()
    st = lib.asora_init(ctypes.byref(h), a["N"], a["cell"], a["sig"], a["lo"], a["hi"], a["n"],
                        a["P"].ctypes.data_as(ctypes.c_void_p), a["dP"].ctypes.data_as(ctypes.c_void_p),
                        a["tw"], a["flags"], a["dev"])
    return st, lib.asora_last_error(None).decode()


@pytest.mark.parametrize("kw,frag", [
    (dict(N=0), "N=0"),
    (dict(cell=-1.0), "cell size"),
    (dict(sig=0.0), "sigma0"),
    (dict(lo=4.0, hi=-20.0), "lo < hi"),
    (dict(n=1), "n_tab"),
    (dict(tw=-1.0), "tau_weight_floor"),
    (dict(flags=0x80), "unknown flags"),
    (dict(P=np.linspace(1, 2, 64)), "node"),
    (dict(P=np.full(64, 1e-40)), "node"),
])
def test_init_rejects_bad_arguments(pkg, kw, frag):
    st, msg = _init(pkg, **kw)
    assert st == -1 and frag in msg


def test_free_null_is_ok(pkg):
    lib = ctypes.CDLL(pkg.lib_path())
    lib.asora_free.restype = ctypes.c_int
    lib.asora_free.argtypes = [ctypes.c_void_p]
    assert lib.asora_free(None) == 0
