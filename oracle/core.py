"""ctypes wrappers for the plain-C oracle (test infrastructure only)."""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fe_oracle.c")
_LIB = os.path.join(_HERE, "libfe_oracle.so")
_lib = None


def build_oracle(force: bool = True) -> str:
    """Compile the oracle with gcc (plain C, OpenMP over element slabs)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        cmd = ["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", "-std=c11", "-Wall",
               "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build_oracle()
        _lib = ctypes.CDLL(_LIB)
    return _lib


_d = ctypes.POINTER(ctypes.c_double)
_u8 = ctypes.POINTER(ctypes.c_uint8)


def _dp(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_d)


def _mp(m):
    if m is None:
        return None
    assert m.dtype == np.uint8 and m.flags.c_contiguous
    return m.ctypes.data_as(_u8)


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def _u8c(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.uint8)


def _grid(p):
    return ctypes.c_int(p.nx), ctypes.c_int(p.ny), ctypes.c_int(p.nz), ctypes.c_double(p.h)


def residual(p, x, gamma=None, mask="walls", forcing=None, s=None):
    """R(x; gamma) with prescribed rows zeroed.  ``mask`` is an array, 'walls', 'solve' or None."""
    lib = _load()
    m = _mask(p, mask)
    g = _f64(p.gamma if gamma is None else gamma)
    ss = _f64(p.s if s is None else s)
    x = _f64(x)
    fo = _f64(forcing)
    r = np.empty(p.n_dof)
    lib.or_residual(*_grid(p), _dp(p.phys()), _mp(m), _dp(x), _dp(g), _dp(ss), _dp(fo), _dp(r))
    return r


def jvp(p, x, v, gamma=None, mask="walls", forcing=None, s=None):
    lib = _load()
    m = _mask(p, mask)
    g = _f64(p.gamma if gamma is None else gamma)
    ss = _f64(p.s if s is None else s)
    x, v, fo = _f64(x), _f64(v), _f64(forcing)
    out = np.empty(p.n_dof)
    lib.or_jvp(*_grid(p), _dp(p.phys()), _mp(m), _dp(x), _dp(g), _dp(ss), _dp(fo), _dp(v), _dp(out))
    return out


def jtvp(p, x, w, gamma=None, mask="walls", forcing=None, s=None):
    lib = _load()
    m = _mask(p, mask)
    g = _f64(p.gamma if gamma is None else gamma)
    ss = _f64(p.s if s is None else s)
    x, w, fo = _f64(x), _f64(w), _f64(forcing)
    out = np.empty(p.n_dof)
    lib.or_jtvp(*_grid(p), _dp(p.phys()), _mp(m), _dp(x), _dp(g), _dp(ss), _dp(fo), _dp(w), _dp(out))
    return out


def dR_dgamma(p, x, lam, gamma=None, mask="walls", s=None):
    """g_e = lambda^T dR/dgamma_e."""
    lib = _load()
    m = _mask(p, mask)
    g = _f64(p.gamma if gamma is None else gamma)
    ss = _f64(p.s if s is None else s)
    x, lam = _f64(x), _f64(lam)
    out = np.empty(p.n_el)
    lib.or_dRdgamma(*_grid(p), _dp(p.phys()), _mp(m), _dp(x), _dp(g), _dp(ss), _dp(lam), _dp(out))
    return out


def element_jacobians(p, x, gamma=None, forcing=None, s=None):
    """Raw element Jacobians [n_el, 40, 40] (row/col = 5*local_node + field)."""
    lib = _load()
    g = _f64(p.gamma if gamma is None else gamma)
    ss = _f64(p.s if s is None else s)
    x, fo = _f64(x), _f64(forcing)
    out = np.empty((p.n_el, 40, 40))
    lib.or_element_jacobians(*_grid(p), _dp(p.phys()), _dp(x), _dp(g), _dp(ss), _dp(fo), _dp(out))
    return out


def element_residual(h, phys, xe, gamma, s=0.0):
    lib = _load()
    xe = _f64(np.asarray(xe).reshape(40))
    out = np.empty(40)
    lib.or_element_residual(ctypes.c_double(h), _dp(_f64(phys)), _dp(xe), ctypes.c_double(gamma),
                            ctypes.c_double(s), _dp(out))
    return out


def element_dR_dgamma(h, phys, xe, gamma, s=0.0):
    lib = _load()
    xe = _f64(np.asarray(xe).reshape(40))
    out = np.empty(40)
    lib.or_element_dRdgamma(ctypes.c_double(h), _dp(_f64(phys)), _dp(xe), ctypes.c_double(gamma),
                            ctypes.c_double(s), _dp(out))
    return out


def material(phys, gamma):
    """(alpha, K, dalpha/dgamma, dK/dgamma) at each gamma."""
    lib = _load()
    g = _f64(np.atleast_1d(gamma))
    a, K, da, dK = (np.empty_like(g) for _ in range(4))
    lib.or_material(_dp(_f64(phys)), ctypes.c_int(g.size), _dp(g), _dp(a), _dp(K), _dp(da), _dp(dK))
    return a, K, da, dK


def taus(h, phys, U2, alpha, K):
    lib = _load()
    out = np.empty(2)
    lib.or_taus(ctypes.c_double(h), _dp(_f64(phys)), ctypes.c_double(U2), ctypes.c_double(alpha),
                ctypes.c_double(K), _dp(out))
    return float(out[0]), float(out[1])


def gauss_points(p):
    lib = _load()
    out = np.empty((p.n_el, 8, 3))
    lib.or_gauss_points(*_grid(p), _dp(out))
    return out


def num_threads() -> int:
    return int(_load().or_num_threads())


def set_num_threads(n: int) -> None:
    """OpenMP threads of the oracle's element loops (timing only)."""
    L = _load()
    L.or_set_num_threads.argtypes = [ctypes.c_int]
    L.or_set_num_threads.restype = None
    L.or_set_num_threads(int(n))


def set_frozen_tau(on: bool) -> None:
    """Test-only: drop the variations of tau and tauT from every derivative
    (the comparison at the end of the appendix "Stabilisation parameters")."""
    L = _load()
    L.or_set_frozen_tau.argtypes = [ctypes.c_int]
    L.or_set_frozen_tau.restype = None
    L.or_set_frozen_tau(1 if on else 0)


def _mask(p, mask):
    if mask is None:
        return None
    if isinstance(mask, str):
        if mask == "walls":
            return _u8c(p.mask_walls)
        if mask == "solve":
            return _u8c(p.mask_solve)
        raise ValueError(mask)
    return _u8c(mask)
