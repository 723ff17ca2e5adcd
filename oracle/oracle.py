"""ctypes binding of the FP64 CPU oracle (test infrastructure only).

Arrays are numpy float64, C-contiguous, shape (nz_g, ny_g, nx) with ghosts;
they are updated in place.  Parameters are the plain dicts built by the input
generators (`paper_1602_02359_amd.workloads`).
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Optional

import numpy as np

from . import build as _build

_GEO = {"cart": 0, "cyl": 1, "sph": 2}
_EOS = {"iso": 0, "adi": 1}
_BC = {"periodic": 0, "reflect": 1, "outflow": 2, "fixed": 3}

ERRORS = {0: "ok", -1: "invalid argument", -2: "out of memory", -4: "non-finite state", -5: "bad time step"}


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__("oracle error %d (%s)" % (code, ERRORS.get(code, "?")))
        self.code = code


class _Params(C.Structure):
    _fields_ = [
        ("geometry", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("xmin", C.c_double), ("xmax", C.c_double),
        ("ymin", C.POINTER(C.c_double)), ("zmin", C.POINTER(C.c_double)),
        ("eos", C.c_int32), ("gamma", C.c_double),
        ("omega", C.c_double), ("courant", C.c_double), ("cvnr", C.c_double), ("shear_c0", C.c_double),
        ("fargo", C.c_int32), ("v0_mean", C.c_int32),
        ("bc", C.c_int32 * 4), ("visc", C.c_int32),
    ]


class _State(C.Structure):
    _fields_ = [(n, C.POINTER(C.c_double)) for n in ("rho", "vx", "vy", "vz", "e", "cs", "pot", "nu")]


_lib = None
_path = None  # the library to load (default: the portable build)


def use_native():
    """Load the copy built with -march=native on this host (built here if
    missing) instead of the portable one; for timing.  Same bits: no
    contraction, no fast-math.  Must be called before the first oracle call."""
    global _path
    if _lib is not None:
        raise RuntimeError("the oracle library is already loaded")
    _build.build(native=True)
    _path = _build.LIB_NATIVE


def lib():
    global _lib
    if _lib is None:
        path = _path or _build.LIB
        if not os.path.exists(path):
            _build.build()
        L = C.CDLL(path)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        P = C.POINTER(_Params)
        S = C.POINTER(_State)
        L.orc_step.argtypes = [P, S, C.c_double, dp]
        L.orc_cfl_dt.argtypes = [P, S, dp]
        L.orc_ring_split.argtypes = [P, dp, C.c_double, dp, ip, dp]
        L.orc_shift.argtypes = [P, dp, ip]
        L.orc_sums.argtypes = [P, S, dp, dp]
        L.orc_geometry.argtypes = [P, dp, dp, dp, dp, dp]
        L.orc_sweep_line.argtypes = [C.c_int, C.c_int, dp, C.POINTER(dp), dp, dp, dp, dp, dp, C.c_double]
        L.orc_sweep_line.restype = None
        L.orc_ppa_faces.argtypes = [C.c_int, dp, C.c_double, dp]
        L.orc_ppa_faces.restype = None
        L.orc_ppa_ring.argtypes = [C.c_int, C.c_int, dp, C.POINTER(dp), C.c_double, C.c_double, C.c_double, C.c_double]
        L.orc_ppa_ring.restype = None
        L.orc_split_shift.argtypes = [C.c_double, C.c_double, C.c_double, ip, dp]
        L.orc_split_shift.restype = None
        L.orc_num_threads.restype = C.c_int
        L.orc_set_num_threads.argtypes = [C.c_int]
        L.orc_set_num_threads.restype = None
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _params(p: Dict):
    ymin = np.ascontiguousarray(p["ymin"], dtype=np.float64)
    zmin = np.ascontiguousarray(p["zmin"], dtype=np.float64)
    s = _Params()
    s.geometry = _GEO[p["geometry"]]
    s.nx, s.ny, s.nz = int(p["nx"]), int(p["ny"]), int(p["nz"])
    s.xmin, s.xmax = float(p["xmin"]), float(p["xmax"])
    s.ymin, s.zmin = _ptr(ymin), _ptr(zmin)
    s.eos = _EOS[p["eos"]]
    s.gamma = float(p["gamma"])
    s.omega, s.courant, s.cvnr, s.shear_c0 = float(p["omega"]), float(p["courant"]), float(p["cvnr"]), float(p["shear_c0"])
    s.fargo = int(bool(p["fargo"]))
    s.v0_mean = int(p.get("v0_mode", "minmax") == "mean")
    for i, b in enumerate(p["bc"]):
        s.bc[i] = _BC[b]
    s.visc = int(bool(p.get("visc", False)))
    return s, (ymin, zmin)


def _state(f: Dict):
    s = _State()
    for n in ("rho", "vx", "vy", "vz", "e", "cs", "pot", "nu"):
        a = f.get(n)
        setattr(s, n, _ptr(a))
    return s


def _check(rc: int):
    if rc != 0:
        raise OracleError(rc)


def step(p: Dict, f: Dict, dt: float = 0.0) -> float:
    """One full update in place; dt > 0 imposes the step.  Returns the dt used."""
    ps, keep = _params(p)
    st = _state(f)
    out = C.c_double(0.0)
    _check(lib().orc_step(C.byref(ps), C.byref(st), float(dt), C.byref(out)))
    return out.value


def cfl_dt(p: Dict, f: Dict) -> float:
    """Boundary fill of the ghosts (in place) and the time step of Eq. cfl2."""
    ps, keep = _params(p)
    st = _state(f)
    out = C.c_double(0.0)
    _check(lib().orc_cfl_dt(C.byref(ps), C.byref(st), C.byref(out)))
    return out.value


def ring_split(p: Dict, vx: np.ndarray, dt: float):
    """(v0, N, xi) per active ring, arrays of shape (nz, ny)."""
    ps, keep = _params(p)
    nz, ny = p["nz"], p["ny"]
    v0 = np.zeros((nz, ny))
    N = np.zeros((nz, ny), dtype=np.int32)
    xi = np.zeros((nz, ny))
    _check(lib().orc_ring_split(C.byref(ps), _ptr(vx), float(dt), _ptr(v0),
                                N.ctypes.data_as(C.POINTER(C.c_int32)), _ptr(xi)))
    return v0, N, xi


def shift(p: Dict, field: np.ndarray, N: np.ndarray):
    ps, keep = _params(p)
    N = np.ascontiguousarray(N, dtype=np.int32)
    _check(lib().orc_shift(C.byref(ps), _ptr(field), N.ctypes.data_as(C.POINTER(C.c_int32))))


def sums(p: Dict, f: Dict):
    """(sums[5], abs_sums[5]): mass, X/Y/Z momenta, internal energy."""
    ps, keep = _params(p)
    st = _state(f)
    out = np.zeros(5)
    aout = np.zeros(5)
    _check(lib().orc_sums(C.byref(ps), C.byref(st), _ptr(out), _ptr(aout)))
    return out, aout


def geometry(p: Dict):
    """Per-(k, j) volume, S_x, S_y, S_z and azimuthal length, shape (nz_g, ny_g)."""
    ps, keep = _params(p)
    nzg = p["nz"] + 6 if p["nz"] > 1 else 1
    nyg = p["ny"] + 6
    out = [np.zeros((nzg, nyg)) for _ in range(5)]
    _check(lib().orc_geometry(C.byref(ps), *[_ptr(a) for a in out]))
    return dict(vol=out[0], sx=out[1], sy=out[2], sz=out[3], dxlen=out[4])


def sweep_line(rho, Q, w, L, h, S, Vi, dt):
    """Directional update of one line (see the C source for the index layout).
    rho and every array of Q (length n+4) are updated in place."""
    n = len(Vi)
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in Q]
    QP = (C.POINTER(C.c_double) * max(1, len(arrs)))(*[_ptr(a) for a in arrs])
    lib().orc_sweep_line(n, len(arrs), _ptr(rho), QP, _ptr(w), _ptr(L), _ptr(h), _ptr(S), _ptr(Vi), float(dt))
    return arrs


def ppa_faces(q: np.ndarray, xi: float) -> np.ndarray:
    q = np.ascontiguousarray(q, dtype=np.float64)
    out = np.zeros_like(q)
    lib().orc_ppa_faces(len(q), _ptr(q), float(xi), _ptr(out))
    return out


def ppa_ring(rho, Q, xi, dX, S, vinv):
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in Q]
    QP = (C.POINTER(C.c_double) * max(1, len(arrs)))(*[_ptr(a) for a in arrs])
    lib().orc_ppa_ring(len(rho), len(arrs), _ptr(rho), QP, float(xi), float(dX), float(S), float(vinv))
    return arrs


def split_shift(v0: float, dt: float, dX: float):
    N = C.c_int32(0)
    xi = C.c_double(0.0)
    lib().orc_split_shift(float(v0), float(dt), float(dX), C.byref(N), C.byref(xi))
    return N.value, xi.value


def num_threads() -> int:
    return lib().orc_num_threads()


def set_num_threads(n: int):
    lib().orc_set_num_threads(int(n))
