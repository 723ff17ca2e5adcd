"""Thin Python binding of libfargo (the C ABI of include/fargo.h).

Argument marshalling only: every step of the hydrodynamics path runs in the
library's HIP kernels.  PyTorch supplies device memory (the state tensors and
the workspace) and the stream.  There is no CPU fallback: if libfargo.so has
not been built, importing this module raises ImportError.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict, Optional

import numpy as np
import torch  # loads the HIP runtime that libfargo binds to

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libfargo.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libfargo.so is not built (run __graft_entry__.build() or "
                      "python paper_1602_02359_amd/csrc/build.py)")

ABI_VERSION = 1
NGH = 3
GEOMETRY = {"cart": 0, "cyl": 1, "sph": 2}
EOS = {"iso": 0, "adi": 1}
BC = {"periodic": 0, "reflect": 1, "outflow": 2, "fixed": 3}
V0_MODE = {"minmax": 0, "mean": 1}
PRECISION = {"fp64": 0, "fp32": 1}  # fp32: FP32-bulk state, FP64 time step, split and sums
DTYPE = {"fp64": torch.float64, "fp32": torch.float32}
FIELDS = ("rho", "vx", "vy", "vz", "e", "cs", "pot", "nu")


class fargo_params(C.Structure):
    _fields_ = [
        ("abi_version", C.c_int32), ("geometry", C.c_int32),
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("xmin", C.c_double), ("xmax", C.c_double),
        ("ymin", C.POINTER(C.c_double)), ("zmin", C.POINTER(C.c_double)),
        ("eos", C.c_int32), ("gamma", C.c_double),
        ("omega", C.c_double), ("courant", C.c_double), ("cvnr", C.c_double), ("shear_c0", C.c_double),
        ("fargo", C.c_int32), ("v0_mode", C.c_int32),
        ("bc", C.c_int32 * 4), ("precision", C.c_int32), ("visc", C.c_int32),
    ]


class fargo_state(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in FIELDS]


_lib = C.CDLL(LIB_PATH)
_P = C.POINTER(fargo_params)
_S = C.POINTER(fargo_state)
_lib.fargo_abi_version.restype = C.c_int
_lib.fargo_strerror.restype = C.c_char_p
_lib.fargo_strerror.argtypes = [C.c_int]
_lib.fargo_layout.argtypes = [_P, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
_lib.fargo_workspace_bytes.argtypes = [_P, C.POINTER(C.c_size_t)]
_lib.fargo_init.argtypes = [_P, C.c_void_p, C.c_size_t, C.POINTER(C.c_void_p)]
_lib.fargo_set_vx_background.argtypes = [C.c_void_p, C.POINTER(C.c_double)]
_lib.fargo_destroy.argtypes = [C.c_void_p]
_lib.fargo_destroy.restype = None
_lib.fargo_cfl_dt.argtypes = [C.c_void_p, _S, C.POINTER(C.c_double), C.c_void_p]
_lib.fargo_step.argtypes = [C.c_void_p, _S, C.c_double, C.c_void_p]
_lib.fargo_shift.argtypes = [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
_lib.fargo_ring_split.argtypes = [C.c_void_p, C.c_void_p, C.c_double, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]
_lib.fargo_conserved_sums.argtypes = [C.c_void_p, _S, C.POINTER(C.c_double), C.c_void_p]
_lib.fargo_conserved_sums_noalloc.argtypes = [C.c_void_p, _S, C.POINTER(C.c_double), C.c_void_p]
_lib.fargo_hbm_copy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int, C.c_void_p]
_lib.fargo_hbm_streams.argtypes = [C.POINTER(C.c_void_p), C.c_int, C.POINTER(C.c_void_p), C.c_int, C.c_int, C.c_int,
                                   C.c_int, C.c_int, C.c_void_p]
_lib.fargo_get_dt.argtypes = [C.c_void_p, C.POINTER(C.c_double), C.c_void_p]
_lib.fargo_check.argtypes = [C.c_void_p]
_lib.fargo_profile_enable.argtypes = [C.c_void_p, C.c_int]
_lib.fargo_timings.argtypes = [C.c_void_p, C.POINTER(C.c_char_p), C.POINTER(C.c_int64), C.POINTER(C.c_double),
                               C.c_int, C.POINTER(C.c_int), C.c_void_p]

_lib.fargo_batch_create.argtypes = [C.POINTER(C.c_void_p), C.POINTER(fargo_state), C.c_int, C.c_int,
                                    C.POINTER(C.c_void_p)]
_lib.fargo_batch_step.argtypes = [C.c_void_p, C.c_void_p]
_lib.fargo_batch_tune.argtypes = [C.c_void_p, C.POINTER(C.c_int32), C.c_int, C.POINTER(C.c_int32), C.c_int, C.c_int,
                                  C.c_void_p, C.POINTER(C.c_int32)]
_lib.fargo_batch_chunks.argtypes = [C.c_void_p, C.POINTER(C.c_int32), C.c_int]
_lib.fargo_batch_destroy.argtypes = [C.c_void_p]
_lib.fargo_batch_destroy.restype = None


class fargo_lfc_params(C.Structure):
    _fields_ = [(n, C.c_double) for n in ("rho_s", "u_s", "r_mid", "r_span", "flux_scale", "sigma", "guard")] + \
        [("max_batch", C.c_int32)]


class fargo_lfc_views(C.Structure):
    _fields_ = [(n, C.c_void_p) for n in ("f", "h1", "h2", "o", "drho", "g3", "g2", "g1")]


LFC_NPARAM = 11010
_lib.fargo_lfc_create.argtypes = [C.c_void_p, C.POINTER(fargo_lfc_params), C.POINTER(C.c_void_p)]
_lib.fargo_lfc_destroy.argtypes = [C.c_void_p]
_lib.fargo_lfc_destroy.restype = None
for _n in ("fargo_lfc_set_params", "fargo_lfc_get_params", "fargo_lfc_get_grad"):
    getattr(_lib, _n).argtypes = [C.c_void_p, C.POINTER(C.c_float), C.c_int32]
_lib.fargo_lfc_forward.argtypes = [C.c_void_p, _S, C.c_void_p]
_lib.fargo_lfc_train_step.argtypes = [C.c_void_p, _S, C.c_void_p, C.c_double, C.c_void_p]
_lib.fargo_lfc_forward_batch.argtypes = [C.c_void_p, _S, C.c_int32, C.c_void_p]
_lib.fargo_lfc_train_batch.argtypes = [C.c_void_p, _S, C.POINTER(C.c_void_p), C.c_int32, C.c_double, C.c_void_p]
LFC_MAXB = 32
_lib.fargo_lfc_apply.argtypes = [C.c_void_p, _S, C.c_void_p]
_lib.fargo_lfc_result.argtypes = [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int32), C.c_void_p]
_lib.fargo_lfc_get_views.argtypes = [C.c_void_p, C.POINTER(fargo_lfc_views)]
_lib.fargo_lfc_restrict.argtypes = [C.c_void_p, _S, C.c_void_p, _S, C.c_void_p]
_lib.fargo_lfc_target.argtypes = [C.c_void_p, _S, _S, C.c_void_p, C.c_void_p]

EXPORTED = ("fargo_abi_version", "fargo_strerror", "fargo_layout", "fargo_workspace_bytes", "fargo_init",
            "fargo_set_vx_background", "fargo_destroy", "fargo_cfl_dt", "fargo_step", "fargo_shift", "fargo_ring_split",
            "fargo_conserved_sums", "fargo_conserved_sums_noalloc", "fargo_hbm_copy", "fargo_hbm_streams", "fargo_get_dt", "fargo_check", "fargo_profile_enable", "fargo_timings",
            "fargo_batch_create", "fargo_batch_step", "fargo_batch_tune", "fargo_batch_chunks", "fargo_batch_destroy",
            "fargo_lfc_create", "fargo_lfc_destroy", "fargo_lfc_set_params", "fargo_lfc_get_params",
            "fargo_lfc_get_grad", "fargo_lfc_forward", "fargo_lfc_forward_batch", "fargo_lfc_train_step",
            "fargo_lfc_train_batch", "fargo_lfc_apply",
            "fargo_lfc_result", "fargo_lfc_get_views", "fargo_lfc_restrict", "fargo_lfc_target")


class FargoError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__("%s: %s (%d)" % (what, _lib.fargo_strerror(code).decode(), code))
        self.code = code


def _check(rc: int, what: str):
    if rc != 0:
        raise FargoError(rc, what)


def fargo_abi_version() -> int:
    return _lib.fargo_abi_version()


def make_params(p: Dict):
    """ctypes fargo_params from a parameter dict; returns (struct, keepalive)."""
    ymin = np.ascontiguousarray(p["ymin"], dtype=np.float64)
    zmin = np.ascontiguousarray(p["zmin"], dtype=np.float64)
    s = fargo_params()
    s.abi_version = ABI_VERSION
    s.geometry = GEOMETRY[p["geometry"]]
    s.nx, s.ny, s.nz = int(p["nx"]), int(p["ny"]), int(p["nz"])
    s.xmin, s.xmax = float(p["xmin"]), float(p["xmax"])
    s.ymin = ymin.ctypes.data_as(C.POINTER(C.c_double))
    s.zmin = zmin.ctypes.data_as(C.POINTER(C.c_double))
    s.eos = EOS[p["eos"]]
    s.gamma = float(p["gamma"])
    s.omega, s.courant, s.cvnr, s.shear_c0 = float(p["omega"]), float(p["courant"]), float(p["cvnr"]), float(p["shear_c0"])
    s.fargo = int(bool(p["fargo"]))
    s.v0_mode = V0_MODE[p.get("v0_mode", "minmax")]
    for i, b in enumerate(p["bc"]):
        s.bc[i] = BC[b]
    s.precision = PRECISION[p.get("precision", "fp64")]
    s.visc = int(bool(p.get("visc", False)))
    return s, (ymin, zmin)


def fargo_layout(p: Dict):
    ps, keep = make_params(p)
    pitch, nyg, nzg = C.c_int32(), C.c_int32(), C.c_int32()
    _check(_lib.fargo_layout(C.byref(ps), C.byref(pitch), C.byref(nyg), C.byref(nzg)), "fargo_layout")
    return pitch.value, nyg.value, nzg.value


def fargo_workspace_bytes(p: Dict) -> int:
    ps, keep = make_params(p)
    n = C.c_size_t()
    _check(_lib.fargo_workspace_bytes(C.byref(ps), C.byref(n)), "fargo_workspace_bytes")
    return n.value


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


class Solver:
    """Owns a fargo context, its workspace and the device state tensors
    (padded layout [nz_g, ny_g, pitch]; float64, or float32 when
    params["precision"] == "fp32")."""

    def __init__(self, params: Dict, device: str = "cuda", workspace: bool = True):
        self.params = dict(params)
        self.device = torch.device(device)
        self.dtype = DTYPE[self.params.get("precision", "fp64")]
        self.pitch, self.nyg, self.nzg = fargo_layout(params)
        self.shape = (self.nzg, self.nyg, self.pitch)
        self._ps, self._keep = make_params(params)
        nbytes = fargo_workspace_bytes(params)
        self._ctx = C.c_void_p()
        with torch.cuda.device(self.device):
            if workspace:
                self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
                _check(_lib.fargo_init(C.byref(self._ps), C.c_void_p(self.workspace.data_ptr()), nbytes,
                                       C.byref(self._ctx)), "fargo_init")
            else:
                self.workspace = None
                _check(_lib.fargo_init(C.byref(self._ps), None, 0, C.byref(self._ctx)), "fargo_init")
        self.state: Dict[str, Optional[torch.Tensor]] = {}
        self.vxbg: Optional[np.ndarray] = None  # FP32 state: background of v_x, (nz_g, ny_g)
        self._st = fargo_state()

    def __del__(self):
        ctx = getattr(self, "_ctx", None)
        if ctx is not None and ctx.value and _lib is not None:  # _lib is None at interpreter exit
            _lib.fargo_destroy(ctx)
            self._ctx = None

    # -- state -------------------------------------------------------------
    def fargo_set_vx_background(self, vb: np.ndarray):
        """FP32-bulk contexts: the FP64 per-ring background of v_x, shape
        (nz_g, ny_g); the state's vx then holds v_x - vb."""
        vb = np.ascontiguousarray(vb, dtype=np.float64).reshape(self.nzg, self.nyg)
        _check(_lib.fargo_set_vx_background(self._ctx, vb.ctypes.data_as(C.POINTER(C.c_double))),
               "fargo_set_vx_background")
        self.vxbg = vb.copy()

    def upload(self, fields: Dict[str, Optional[np.ndarray]]):
        """Copy host arrays (nz_g, ny_g, nx) into padded device tensors of the
        state type (FP64 values are rounded to nearest for an FP32 state).
        For an FP32 state the background of v_x is each ring's mean of the
        given v_x (ghost rings included), and vx holds the rounded deviation."""
        nx = self.params["nx"]
        self.state = {}
        if self.dtype == torch.float32 and fields.get("vx") is not None:
            self.fargo_set_vx_background(np.asarray(fields["vx"], dtype=np.float64).mean(axis=2))
        for n in FIELDS:
            a = fields.get(n)
            if a is None:
                self.state[n] = None
                continue
            dt = torch.float64 if n == "pot" else self.dtype  # the potential is FP64 in every mode
            t = torch.zeros(self.shape, dtype=dt, device=self.device)
            src = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64)).to(self.device)
            if n == "vx" and self.vxbg is not None:
                src = src - torch.from_numpy(self.vxbg).to(self.device)[:, :, None]
            t[:, :, :nx] = src.to(dt)
            self.state[n] = t
        self._bind()

    def field64(self, name: str) -> torch.Tensor:
        """The device field (nz_g, ny_g, nx) as FP64, with the background of
        v_x added back for an FP32 state."""
        nx = self.params["nx"]
        t = self.state[name][:, :, :nx].double()
        if name == "vx" and self.vxbg is not None:
            t = t + torch.from_numpy(self.vxbg).to(t.device)[:, :, None]
        return t

    def _bind(self):
        for n in FIELDS:
            t = self.state.get(n)
            setattr(self._st, n, C.c_void_p(t.data_ptr()) if t is not None else None)

    def download(self) -> Dict[str, Optional[np.ndarray]]:
        """Host FP64 copies (nz_g, ny_g, nx) of the state (v_x in full)."""
        torch.cuda.synchronize(self.device)
        return {n: (None if t is None else self.field64(n).cpu().numpy().copy())
                for n, t in self.state.items()}

    # -- C ABI calls -------------------------------------------------------
    def fargo_step(self, dt: float = 0.0, stream=None):
        _check(_lib.fargo_step(self._ctx, C.byref(self._st), float(dt), _stream(stream)), "fargo_step")

    def fargo_cfl_dt(self, stream=None) -> float:
        out = C.c_double()
        _check(_lib.fargo_cfl_dt(self._ctx, C.byref(self._st), C.byref(out), _stream(stream)), "fargo_cfl_dt")
        return out.value

    def fargo_get_dt(self, stream=None) -> float:
        out = C.c_double()
        _check(_lib.fargo_get_dt(self._ctx, C.byref(out), _stream(stream)), "fargo_get_dt")
        return out.value

    def fargo_shift(self, field: torch.Tensor, nshift: torch.Tensor, stream=None):
        assert field.dtype == self.dtype and tuple(field.shape) == self.shape and field.is_contiguous()
        assert nshift.dtype == torch.int32 and nshift.numel() == self.params["ny"] * self.params["nz"]
        _check(_lib.fargo_shift(self._ctx, C.c_void_p(field.data_ptr()), C.c_void_p(nshift.data_ptr()),
                                _stream(stream)), "fargo_shift")

    def fargo_ring_split(self, vx: torch.Tensor, dt: float, stream=None):
        assert vx.dtype == self.dtype and tuple(vx.shape) == self.shape and vx.is_contiguous()
        nr = self.params["ny"] * self.params["nz"]
        v0 = torch.empty(nr, dtype=torch.float64, device=self.device)
        N = torch.empty(nr, dtype=torch.int32, device=self.device)
        xi = torch.empty(nr, dtype=torch.float64, device=self.device)
        _check(_lib.fargo_ring_split(self._ctx, C.c_void_p(vx.data_ptr()), float(dt), C.c_void_p(v0.data_ptr()),
                                     C.c_void_p(N.data_ptr()), C.c_void_p(xi.data_ptr()), _stream(stream)),
               "fargo_ring_split")
        return v0, N, xi

    def fargo_conserved_sums(self, stream=None) -> np.ndarray:
        out = (C.c_double * 5)()
        _check(_lib.fargo_conserved_sums(self._ctx, C.byref(self._st), out, _stream(stream)), "fargo_conserved_sums")
        return np.array(list(out))

    def fargo_conserved_sums_noalloc(self, stream=None) -> np.ndarray:
        out = (C.c_double * 5)()
        _check(_lib.fargo_conserved_sums_noalloc(self._ctx, C.byref(self._st), out, _stream(stream)),
               "fargo_conserved_sums_noalloc")
        return np.array(list(out))

    def fargo_check(self):
        _check(_lib.fargo_check(self._ctx), "fargo_check")

    def fargo_profile_enable(self, on: bool = True):
        _check(_lib.fargo_profile_enable(self._ctx, int(on)), "fargo_profile_enable")

    def fargo_timings(self, stream=None) -> Dict[str, tuple]:
        cap = 64
        names = (C.c_char_p * cap)()
        counts = (C.c_int64 * cap)()
        tot = (C.c_double * cap)()
        n = C.c_int()
        _check(_lib.fargo_timings(self._ctx, names, counts, tot, cap, C.byref(n), _stream(stream)), "fargo_timings")
        return {names[i].decode(): (counts[i], tot[i]) for i in range(n.value) if counts[i] > 0}


def fargo_hbm_copy(src: torch.Tensor, dst: torch.Tensor, blocks: int, stream=None):
    """The library's streaming copy (bandwidth probe) of src into dst."""
    assert src.is_contiguous() and dst.is_contiguous() and src.nbytes == dst.nbytes
    _check(_lib.fargo_hbm_copy(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), src.nbytes, int(blocks),
                               _stream(stream)), "fargo_hbm_copy")


def fargo_hbm_streams(ins, outs, nx: int, ny: int, nz: int, march: bool, stream=None):
    """The library's access-pattern probe: outs[q] = ins[q] + ins[-1] (FP64
    fields of nx * ny * nz), flat or as a column march."""
    for t in list(ins) + list(outs):
        assert t.dtype == torch.float64 and t.is_contiguous() and t.numel() == nx * ny * nz
    pi = (C.c_void_p * len(ins))(*[t.data_ptr() for t in ins])
    po = (C.c_void_p * len(outs))(*[t.data_ptr() for t in outs])
    _check(_lib.fargo_hbm_streams(pi, len(ins), po, len(outs), int(nx), int(ny), int(nz), int(bool(march)),
                                  _stream(stream)), "fargo_hbm_streams")


class Batch:
    """Many Solvers advanced together: one captured hipGraph per step
    (fargo_batch_*).  lanes >= 1: a graph of every solver's own step over that
    many streams; lanes = 0: the fused form, each kernel of the step launched
    once over all solvers.  The solvers must stay alive and keep their state
    tensors while the batch exists."""

    def __init__(self, solvers, lanes: int = 8):
        self.solvers = list(solvers)
        n = len(self.solvers)
        ctxs = (C.c_void_p * n)(*[s._ctx.value for s in self.solvers])
        sts = (fargo_state * n)(*[s._st for s in self.solvers])
        self._b = C.c_void_p()
        _check(_lib.fargo_batch_create(ctxs, sts, n, int(lanes), C.byref(self._b)), "fargo_batch_create")

    def __del__(self):
        b = getattr(self, "_b", None)
        if b is not None and b.value:
            _lib.fargo_batch_destroy(b)
            self._b = None

    def fargo_batch_step(self, stream=None):
        _check(_lib.fargo_batch_step(self._b, _stream(stream)), "fargo_batch_step")

    def fargo_batch_tune(self, lanes=(1, 2, 4, 8, 16), chunks=(16, 32, 64), steps=3, stream=None):
        la = (C.c_int32 * len(lanes))(*lanes)
        ch = (C.c_int32 * len(chunks))(*chunks)
        best = (C.c_int32 * 2)()
        _check(_lib.fargo_batch_tune(self._b, la, len(lanes), ch, len(chunks), int(steps), _stream(stream), best),
               "fargo_batch_tune")
        return int(best[0]), int(best[1])

    def chunks(self):
        out = (C.c_int32 * len(self.solvers))()
        _check(_lib.fargo_batch_chunks(self._b, out, len(self.solvers)), "fargo_batch_chunks")
        return [int(v) for v in out]


class LFC:
    """A learned flux correction bound to a 2D cylindrical FP64 Solver
    (fargo_lfc_*).  The solver must outlive it.  Batches (up to max_batch
    samples) are lists of dicts holding "rho", "vx", "vy" tensors laid out as
    the solver's own state (and "target" for training)."""

    def __init__(self, solver: Solver, rho_s: float, u_s: float, r_mid: float, r_span: float,
                 flux_scale: float, sigma: float, guard: float = 0.5, max_batch: int = 1):
        self.solver = solver
        self.max_batch = int(max_batch)
        self._p = fargo_lfc_params(rho_s, u_s, r_mid, r_span, flux_scale, sigma, guard, self.max_batch)
        self._l = C.c_void_p()
        _check(_lib.fargo_lfc_create(solver._ctx, C.byref(self._p), C.byref(self._l)), "fargo_lfc_create")
        self.nx, self.ny = solver.params["nx"], solver.params["ny"]

    def __del__(self):
        l = getattr(self, "_l", None)
        if l is not None and l.value:
            _lib.fargo_lfc_destroy(l)
            self._l = None

    def _vec(self, name: str, arr=None) -> np.ndarray:
        a = np.zeros(LFC_NPARAM, dtype=np.float32) if arr is None else np.ascontiguousarray(arr, dtype=np.float32)
        assert a.size == LFC_NPARAM
        _check(getattr(_lib, name)(self._l, a.ctypes.data_as(C.POINTER(C.c_float)), LFC_NPARAM), name)
        return a

    def set_params(self, flat: np.ndarray):
        self._vec("fargo_lfc_set_params", flat)

    def get_params(self) -> np.ndarray:
        return self._vec("fargo_lfc_get_params")

    def get_grad(self) -> np.ndarray:
        return self._vec("fargo_lfc_get_grad")

    def forward(self, stream=None):
        _check(_lib.fargo_lfc_forward(self._l, C.byref(self.solver._st), _stream(stream)), "fargo_lfc_forward")

    def train_step(self, target: torch.Tensor, lr: float, stream=None):
        assert target.dtype == torch.float64 and target.is_contiguous() and target.numel() == self.nx * self.ny
        _check(_lib.fargo_lfc_train_step(self._l, C.byref(self.solver._st), C.c_void_p(target.data_ptr()),
                                         float(lr), _stream(stream)), "fargo_lfc_train_step")

    def _states(self, samples):
        arr = (fargo_state * len(samples))()
        for i, smp in enumerate(samples):
            st = arr[i]
            for f in FIELDS:
                setattr(st, f, getattr(self.solver._st, f))
            for k in ("rho", "vx", "vy"):
                t, ref = smp[k], self.solver.state[k]
                assert t.dtype == ref.dtype and t.shape == ref.shape and t.device == ref.device and t.is_contiguous()
                setattr(st, k, C.c_void_p(t.data_ptr()))
        return arr

    def forward_batch(self, samples, stream=None):
        _check(_lib.fargo_lfc_forward_batch(self._l, self._states(samples), len(samples), _stream(stream)),
               "fargo_lfc_forward_batch")

    def train_batch(self, samples, lr: float, stream=None):
        for smp in samples:
            t = smp["target"]
            assert t.dtype == torch.float64 and t.is_contiguous() and t.numel() == self.nx * self.ny
        tg = (C.c_void_p * len(samples))(*[smp["target"].data_ptr() for smp in samples])
        _check(_lib.fargo_lfc_train_batch(self._l, self._states(samples), tg, len(samples), float(lr),
                                          _stream(stream)), "fargo_lfc_train_batch")

    def apply(self, stream=None):
        _check(_lib.fargo_lfc_apply(self._l, C.byref(self.solver._st), _stream(stream)), "fargo_lfc_apply")

    def result(self, stream=None):
        loss, skipped = C.c_double(), C.c_int32()
        _check(_lib.fargo_lfc_result(self._l, C.byref(loss), C.byref(skipped), _stream(stream)), "fargo_lfc_result")
        return loss.value, bool(skipped.value)

    def views(self, nsamp: int = 0) -> Dict[str, torch.Tensor]:
        """Device buffers of the last forward or training step as tensors
        (bfloat16 buffers as torch.bfloat16), shaped (ny, nx, channels), or
        (nsamp, ny, nx, channels) for the first nsamp samples of a batch."""
        v = fargo_lfc_views()
        _check(_lib.fargo_lfc_get_views(self._l, C.byref(v)), "fargo_lfc_get_views")
        ns = max(1, nsamp)
        n = self.nx * self.ny * ns
        dev = self.solver.device

        def wrap(ptr, count, dtype):
            # alias the library's buffer (CUDA array interface), then copy it
            code = {torch.bfloat16: "<i2", torch.float32: "<f4", torch.float64: "<f8"}[dtype]
            t = torch.as_tensor(_DevBuf(ptr, count, code), device=dev)
            t = t.clone()
            return t.view(torch.bfloat16) if dtype == torch.bfloat16 else t

        out = {}
        for name, ch, dt in (("f", 4, torch.bfloat16), ("h1", 32, torch.bfloat16), ("h2", 32, torch.bfloat16),
                             ("o", 2, torch.float32), ("drho", 1, torch.float64), ("g3", 4, torch.bfloat16),
                             ("g2", 32, torch.bfloat16), ("g1", 32, torch.bfloat16)):
            t = wrap(getattr(v, name), n * ch, dt)
            shape = ((nsamp,) if nsamp else ()) + (self.ny, self.nx) + ((ch,) if ch > 1 else ())
            out[name] = t.view(*shape)
        return out


class _DevBuf:
    """A device buffer of the library seen through the CUDA array interface."""

    def __init__(self, ptr: int, count: int, typestr: str):
        self.__cuda_array_interface__ = {"shape": (count,), "typestr": typestr, "data": (int(ptr), False),
                                         "version": 2, "strides": None}


def lfc_restrict(fine: Solver, coarse: Solver, stream=None):
    """4 x 4 conservative restriction of fine's active zones into coarse."""
    _check(_lib.fargo_lfc_restrict(fine._ctx, C.byref(fine._st), coarse._ctx, C.byref(coarse._st), _stream(stream)),
           "fargo_lfc_restrict")


def lfc_target(ref: Solver, plain: Solver, out: torch.Tensor, stream=None):
    """out[j, i] = ref.rho - plain.rho over the active zones (same mesh)."""
    assert out.dtype == torch.float64 and out.is_contiguous()
    assert out.numel() == ref.params["nx"] * ref.params["ny"]
    _check(_lib.fargo_lfc_target(ref._ctx, C.byref(ref._st), C.byref(plain._st), C.c_void_p(out.data_ptr()),
                                 _stream(stream)), "fargo_lfc_target")
