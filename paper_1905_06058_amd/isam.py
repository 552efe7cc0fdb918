"""Thin ctypes binding of libisam.so (the MI355X full-range ISAM operator and FISTA solve).

Argument marshalling only: every step of the computation runs in the library's
HIP kernels.  PyTorch supplies device memory (tensor data pointers) and the
current HIP stream.  There is no fallback: if the library is missing or no GPU
is visible, calls raise.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libisam.so")

ISAM_OK = 0
ERRORS = {
    -1: "ISAM_EINVAL", -2: "ISAM_EALIAS", -3: "ISAM_EUNSUPPORTED", -4: "ISAM_ENOMEM",
    -5: "ISAM_ENODEV", -6: "ISAM_EHIP", -7: "ISAM_ENONFINITE",
}

# Every symbol the public header declares.
EXPORTS = (
    "isam_plan", "isam_set_calibration", "isam_forward", "isam_adjoint", "isam_normal",
    "isam_lipschitz", "isam_lambda_max", "isam_fista", "isam_destroy", "isam_strerror",
    "isam_plan_dims", "isam_timing", "isam_calibration_grad",
    "isam_batch_plan", "isam_batch_offsets", "isam_batch_scan_plan", "isam_batch_set_calibration",
    "isam_batch_forward", "isam_batch_adjoint", "isam_batch_fista", "isam_batch_tune", "isam_batch_tiles",
    "isam_batch_set_tiles", "isam_batch_destroy", "isam_fista_ex", "isam_fista_state_bytes", "isam_direct",
    "isam_direct_static", "isam_plan_stolt", "isam_plan_weights", "isam_batch_set_schedule",
    "isam_batch_schedule",
)
ISAM_BATCH_NO_GRAPH = 1
SCHEDULES = ("grouped", "streams")      # ISAM_BATCH_SCHED_GROUPED, ISAM_BATCH_SCHED_STREAMS

PASS_NAMES = ("lateral_fft_fwd", "nufft_fwd", "lateral_c2r", "lateral_r2c", "nufft_adj",
              "lateral_fft_inv", "fista_update", "lateral_y", "direct")


class IsamError(RuntimeError):
    def __init__(self, code: int, what: str):
        self.code = code
        super().__init__(f"{what}: {ERRORS.get(code, code)} ({_strerror(code)})")


class Geometry(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nk", ctypes.c_int32),
        ("dx", ctypes.c_double), ("dy", ctypes.c_double),
        ("lambda_c", ctypes.c_double), ("dlambda", ctypes.c_double),
        ("waist", ctypes.c_double), ("z_focus", ctypes.c_double),
        ("a2", ctypes.c_double), ("a3", ctypes.c_double),
        ("J", ctypes.c_int32), ("osf", ctypes.c_int32), ("kb_beta", ctypes.c_double),
    ]

    def __init__(self, nx=0, ny=1, nk=0, dx=0.0, dy=0.0, lambda_c=0.0, dlambda=0.0, waist=0.0,
                 z_focus=0.0, a2=0.0, a3=0.0, J=6, osf=2, kb_beta=0.0):
        """B-scan by default (ny = 1); J = 6, 2x oversampling and the default Kaiser-Bessel
        scaling (kb_beta = 0) are the values the library implements."""
        super().__init__(nx, ny, nk, dx, dy, lambda_c, dlambda, waist, z_focus, a2, a3, J, osf, kb_beta)

    @classmethod
    def of(cls, o, **overrides) -> "Geometry":
        """From any record carrying nx, nk, dx, lambda_c, dlambda, waist, z_focus, a2, a3."""
        vals = dict(nx=o.nx, ny=getattr(o, "ny", 1), nk=o.nk, dx=o.dx, dy=getattr(o, "dy", o.dx),
                    lambda_c=o.lambda_c, dlambda=o.dlambda, waist=o.waist, z_focus=o.z_focus,
                    a2=o.a2, a3=o.a3, J=getattr(o, "J", 6), osf=getattr(o, "osf", 2),
                    kb_beta=getattr(o, "kb_beta", 0.0))
        vals.update(overrides)
        return cls(**vals)


class FistaStateRec(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("t", ctypes.c_double), ("data", ctypes.c_void_p)]


class FistaInfo(ctypes.Structure):
    _fields_ = [
        ("iters_run", ctypes.c_int32), ("status", ctypes.c_int32), ("rel_res", ctypes.c_double),
        ("resid2", ctypes.c_double), ("l1", ctypes.c_double), ("L", ctypes.c_double),
    ]


_lib = None


def load_library() -> ctypes.CDLL:
    """Load libisam.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "or python -m paper_1905_06058_amd.build")
        lib = ctypes.CDLL(LIB_PATH)
        vp, i32, dbl, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double, ctypes.c_float
        lib.isam_plan.argtypes = [ctypes.POINTER(Geometry), vp, ctypes.POINTER(vp)]
        lib.isam_set_calibration.argtypes = [vp, dbl, dbl, dbl, vp]
        lib.isam_forward.argtypes = [vp, vp, vp, vp]
        lib.isam_adjoint.argtypes = [vp, vp, vp, vp]
        lib.isam_normal.argtypes = [vp, vp, vp, vp]
        lib.isam_lipschitz.argtypes = [vp, ctypes.c_int, ctypes.c_uint64, vp, ctypes.POINTER(dbl), vp]
        lib.isam_lambda_max.argtypes = [vp, vp, vp, ctypes.POINTER(dbl), vp]
        lib.isam_fista.argtypes = [vp, vp, f32, vp, ctypes.c_int, f32, dbl, ctypes.c_int, vp,
                                   ctypes.POINTER(FistaInfo), vp]
        lib.isam_fista_ex.argtypes = [vp, vp, f32, vp, ctypes.c_int, f32, dbl, ctypes.c_int,
                                      ctypes.POINTER(FistaStateRec), ctypes.POINTER(FistaStateRec),
                                      ctypes.POINTER(dbl), vp, ctypes.POINTER(FistaInfo), vp]
        lib.isam_fista_state_bytes.argtypes = [vp, ctypes.POINTER(ctypes.c_int64)]
        lib.isam_direct.argtypes = [vp, vp, vp, vp]
        lib.isam_plan_stolt.argtypes = [vp, ctypes.c_int, vp, vp, vp]
        lib.isam_plan_weights.argtypes = [vp, vp, ctypes.c_int, vp, vp]
        lib.isam_direct_static.argtypes = [ctypes.POINTER(Geometry), vp, vp, vp]
        lib.isam_destroy.argtypes = [vp]
        lib.isam_destroy.restype = None
        lib.isam_strerror.argtypes = [ctypes.c_int]
        lib.isam_strerror.restype = ctypes.c_char_p
        lib.isam_plan_dims.argtypes = [vp, ctypes.POINTER(i32), ctypes.POINTER(i32), ctypes.POINTER(i32)]
        lib.isam_timing.argtypes = [vp, ctypes.c_int, ctypes.POINTER(dbl), ctypes.POINTER(ctypes.c_int64)]
        lib.isam_calibration_grad.argtypes = [vp, vp, vp, ctypes.POINTER(dbl), vp]
        i64p = ctypes.POINTER(ctypes.c_int64)
        i32p = ctypes.POINTER(i32)
        lib.isam_batch_plan.argtypes = [ctypes.POINTER(Geometry), ctypes.c_int, vp, ctypes.POINTER(vp)]
        lib.isam_batch_offsets.argtypes = [vp, i64p]
        lib.isam_batch_scan_plan.argtypes = [vp, ctypes.c_int, ctypes.POINTER(vp)]
        lib.isam_batch_set_calibration.argtypes = [vp, ctypes.c_int, dbl, dbl, dbl, vp]
        lib.isam_batch_forward.argtypes = [vp, vp, vp, vp]
        lib.isam_batch_adjoint.argtypes = [vp, vp, vp, vp]
        lib.isam_batch_fista.argtypes = [vp, vp, ctypes.POINTER(f32), vp, ctypes.c_int, f32, ctypes.POINTER(dbl),
                                         ctypes.c_int, ctypes.c_int, vp, ctypes.POINTER(FistaInfo), vp]
        lib.isam_batch_tune.argtypes = [vp, ctypes.c_int, vp]
        lib.isam_batch_tiles.argtypes = [vp, i32p, i32p, i32p, i32, i32p]
        lib.isam_batch_set_tiles.argtypes = [vp, i32, i32, i32]
        lib.isam_batch_set_schedule.argtypes = [vp, ctypes.c_int]
        lib.isam_batch_schedule.argtypes = [vp, ctypes.POINTER(ctypes.c_int)]
        lib.isam_batch_destroy.argtypes = [vp]
        lib.isam_batch_destroy.restype = None
        for name in EXPORTS:
            if name not in ("isam_destroy", "isam_strerror", "isam_batch_destroy"):
                getattr(lib, name).restype = ctypes.c_int
        _lib = lib
    return _lib


def _strerror(code: int) -> str:
    try:
        return load_library().isam_strerror(code).decode()
    except Exception:  # pragma: no cover - message formatting only
        return "?"


def _check(code: int, what: str) -> None:
    if code != ISAM_OK:
        raise IsamError(code, what)


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev_tensor(t: torch.Tensor, dtype, shape, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype or tuple(t.shape) != tuple(shape) or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} tensor of shape {tuple(shape)}")
    return t


@dataclass
class FistaResult:
    eta: torch.Tensor
    iters: int
    status: int
    rel_res: float
    resid2: float
    l1: float
    L: float
    history: object = None        # (iters, 3) float64 numpy array: r_r, ||A eta - y||^2, sum w|z|


class FistaState:
    """A FISTA checkpoint: iterations done, the momentum value t, and a device buffer holding
    the momentum point and last iterate (opaque layout of the plan that saved it)."""

    def __init__(self, plan: "Plan", device=None):
        nbytes = ctypes.c_int64()
        _check(plan._lib.isam_fista_state_bytes(plan._h, ctypes.byref(nbytes)), "isam_fista_state_bytes")
        self.buffer = torch.empty(int(nbytes.value), dtype=torch.uint8,
                                  device=device if device is not None else torch.device("cuda"))
        self.k = 0
        self.t = 1.0

    def _rec(self) -> FistaStateRec:
        return FistaStateRec(self.k, self.t, self.buffer.data_ptr())


class Plan:
    """An ISAM operator plan for one geometry on the current device."""

    def __init__(self, geometry, stream=None):
        lib = load_library()
        g = geometry if isinstance(geometry, Geometry) else Geometry.of(geometry)
        self.geometry = g
        self.nx, self.ny, self.nk = int(g.nx), int(g.ny), int(g.nk)
        self._h = ctypes.c_void_p()
        _check(lib.isam_plan(ctypes.byref(g), _stream(stream), ctypes.byref(self._h)), "isam_plan")
        self._lib = lib

    @property
    def shape(self):
        """(nx, nk) for a B-scan, (ny, nx, nk) for a volume."""
        return (self.nx, self.nk) if self.ny == 1 else (self.ny, self.nx, self.nk)

    def close(self) -> None:
        if getattr(self, "_h", None) and self._h.value:
            self._lib.isam_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def timing(self, enable: bool) -> dict:
        """Per-pass event timing: returns {pass: (total_ms, launches)} accumulated so far and
        then enables (clearing) or disables recording."""
        ms = (ctypes.c_double * len(PASS_NAMES))()
        cnt = (ctypes.c_int64 * len(PASS_NAMES))()
        _check(self._lib.isam_timing(self._h, int(bool(enable)), ms, cnt), "isam_timing")
        return {name: (ms[i], cnt[i]) for i, name in enumerate(PASS_NAMES)}

    def set_calibration(self, a2: float, a3: float, z_focus: float, stream=None) -> None:
        _check(self._lib.isam_set_calibration(self._h, a2, a3, z_focus, _stream(stream)),
               "isam_set_calibration")

    def forward(self, eta: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        _dev_tensor(eta, torch.complex64, self.shape, "eta")
        if out is None:
            out = torch.empty(self.shape, dtype=torch.float32, device=eta.device)
        _dev_tensor(out, torch.float32, self.shape, "out")
        _check(self._lib.isam_forward(self._h, eta.data_ptr(), out.data_ptr(), _stream(stream)),
               "isam_forward")
        return out

    def adjoint(self, r: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        _dev_tensor(r, torch.float32, self.shape, "r")
        if out is None:
            out = torch.empty(self.shape, dtype=torch.complex64, device=r.device)
        _dev_tensor(out, torch.complex64, self.shape, "out")
        _check(self._lib.isam_adjoint(self._h, r.data_ptr(), out.data_ptr(), _stream(stream)),
               "isam_adjoint")
        return out

    def normal(self, eta: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        _dev_tensor(eta, torch.complex64, self.shape, "eta")
        if out is None:
            out = torch.empty_like(eta)
        _dev_tensor(out, torch.complex64, self.shape, "out")
        _check(self._lib.isam_normal(self._h, eta.data_ptr(), out.data_ptr(), _stream(stream)),
               "isam_normal")
        return out

    def lipschitz(self, iters: int = 50, seed: int = 0, x0: torch.Tensor | None = None, stream=None) -> float:
        L = ctypes.c_double()
        ptr = None
        if x0 is not None:
            ptr = _dev_tensor(x0, torch.complex64, self.shape, "x0").data_ptr()
        _check(self._lib.isam_lipschitz(self._h, iters, seed, ptr, ctypes.byref(L), _stream(stream)),
               "isam_lipschitz")
        return L.value

    def lambda_max(self, y: torch.Tensor, w: torch.Tensor | None = None, stream=None) -> float:
        _dev_tensor(y, torch.float32, self.shape, "y")
        wp = None if w is None else _dev_tensor(w, torch.float32, self.shape, "w").data_ptr()
        out = ctypes.c_double()
        _check(self._lib.isam_lambda_max(self._h, y.data_ptr(), wp, ctypes.byref(out), _stream(stream)),
               "isam_lambda_max")
        return out.value

    def calibration_grad(self, eta: torch.Tensor, g: torch.Tensor, stream=None) -> tuple:
        """d/d(a2, a3, z_focus) of sum(g * forward(eta)) at the current calibration."""
        _dev_tensor(eta, torch.complex64, self.shape, "eta")
        _dev_tensor(g, torch.float32, self.shape, "g")
        out = (ctypes.c_double * 3)()
        _check(self._lib.isam_calibration_grad(self._h, eta.data_ptr(), g.data_ptr(), out, _stream(stream)),
               "isam_calibration_grad")
        return (out[0], out[1], out[2])

    def fista(self, y: torch.Tensor, lam: float, iters: int, w: torch.Tensor | None = None,
              tol: float = 0.0, L: float = 0.0, add_residual: bool = False,
              out: torch.Tensor | None = None, resume: "FistaState | None" = None,
              save: "FistaState | None" = None, history: bool = False, stream=None) -> FistaResult:
        """Alg. 1.  resume / save: FistaState checkpoints (save is updated in place; it may be
        the resume state); history: also return the per-iteration records."""
        _dev_tensor(y, torch.float32, self.shape, "y")
        wp = None if w is None else _dev_tensor(w, torch.float32, self.shape, "w").data_ptr()
        if out is None:
            out = torch.empty(self.shape, dtype=torch.complex64, device=y.device)
        _dev_tensor(out, torch.complex64, self.shape, "out")
        info = FistaInfo()
        if resume is None and save is None and not history:
            code = self._lib.isam_fista(self._h, y.data_ptr(), float(lam), wp, int(iters), float(tol),
                                        float(L), int(bool(add_residual)), out.data_ptr(),
                                        ctypes.byref(info), _stream(stream))
            _check(code, "isam_fista")
            return FistaResult(out, info.iters_run, info.status, info.rel_res, info.resid2, info.l1, info.L)
        rin = resume._rec() if resume is not None else None
        rout = save._rec() if save is not None else None
        hist = (ctypes.c_double * (3 * max(int(iters), 1)))() if history else None
        code = self._lib.isam_fista_ex(self._h, y.data_ptr(), float(lam), wp, int(iters), float(tol),
                                       float(L), int(bool(add_residual)),
                                       ctypes.byref(rin) if rin is not None else None,
                                       ctypes.byref(rout) if rout is not None else None,
                                       hist, out.data_ptr(), ctypes.byref(info), _stream(stream))
        _check(code, "isam_fista_ex")
        if save is not None:
            save.k, save.t = int(rout.k), float(rout.t)
        h = None
        if history:
            import numpy as np
            h = np.ctypeslib.as_array(hist)[:3 * info.iters_run].reshape(info.iters_run, 3).copy()
        return FistaResult(out, info.iters_run, info.status, info.rel_res, info.resid2, info.l1, info.L, h)

    def stolt_points(self, col: int, stream=None):
        """(floor(t), tau) of every sample of column col, as the kernels compute them."""
        fl = torch.empty(self.nk, dtype=torch.int32, device="cuda")
        tau = torch.empty(self.nk, dtype=torch.float32, device="cuda")
        _check(self._lib.isam_plan_stolt(self._h, int(col), fl.data_ptr(), tau.data_ptr(), _stream(stream)),
               "isam_plan_stolt")
        return fl, tau

    def weights(self, tau: torch.Tensor, stream=None) -> torch.Tensor:
        """The plan's min-max weight table evaluated at tau (device float32): complex64 [n][6]."""
        _dev_tensor(tau, torch.float32, tuple(tau.shape), "tau")
        n = tau.numel()
        out = torch.empty((n, 6), dtype=torch.complex64, device=tau.device)
        _check(self._lib.isam_plan_weights(self._h, tau.data_ptr(), n, out.data_ptr(), _stream(stream)),
               "isam_plan_weights")
        return out

    def direct(self, y: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """The direct IFFT image of Eq. 9 (dispersion-compensated per-A-scan transform)."""
        _dev_tensor(y, torch.float32, self.shape, "y")
        if out is None:
            out = torch.empty(self.shape, dtype=torch.complex64, device=y.device)
        _dev_tensor(out, torch.complex64, self.shape, "out")
        _check(self._lib.isam_direct(self._h, y.data_ptr(), out.data_ptr(), _stream(stream)), "isam_direct")
        return out


def direct_static(geometry, y: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """The direct image of Eq. 9 without a plan (isam_direct_static: allocates nothing on the
    device; its tables live in the library's static array, so concurrent calls on one GPU race)."""
    lib = load_library()
    g = geometry if isinstance(geometry, Geometry) else Geometry.of(geometry)
    shape = (int(g.nx), int(g.nk)) if int(g.ny) == 1 else (int(g.ny), int(g.nx), int(g.nk))
    _dev_tensor(y, torch.float32, shape, "y")
    if out is None:
        out = torch.empty(shape, dtype=torch.complex64, device=y.device)
    _dev_tensor(out, torch.complex64, shape, "out")
    _check(lib.isam_direct_static(ctypes.byref(g), y.data_ptr(), out.data_ptr(), _stream(stream)),
           "isam_direct_static")
    return out


class _BorrowedPlan(Plan):
    """A scan's plan inside a batch (owned by the batch)."""

    def __init__(self, handle, geometry, batch):
        self._lib = load_library()
        self._h = handle
        self.geometry = geometry
        self.nx, self.ny, self.nk = int(geometry.nx), int(geometry.ny), int(geometry.nk)
        self._batch = batch            # keeps the batch alive

    def close(self) -> None:
        self._h = ctypes.c_void_p()


class Batch:
    """Many B-scans of uneven size run together (one launch per pass per group of scans).

    Packed device buffers hold scan i at elements [offsets[i], offsets[i+1]), each scan
    row-major [nx_i][nk_i]: complex64 objects, float32 spectra.
    """

    def __init__(self, geometries, stream=None):
        lib = load_library()
        gs = [g if isinstance(g, Geometry) else Geometry.of(g) for g in geometries]
        arr = (Geometry * len(gs))(*gs)
        self.geometries = gs
        self.n = len(gs)
        self._h = ctypes.c_void_p()
        _check(lib.isam_batch_plan(arr, self.n, _stream(stream), ctypes.byref(self._h)), "isam_batch_plan")
        self._lib = lib
        off = (ctypes.c_int64 * (self.n + 1))()
        _check(lib.isam_batch_offsets(self._h, off), "isam_batch_offsets")
        self.offsets = [int(v) for v in off]
        self.total = self.offsets[-1]

    def close(self) -> None:
        if getattr(self, "_h", None) and self._h.value:
            self._lib.isam_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):  # pragma: no cover
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def scan(self, t: torch.Tensor, i: int) -> torch.Tensor:
        """View of scan i in a packed buffer, shaped [nx_i][nk_i]."""
        g = self.geometries[i]
        return t[self.offsets[i]:self.offsets[i + 1]].view(int(g.nx), int(g.nk))

    def plan(self, i: int) -> Plan:
        h = ctypes.c_void_p()
        _check(self._lib.isam_batch_scan_plan(self._h, i, ctypes.byref(h)), "isam_batch_scan_plan")
        return _BorrowedPlan(h, self.geometries[i], self)

    def set_calibration(self, i: int, a2: float, a3: float, z_focus: float, stream=None) -> None:
        _check(self._lib.isam_batch_set_calibration(self._h, i, a2, a3, z_focus, _stream(stream)),
               "isam_batch_set_calibration")

    def forward(self, eta: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        _dev_tensor(eta, torch.complex64, (self.total,), "eta")
        if out is None:
            out = torch.empty(self.total, dtype=torch.float32, device=eta.device)
        _dev_tensor(out, torch.float32, (self.total,), "out")
        _check(self._lib.isam_batch_forward(self._h, eta.data_ptr(), out.data_ptr(), _stream(stream)),
               "isam_batch_forward")
        return out

    def adjoint(self, r: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        _dev_tensor(r, torch.float32, (self.total,), "r")
        if out is None:
            out = torch.empty(self.total, dtype=torch.complex64, device=r.device)
        _dev_tensor(out, torch.complex64, (self.total,), "out")
        _check(self._lib.isam_batch_adjoint(self._h, r.data_ptr(), out.data_ptr(), _stream(stream)),
               "isam_batch_adjoint")
        return out

    def fista(self, y: torch.Tensor, lam, iters: int, w: torch.Tensor | None = None, tol: float = 0.0,
              L=None, add_residual: bool = False, graph: bool = True, out: torch.Tensor | None = None,
              stream=None):
        """Returns (eta_packed, [FistaInfo per scan])."""
        _dev_tensor(y, torch.float32, (self.total,), "y")
        wp = None if w is None else _dev_tensor(w, torch.float32, (self.total,), "w").data_ptr()
        if out is None:
            out = torch.empty(self.total, dtype=torch.complex64, device=y.device)
        _dev_tensor(out, torch.complex64, (self.total,), "out")
        lam_a = (ctypes.c_float * self.n)(*[float(v) for v in lam])
        L_a = None if L is None else (ctypes.c_double * self.n)(*[float(v) for v in L])
        info = (FistaInfo * self.n)()
        code = self._lib.isam_batch_fista(self._h, y.data_ptr(), lam_a, wp, int(iters), float(tol), L_a,
                                          int(bool(add_residual)), 0 if graph else ISAM_BATCH_NO_GRAPH,
                                          out.data_ptr(), info, _stream(stream))
        _check(code, "isam_batch_fista")
        return out, list(info)

    def tune(self, reps: int = 10, stream=None) -> dict:
        _check(self._lib.isam_batch_tune(self._h, int(reps), _stream(stream)), "isam_batch_tune")
        return self.tiles()

    def tiles(self) -> dict:
        """{nx: (lanes of complex passes, lanes of real passes)} per lateral group."""
        ng = ctypes.c_int32()
        cap = 64
        nx, c, r = (ctypes.c_int32 * cap)(), (ctypes.c_int32 * cap)(), (ctypes.c_int32 * cap)()
        _check(self._lib.isam_batch_tiles(self._h, nx, c, r, cap, ctypes.byref(ng)), "isam_batch_tiles")
        return {int(nx[i]): (int(c[i]), int(r[i])) for i in range(min(ng.value, cap))}

    def schedule(self) -> str:
        """FISTA schedule in use: "grouped" (one launch per pass per group of scans, replayed
        graph) or "streams" (each scan's own solve, scans spread over the batch's streams)."""
        v = ctypes.c_int()
        _check(self._lib.isam_batch_schedule(self._h, ctypes.byref(v)), "isam_batch_schedule")
        return SCHEDULES[v.value]

    def set_schedule(self, name: str) -> None:
        if name not in SCHEDULES:
            raise ValueError(f"schedule must be one of {SCHEDULES}")
        _check(self._lib.isam_batch_set_schedule(self._h, SCHEDULES.index(name)), "isam_batch_set_schedule")

    def set_tiles(self, nx: int, lanes_complex: int, lanes_real: int) -> None:
        _check(self._lib.isam_batch_set_tiles(self._h, int(nx), int(lanes_complex), int(lanes_real)),
               "isam_batch_set_tiles")
