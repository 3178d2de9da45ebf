"""Thin Python binding of the C ABI in include/hmg.h (argument marshalling only).

Every method forwards to the ``hmg_*`` entry point of the same name; PyTorch
provides the device buffers and the stream.  Fields of the six load cases are
``(6, 3, n)`` tensors ("case-major SoA"); scalar fields are ``(n,)`` float32.
"""
from __future__ import annotations

import ctypes
from dataclasses import dataclass

import numpy as np
import torch

from . import _lib

OK, E_INVALID, E_OOM, E_DEVICE, E_NOT_CONVERGED, E_STATE = range(6)
KERNELS = {"matvec": 0, "residual": 1, "post_smooth": 2, "update": 3, "true_residual": 4,
           "jacobi": 5, "gs_forward": 6, "gs_backward": 7, "prolong": 8}
PRECISIONS = {"fp64": 0, "fp32": 1, "mixed_bf16": 2, "mixed_bf16_stencil": 4}
SMOOTHERS = {"jacobi": 0, "gs": 1}
SYMMETRIES = {"reflect3": 0, "reflect6": 1, "rotate3": 2}
OBJECTIVES = {"bulk": 0, "shear": 1, "poisson_relaxed": 2, "poisson_log": 3}


def _dbl(values):
    a = np.ascontiguousarray(values, dtype=np.float64).ravel()
    return (ctypes.c_double * a.size)(*a.tolist())


def objective(kind: str, C, iteration: int = 0, params=None):
    """hmg_objective: (F, W = dF/dC^H) of one of the objectives (host only)."""
    lib = _lib.load()
    F = ctypes.c_double()
    W = (ctypes.c_double * 36)()
    st = lib.hmg_objective(OBJECTIVES[kind], _dbl(C), int(iteration),
                           _dbl(params) if params is not None else None, ctypes.byref(F), W)
    if st != OK:
        raise HmgError(st, f"hmg_objective({kind}) failed")
    return F.value, np.array(W[:]).reshape(6, 6)


def should_stop(history, rel_change=5e-4, window=3, max_iter=300) -> bool:
    """hmg_should_stop: the stopping rule on an objective history (host only)."""
    lib = _lib.load()
    h = np.ascontiguousarray(history, dtype=np.float64)
    out = ctypes.c_int32()
    st = lib.hmg_should_stop(_dbl(h) if h.size else None, int(h.size), rel_change, window,
                             max_iter, ctypes.byref(out))
    if st != OK:
        raise HmgError(st, "hmg_should_stop failed")
    return bool(out.value)


class HmgError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"hmg status {status}: {message}")
        self.status = status


@dataclass
class SolveResult:
    iters: np.ndarray      # PCG iterations per case
    relres: np.ndarray     # recomputed ||f - K u|| / ||f|| per case
    converged: bool


def _ptr(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


class Context:
    """One periodic cell on the current GPU (``hmg_create`` / ``hmg_destroy``)."""

    def __init__(self, shape, *, E0=1.0, nu=0.3, penal=3.0, Emin=1e-9, levels=0, omega=0.0,
                 precision="fp32", replace_every=None, smoother="jacobi", post_fp16=False,
                 nondyadic=False, stream: torch.cuda.Stream | None = None):
        self.lib = _lib.load()
        nx, ny, nz = (int(v) for v in shape)
        self.shape = (nx, ny, nz)
        self.n = nx * ny * nz
        self.precision = precision
        self.field_dtype = torch.float64 if precision == "fp64" else torch.float32
        self.device = torch.device("cuda", torch.cuda.current_device())
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        if replace_every is None:  # the mixed form recomputes r in FP64 every 20 iterations
            replace_every = 20 if precision.startswith("mixed") else 0
        cfg = _lib.HmgConfig(nx, ny, nz, E0, nu, penal, Emin, levels, omega, 1, 1,
                             PRECISIONS[precision], replace_every, SMOOTHERS[smoother],
                             int(bool(post_fp16)), int(bool(nondyadic)))
        self.config = cfg
        handle = ctypes.c_void_p()
        st = self.lib.hmg_create(ctypes.byref(cfg), ctypes.c_void_p(self.stream.cuda_stream),
                                 ctypes.byref(handle))
        if st != OK:
            raise HmgError(st, "hmg_create failed (see stderr)")
        self._h = handle

    # -- helpers ----------------------------------------------------------------------------
    def _check(self, st: int, allow=(OK,)):
        if st not in allow:
            msg = self.lib.hmg_last_error(self._h).decode()
            raise HmgError(st, msg)
        return st

    def _field(self, t: torch.Tensor, n: int | None = None, name="field") -> torch.Tensor:
        n = self.n if n is None else n
        if t.device != self.device or t.dtype != self.field_dtype or not t.is_contiguous() \
                or t.numel() != 18 * n:
            raise ValueError(f"{name} must be a contiguous {self.field_dtype} tensor on "
                             f"{self.device} with 6*3*{n} elements")
        return t

    def _scalar(self, t: torch.Tensor, name="array") -> torch.Tensor:
        if t.device != self.device or t.dtype != torch.float32 or not t.is_contiguous() \
                or t.numel() != self.n:
            raise ValueError(f"{name} must be a contiguous float32 tensor on {self.device} with n elements")
        return t

    def new_field(self, level: int = 0) -> torch.Tensor:
        n = int(np.prod(self.level_dims(level)))
        return torch.empty((6, 3, n), dtype=self.field_dtype, device=self.device)

    # -- entry points ---------------------------------------------------------------------
    def destroy(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self.lib.hmg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def set_density(self, rho: torch.Tensor):
        self._check(self.lib.hmg_set_density(self._h, _ptr(self._scalar(rho, "rho"))))

    def solve_cases(self, rel_tol: float, max_iter: int, init: int = 0,
                    u0: torch.Tensor | None = None) -> SolveResult:
        it = (ctypes.c_int32 * 6)()
        rr = (ctypes.c_double * 6)()
        u0p = _ptr(self._field(u0, name="u0")) if u0 is not None else ctypes.c_void_p()
        st = self.lib.hmg_solve_cases(self._h, rel_tol, max_iter, init, u0p, it, rr)
        self._check(st, allow=(OK, E_NOT_CONVERGED))
        return SolveResult(np.array(it[:]), np.array(rr[:]), st == OK)

    def elastic_tensor(self) -> np.ndarray:
        C = (ctypes.c_double * 36)()
        self._check(self.lib.hmg_elastic_tensor(self._h, C))
        return np.array(C[:]).reshape(6, 6)

    def sensitivity(self, W, out: torch.Tensor | None = None) -> torch.Tensor:
        Wa = (ctypes.c_double * 36)(*np.asarray(W, dtype=np.float64).ravel().tolist())
        out = torch.empty(self.n, dtype=torch.float32, device=self.device) if out is None else out
        self._check(self.lib.hmg_sensitivity(self._h, Wa, _ptr(self._scalar(out, "out"))))
        return out

    def oc_update(self, x: torch.Tensor, dfdx: torch.Tensor, volfrac: float, move=0.05,
                  damp=0.5, xmin=1e-3) -> float:
        lam = ctypes.c_double()
        self._check(self.lib.hmg_oc_update(self._h, _ptr(self._scalar(x, "x")),
                                           _ptr(self._scalar(dfdx, "dfdx")), volfrac, move, damp,
                                           xmin, ctypes.byref(lam)))
        return lam.value

    def filter(self, inp: torch.Tensor, out: torch.Tensor | None = None, radius=2.0,
               adjoint=False) -> torch.Tensor:
        out = torch.empty(self.n, dtype=torch.float32, device=self.device) if out is None else out
        self._check(self.lib.hmg_filter(self._h, _ptr(self._scalar(inp, "in")),
                                        _ptr(self._scalar(out, "out")), radius, int(adjoint)))
        return out

    def filter_sensitivity(self, x: torch.Tensor, g: torch.Tensor,
                           out: torch.Tensor | None = None, radius=2.0) -> torch.Tensor:
        out = torch.empty(self.n, dtype=torch.float32, device=self.device) if out is None else out
        self._check(self.lib.hmg_filter_sensitivity(self._h, _ptr(self._scalar(x, "x")),
                                                    _ptr(self._scalar(g, "g")),
                                                    _ptr(self._scalar(out, "out")), radius))
        return out

    def symmetrize(self, inp: torch.Tensor, kind: str,
                   out: torch.Tensor | None = None) -> torch.Tensor:
        out = torch.empty(self.n, dtype=torch.float32, device=self.device) if out is None else out
        self._check(self.lib.hmg_symmetrize(self._h, _ptr(self._scalar(inp, "in")),
                                            _ptr(self._scalar(out, "out")), SYMMETRIES[kind]))
        return out

    def trig_init(self, nfreq: int, q, weights, volfrac: float, rho_min=1e-3, k=15.0,
                  out: torch.Tensor | None = None):
        """hmg_trig_init; returns (density, mu)."""
        out = torch.empty(self.n, dtype=torch.float32, device=self.device) if out is None else out
        w = np.ascontiguousarray(weights, dtype=np.float64)
        mu = ctypes.c_double()
        self._check(self.lib.hmg_trig_init(self._h, int(nfreq), _dbl(q), _dbl(w), int(w.size),
                                           volfrac, rho_min, k, _ptr(self._scalar(out, "out")),
                                           ctypes.byref(mu)))
        return out, mu.value

    def get_displacement(self, out: torch.Tensor | None = None) -> torch.Tensor:
        out = self.new_field() if out is None else out
        self._check(self.lib.hmg_get_displacement(self._h, _ptr(self._field(out, name="u"))))
        return out

    def num_levels(self) -> int:
        v = ctypes.c_int32()
        self._check(self.lib.hmg_num_levels(self._h, ctypes.byref(v)))
        return v.value

    def level_dims(self, level: int):
        d = (ctypes.c_int32 * 3)()
        self._check(self.lib.hmg_level_dims(self._h, level, d))
        return tuple(d[:])

    def profile(self, enable: bool):
        self._check(self.lib.hmg_profile(self._h, int(enable)))

    def profile_read(self) -> dict:
        """{kernel: (launches, total_ms, total_algorithmic_bytes)} since profile(True)."""
        out = {}
        for name, k in KERNELS.items():
            cnt, ms, by = ctypes.c_int64(), ctypes.c_double(), ctypes.c_double()
            self._check(self.lib.hmg_profile_read(self._h, k, ctypes.byref(cnt), ctypes.byref(ms),
                                                  ctypes.byref(by)))
            out[name] = (cnt.value, ms.value, by.value)
        return out

    def level_omega(self, level: int) -> float:
        v = ctypes.c_double()
        self._check(self.lib.hmg_level_omega(self._h, level, ctypes.byref(v)))
        return v.value

    def apply_operator(self, level: int, u: torch.Tensor, y: torch.Tensor | None = None):
        n = int(np.prod(self.level_dims(level)))
        y = self.new_field(level) if y is None else y
        self._check(self.lib.hmg_apply_operator(self._h, level, _ptr(self._field(u, n, "u")),
                                                _ptr(self._field(y, n, "y"))))
        return y

    def get_stencil(self, level: int, out: torch.Tensor | None = None) -> torch.Tensor:
        n = int(np.prod(self.level_dims(level)))
        if out is None:
            out = torch.empty((27, 3, 3, n), dtype=self.field_dtype, device=self.device)
        if out.numel() != 243 * n or out.dtype != self.field_dtype or not out.is_contiguous():
            raise ValueError("stencil buffer must hold 243*n field-type values")
        self._check(self.lib.hmg_get_stencil(self._h, level, _ptr(out)))
        return out

    def load_vectors(self, out: torch.Tensor | None = None) -> torch.Tensor:
        out = self.new_field() if out is None else out
        self._check(self.lib.hmg_load_vectors(self._h, _ptr(self._field(out, name="f"))))
        return out

    def vcycle(self, r: torch.Tensor, z: torch.Tensor | None = None) -> torch.Tensor:
        z = self.new_field() if z is None else z
        self._check(self.lib.hmg_vcycle(self._h, _ptr(self._field(r, name="r")),
                                        _ptr(self._field(z, name="z"))))
        return z

    def transfer(self, level: int, direction: int, inp: torch.Tensor,
                 out: torch.Tensor | None = None) -> torch.Tensor:
        src_level = level if direction == 0 else level + 1
        dst_level = level + 1 if direction == 0 else level
        nin = int(np.prod(self.level_dims(src_level)))
        out = self.new_field(dst_level) if out is None else out
        nout = int(np.prod(self.level_dims(dst_level)))
        self._check(self.lib.hmg_transfer(self._h, level, direction,
                                          _ptr(self._field(inp, nin, "in")),
                                          _ptr(self._field(out, nout, "out"))))
        return out


class Batch:
    """Many cells solved in lockstep (hmg_batch_create ... hmg_batch_destroy)."""

    def __init__(self, shapes, *, E0=1.0, nu=0.3, penal=3.0, Emin=1e-9, replace_every=0,
                 stream: torch.cuda.Stream | None = None):
        self.lib = _lib.load()
        self.shapes = [tuple(int(v) for v in s) for s in shapes]
        self.device = torch.device("cuda", torch.cuda.current_device())
        # graphs cannot be captured on the legacy default stream: own a stream
        self.stream = stream if stream is not None else torch.cuda.Stream()
        cfg = _lib.HmgConfig(0, 0, 0, E0, nu, penal, Emin, 0, 0.0, 1, 1, PRECISIONS["fp32"],
                             replace_every)
        dims = (ctypes.c_int32 * (3 * len(self.shapes)))(*[v for s in self.shapes for v in s])
        h = ctypes.c_void_p()
        st = self.lib.hmg_batch_create(ctypes.byref(cfg), len(self.shapes), dims,
                                       ctypes.c_void_p(self.stream.cuda_stream), ctypes.byref(h))
        if st != OK:
            raise HmgError(st, "hmg_batch_create failed (see stderr)")
        self._h = h

    def _check(self, st, allow=(OK,)):
        if st not in allow:
            raise HmgError(st, self.lib.hmg_batch_last_error(self._h).decode())
        return st

    def destroy(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            self.lib.hmg_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.destroy()
        except Exception:
            pass

    def set_density(self, cell: int, rho: torch.Tensor):
        nx, ny, nz = self.shapes[cell]
        if rho.device != self.device or rho.dtype != torch.float32 or not rho.is_contiguous() \
                or rho.numel() != nx * ny * nz:
            raise ValueError(f"rho must be a contiguous float32 tensor on {self.device} "
                             "of the cell's size")
        self.stream.wait_stream(torch.cuda.current_stream())
        self._check(self.lib.hmg_batch_set_density(self._h, cell, _ptr(rho)))

    def tune(self):
        g = ctypes.c_int32()
        lz = (ctypes.c_int32 * len(self.shapes))()
        self._check(self.lib.hmg_batch_tune(self._h, ctypes.byref(g), lz))
        return g.value, list(lz)

    def solve(self, rel_tol: float, max_iter: int) -> SolveResult:
        B = len(self.shapes)
        it = (ctypes.c_int32 * (6 * B))()
        rr = (ctypes.c_double * (6 * B))()
        st = self._check(self.lib.hmg_batch_solve(self._h, rel_tol, max_iter, it, rr),
                         allow=(OK, E_NOT_CONVERGED))
        return SolveResult(np.array(it[:]).reshape(B, 6), np.array(rr[:]).reshape(B, 6), st == OK)

    def elastic_tensors(self) -> np.ndarray:
        B = len(self.shapes)
        C = (ctypes.c_double * (36 * B))()
        self._check(self.lib.hmg_batch_elastic_tensors(self._h, C))
        return np.array(C[:]).reshape(B, 6, 6)
