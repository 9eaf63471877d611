"""Torch-facing wrapper of the DG library: device tensors in, device tensors out.

PyTorch supplies device memory and the current HIP stream; every step of the DG
update runs in the HIP kernels behind ``include/dg.h``.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import capi as C


def _f64p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t: torch.Tensor):
    return ctypes.c_void_p(t.data_ptr())


class Solver:
    """One mesh handle: geometry on the device, configuration, workspace.

    ``mesh`` is ``{"kind": "cartesian", "n": (nx, ny[, nz]), "lo": ..., "hi": ...}``
    or a 2D face-list descriptor (see ``workloads.voronoi``) with ``"kind": "facelist"``.
    """

    def __init__(self, mesh: dict, physics: str = "euler", precision: str = "fp64",
                 limiter: bool = True, gamma: float = 1.4, device: int | None = None):
        if not torch.cuda.is_available():
            raise RuntimeError("the DG library needs a ROCm GPU; none is visible")
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.physics = physics
        self.precision = precision
        self.limiter = bool(limiter)
        self.gamma = float(gamma)
        self.dtype = torch.float64 if precision == "fp64" else torch.float32
        cfg = C.dg_config(C.DG_MHD if physics == "mhd" else C.DG_EULER,
                          C.DG_FP64 if precision == "fp64" else C.DG_FP32,
                          C.DG_FLUX_HLLD if physics == "mhd" else C.DG_FLUX_HLL,
                          C.DG_LIMITER_MINMOD if limiter else C.DG_LIMITER_NONE, self.gamma)
        d = C.dg_mesh_desc()
        self._keep = []
        if mesh["kind"] == "cartesian":
            n = list(mesh["n"])
            d.dim = len(n)
            d.kind = 0
            for k in range(d.dim):
                d.n[k] = int(n[k])
                d.lo[k] = float(mesh["lo"][k])
                d.hi[k] = float(mesh["hi"][k])
            self.ncells = int(np.prod(n))
        elif mesh["kind"] == "facelist":
            d.dim = 2
            d.kind = 1
            arrs = {}
            for key in ("cell_volume", "cell_centroid", "cell_moments", "face_area",
                        "face_normal", "face_centroid"):
                arrs[key] = np.ascontiguousarray(mesh[key], dtype=np.float64)
                setattr(d, key, _f64p(arrs[key]))
            fc = np.ascontiguousarray(mesh["face_cells"], dtype=np.int32)
            fs = np.ascontiguousarray(mesh["face_shift"], dtype=np.int8)
            d.face_cells = fc.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
            d.face_shift = fs.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))
            d.ncells = len(arrs["cell_volume"])
            d.nfaces = len(arrs["face_area"])
            d.box[0], d.box[1] = float(mesh["box"][0]), float(mesh["box"][1])
            self._keep = [arrs, fc, fs]
            self.ncells = int(d.ncells)
        else:
            raise ValueError(f"unknown mesh kind {mesh['kind']!r}")
        h = ctypes.c_void_p()
        with torch.cuda.device(self.device):
            C.check(C.lib().dg_mesh_create(ctypes.byref(d), ctypes.byref(cfg), ctypes.byref(h)),
                    "dg_mesh_create")
        self._h = h
        self._keep = []
        self.ncoef = C.lib().dg_ncoef(h)
        self.state_len = C.lib().dg_state_len(h)

    # -------------------------------------------------------------- helpers
    def _check_state(self, U: torch.Tensor, name: str = "U") -> None:
        if not isinstance(U, torch.Tensor) or U.device != self.device:
            raise ValueError(f"{name} must be a tensor on {self.device}")
        if U.dtype != self.dtype or not U.is_contiguous() or U.numel() != self.state_len:
            raise ValueError(f"{name} must be a contiguous {self.dtype} tensor of "
                             f"{self.state_len} elements")

    def empty(self) -> torch.Tensor:
        return torch.empty(self.state_len, dtype=self.dtype, device=self.device)

    def to_device(self, U: np.ndarray) -> torch.Tensor:
        return torch.as_tensor(np.ascontiguousarray(U).reshape(-1)).to(self.device, self.dtype)

    # ---------------------------------------------------------- entry points
    def rhs(self, U: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        self._check_state(U)
        out = self.empty() if out is None else out
        self._check_state(out, "out")
        C.check(C.lib().dg_rhs(self._h, _ptr(U), _ptr(out), _stream()), "dg_rhs")
        return out

    def limit(self, U: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        self._check_state(U)
        out = self.empty() if out is None else out
        self._check_state(out, "out")
        C.check(C.lib().dg_limit(self._h, _ptr(U), _ptr(out), _stream()), "dg_limit")
        return out

    def step(self, U: torch.Tensor, dt, out: torch.Tensor | None = None) -> torch.Tensor:
        """One SSP-RK2 step; ``dt`` is a float or a device float64 tensor of one element."""
        self._check_state(U)
        out = self.empty() if out is None else out
        self._check_state(out, "out")
        if isinstance(dt, torch.Tensor):
            if dt.dtype != torch.float64 or dt.device != self.device or dt.numel() != 1:
                raise ValueError("device dt must be a one-element float64 tensor")
            st = C.lib().dg_step_devdt(self._h, _ptr(U), _ptr(out), _ptr(dt), _stream())
        else:
            st = C.lib().dg_step(self._h, _ptr(U), _ptr(out), float(dt), _stream())
        C.check(st, "dg_step")
        return out

    @staticmethod
    def _dt_args(dt):
        if isinstance(dt, torch.Tensor):
            if dt.dtype != torch.float64 or dt.numel() != 1:
                raise ValueError("device dt must be a one-element float64 tensor")
            return 0.0, _ptr(dt)
        return float(dt), None

    def stage1(self, U: torch.Tensor, dt, out: torch.Tensor) -> torch.Tensor:
        """V1 = Pi(U) + dt L(Pi(U)); dt a float or a device float64 scalar tensor."""
        self._check_state(U)
        self._check_state(out, "out")
        h, d = self._dt_args(dt)
        C.check(C.lib().dg_stage1(self._h, _ptr(U), _ptr(out), h, d, _stream()), "dg_stage1")
        return out

    def stage2(self, U: torch.Tensor, V1: torch.Tensor, dt, out: torch.Tensor,
               cfl: float = 0.0, dt_next: torch.Tensor | None = None) -> torch.Tensor:
        """U' = Pi(U)/2 + (Pi(V1) + dt L(Pi(V1)))/2; optionally dt_next = CFL step of U'."""
        self._check_state(U)
        self._check_state(V1, "V1")
        self._check_state(out, "out")
        h, d = self._dt_args(dt)
        nxt = None if dt_next is None else _ptr(dt_next)
        C.check(C.lib().dg_stage2(self._h, _ptr(U), _ptr(V1), _ptr(out), h, d, float(cfl), nxt,
                                  _stream()), "dg_stage2")
        return out

    def adjoint_step(self, U: torch.Tensor, dt: float, lam_next: torch.Tensor,
                     V1: torch.Tensor | None = None, out: torch.Tensor | None = None):
        """lam_n = (d step(U, dt)/dU)^T lam_next (dt frozen)."""
        self._check_state(U)
        self._check_state(lam_next, "lam_next")
        out = self.empty() if out is None else out
        self._check_state(out, "out")
        v1 = None if V1 is None else _ptr(V1)
        C.check(C.lib().dg_adjoint_step(self._h, _ptr(U), v1, float(dt), _ptr(lam_next),
                                        _ptr(out), _stream()), "dg_adjoint_step")
        return out

    def cfl_dt(self, U: torch.Tensor, cfl: float, out: torch.Tensor | None = None) -> torch.Tensor:
        self._check_state(U)
        out = torch.empty(1, dtype=torch.float64, device=self.device) if out is None else out
        C.check(C.lib().dg_cfl_dt(self._h, _ptr(U), float(cfl), _ptr(out), _stream()),
                "dg_cfl_dt")
        return out

    @property
    def tiling(self) -> int:
        return C.lib().dg_get_tiling(self._h)

    @tiling.setter
    def tiling(self, rows: int) -> None:
        C.check(C.lib().dg_set_tiling(self._h, int(rows)), "dg_set_tiling")

    def check(self) -> None:
        """Synchronise and raise NonPhysicalState if a kernel met one."""
        C.check(C.lib().dg_check(self._h), "dg_check")

    def close(self) -> None:
        if getattr(self, "_h", None):
            C.lib().dg_mesh_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def cartesian(n, lo, hi) -> dict:
    return {"kind": "cartesian", "n": tuple(int(v) for v in n), "lo": tuple(lo), "hi": tuple(hi)}
