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

    ``mesh`` is ``{"kind": "cartesian", "n": (nx, ny[, nz]), "lo": ..., "hi": ...}``,
    a 2D face-list descriptor (see ``workloads.voronoi``) with ``"kind": "facelist"``,
    or ``moving(descriptor)``: a moving Voronoi mesh built from the descriptor's
    generators and faces, which ``step_mh`` moves with the flow.
    """

    def __init__(self, mesh: dict, physics: str = "euler", precision: str = "fp64",
                 limiter: bool = True, gamma: float = 1.4, device: int | None = None,
                 flux: str | None = None):
        if not torch.cuda.is_available():
            raise RuntimeError("the DG library needs a ROCm GPU; none is visible")
        self.device = torch.device("cuda", torch.cuda.current_device() if device is None else device)
        self.physics = physics
        self.precision = precision
        # limiter: False (none), True or "arepo" (the Arepo limiter), "weno"
        # (the WENO-type limiter, 2D Cartesian Euler)
        limiters = {False: C.DG_LIMITER_NONE, True: C.DG_LIMITER_MINMOD,
                    "arepo": C.DG_LIMITER_MINMOD, "weno": C.DG_LIMITER_WENO}
        if limiter not in limiters:
            raise ValueError(f"unknown limiter {limiter!r}")
        self.limiter = limiter
        self.gamma = float(gamma)
        self.dtype = torch.float64 if precision == "fp64" else torch.float32
        # face flux: "hll" or "exact" for Euler (default "hll"), "hlld" for MHD
        self.flux = flux or ("hlld" if physics == "mhd" else "hll")
        fluxes = {"hll": C.DG_FLUX_HLL, "hlld": C.DG_FLUX_HLLD, "exact": C.DG_FLUX_EXACT}
        if self.flux not in fluxes:
            raise ValueError(f"unknown flux {self.flux!r}")
        cfg = C.dg_config(C.DG_MHD if physics == "mhd" else C.DG_EULER,
                          C.DG_FP64 if precision == "fp64" else C.DG_FP32,
                          fluxes[self.flux],
                          limiters[limiter], self.gamma)
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
        elif mesh["kind"] == "moving":
            d.dim = 2
            d.kind = 3
            gen = np.ascontiguousarray(mesh["generators"], dtype=np.float64).reshape(-1, 2)
            fc = np.ascontiguousarray(mesh["face_cells"], dtype=np.int32)
            fs = np.ascontiguousarray(mesh["face_shift"], dtype=np.int8)
            d.generators = _f64p(gen)
            d.face_cells = fc.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
            d.face_shift = fs.ctypes.data_as(ctypes.POINTER(ctypes.c_int8))
            d.ncells = len(gen)
            d.nfaces = len(fc)
            d.box[0], d.box[1] = float(mesh["box"][0]), float(mesh["box"][1])
            self._keep = [gen, fc, fs]
            self.ncells = int(d.ncells)
        elif mesh["kind"] == "batch":
            n = np.ascontiguousarray(mesh["n"], dtype=np.int32).reshape(-1, 2)
            box = mesh.get("box")
            if box is None:
                box = np.tile(np.array([0.0, 0.0, 1.0, 1.0]), (len(n), 1))
            box = np.ascontiguousarray(box, dtype=np.float64).reshape(-1, 4)
            if len(box) != len(n):
                raise ValueError("batch: one box per instance")
            d.dim = 2
            d.kind = 2
            d.ninst = len(n)
            d.inst_n = n.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
            d.inst_box = _f64p(box)
            self._keep = [n, box]
            self.ncells = int((n[:, 0].astype(np.int64) * n[:, 1]).sum())
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
        self.ninst = C.lib().dg_ninst(h)
        off = (ctypes.c_int64 * (self.ninst + 1))()
        C.check(C.lib().dg_instance_offsets(h, off), "dg_instance_offsets")
        self.offsets = np.array(off[:], dtype=np.int64)

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

    def pack(self, states) -> torch.Tensor:
        """Device state of a batch from one (ncoef * n_i) host array per instance."""
        parts = [np.asarray(u, dtype=np.float64).reshape(self.ncoef, -1) for u in states]
        if len(parts) != self.ninst:
            raise ValueError(f"expected {self.ninst} instance states")
        return self.to_device(np.concatenate(parts, axis=1))

    def unpack(self, U: torch.Tensor):
        """Per-instance host arrays (ncoef * n_i, float64) of a batch state."""
        A = U.double().cpu().numpy().reshape(self.ncoef, -1)
        return [A[:, self.offsets[i]:self.offsets[i + 1]].reshape(-1).copy()
                for i in range(self.ninst)]

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

    def step(self, U: torch.Tensor, dt, out: torch.Tensor | None = None, cfl: float = 0.0,
             dt_next: torch.Tensor | None = None) -> torch.Tensor:
        """One SSP-RK2 step; ``dt`` is a float or a device float64 tensor of one
        element; with a device ``dt``, optionally dt_next = CFL step of the result."""
        self._check_state(U)
        out = self.empty() if out is None else out
        self._check_state(out, "out")
        if dt_next is not None:
            if not isinstance(dt, torch.Tensor):
                raise ValueError("dt_next needs the step size as a device tensor")
            self._check_dt(dt)
            self._check_dt(dt_next)
            st = C.lib().dg_step_cfl(self._h, _ptr(U), _ptr(out), _ptr(dt), float(cfl),
                                     _ptr(dt_next), _stream())
        elif isinstance(dt, torch.Tensor):
            self._check_dt(dt)
            st = C.lib().dg_step_devdt(self._h, _ptr(U), _ptr(out), _ptr(dt), _stream())
        else:
            st = C.lib().dg_step(self._h, _ptr(U), _ptr(out), float(dt), _stream())
        C.check(st, "dg_step")
        return out

    def _check_dt(self, dt: torch.Tensor, n: int = 1) -> None:
        if (dt.dtype != torch.float64 or dt.device != self.device or not dt.is_contiguous()
                or dt.numel() < n * self.ninst):
            raise ValueError(f"device dt must be a contiguous float64 tensor of "
                             f"{n * self.ninst} elements on {self.device}")

    def _dt_args(self, dt):
        if isinstance(dt, torch.Tensor):
            self._check_dt(dt)
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

    def step_mh(self, U: torch.Tensor, dt, out: torch.Tensor | None = None, cfl: float = 0.0,
                dt_next: torch.Tensor | None = None) -> torch.Tensor:
        """One MUSCL-Hancock step (one kernel); dt a float or a device float64
        tensor (one value per instance); optionally dt_next = CFL step of U'."""
        self._check_state(U)
        out = self.empty() if out is None else out
        self._check_state(out, "out")
        h, d = self._dt_args(dt)
        nxt = None
        if dt_next is not None:
            self._check_dt(dt_next)
            nxt = _ptr(dt_next)
        C.check(C.lib().dg_step_mh(self._h, _ptr(U), _ptr(out), h, d, float(cfl), nxt,
                                   _stream()), "dg_step_mh")
        return out

    def adjoint_step(self, U: torch.Tensor, dt, lam_next: torch.Tensor,
                     V1: torch.Tensor | None = None, out: torch.Tensor | None = None):
        """lam_n = (d step(U, dt)/dU)^T lam_next (dt frozen; a float, or a device
        float64 tensor with one value per instance)."""
        self._check_state(U)
        self._check_state(lam_next, "lam_next")
        out = self.empty() if out is None else out
        self._check_state(out, "out")
        v1 = None if V1 is None else _ptr(V1)
        h, d = self._dt_args(dt)
        C.check(C.lib().dg_adjoint_step(self._h, _ptr(U), v1, h, d, _ptr(lam_next), _ptr(out),
                                        _stream()), "dg_adjoint_step")
        return out

    def run(self, U: torch.Tensor, nsteps: int, cfl: float = 0.0,
            dt_hist: torch.Tensor | None = None, out: torch.Tensor | None = None,
            ckpt_every: int = 0, ckpts=None, v1_keep=None, graph: bool = True,
            integrator: str = "rk2", two_stage: bool = False):
        """nsteps steps from U (dg_run).  cfl > 0: adaptive step sizes, written
        to dt_hist ((nsteps + 1) x ninst); cfl = 0: dt_hist (nsteps x ninst) is
        read.  integrator: "rk2" (SSP-RK2) or "mh" (MUSCL-Hancock).  two_stage:
        step with the stage-1/stage-2 kernel pair where a fused step kernel
        exists.  Returns (U_out, dt_hist)."""
        if integrator not in ("rk2", "mh"):
            raise ValueError("integrator must be 'rk2' or 'mh'")
        self._check_state(U)
        out = self.empty() if out is None else out
        self._check_state(out, "out")
        if dt_hist is None:
            if cfl <= 0:
                raise ValueError("a fixed-step run needs dt_hist")
            dt_hist = torch.empty((nsteps + 1) * self.ninst, dtype=torch.float64,
                                  device=self.device)
        self._check_dt(dt_hist, nsteps + (1 if cfl > 0 else 0))
        ck = None
        if ckpt_every > 0:
            need = (nsteps - 1) // ckpt_every
            ckpts = list(ckpts or [])
            if len(ckpts) < need:
                raise ValueError(f"need {need} checkpoint buffers")
            for c in ckpts:
                self._check_state(c, "checkpoint")
            ck = (ctypes.c_void_p * max(need, 1))(*[_ptr(c) for c in ckpts[:need]])
        v1 = None
        if v1_keep is not None:
            if len(v1_keep) < nsteps:
                raise ValueError(f"need {nsteps} V1 buffers")
            for c in v1_keep:
                self._check_state(c, "v1_keep")
            v1 = (ctypes.c_void_p * nsteps)(*[_ptr(c) for c in v1_keep[:nsteps]])
        C.check(C.lib().dg_run(self._h, _ptr(U), _ptr(out), int(nsteps), float(cfl),
                               _ptr(dt_hist), int(ckpt_every), ck, v1,
                               (C.DG_RUN_GRAPH if graph else 0) |
                               (C.DG_RUN_MUSCL_HANCOCK if integrator == "mh" else 0) |
                               (C.DG_RUN_TWO_STAGE if two_stage else 0),
                               _stream()), "dg_run")
        return out, dt_hist

    def cfl_dt(self, U: torch.Tensor, cfl: float, out: torch.Tensor | None = None) -> torch.Tensor:
        self._check_state(U)
        if out is None:
            out = torch.empty(self.ninst, dtype=torch.float64, device=self.device)
        self._check_dt(out)
        C.check(C.lib().dg_cfl_dt(self._h, _ptr(U), float(cfl), _ptr(out), _stream()),
                "dg_cfl_dt")
        return out

    @property
    def tiling(self) -> int:
        return C.lib().dg_get_tiling(self._h)

    @tiling.setter
    def tiling(self, rows: int) -> None:
        C.check(C.lib().dg_set_tiling(self._h, int(rows)), "dg_set_tiling")

    @property
    def launch(self):
        """(waves per workgroup, persistent grid waves) of the batched stage kernel."""
        w, g = ctypes.c_int(), ctypes.c_int()
        C.check(C.lib().dg_get_launch(self._h, ctypes.byref(w), ctypes.byref(g)), "dg_get_launch")
        return w.value, g.value

    @launch.setter
    def launch(self, wg) -> None:
        C.check(C.lib().dg_set_launch(self._h, int(wg[0]), int(wg[1])), "dg_set_launch")

    def check(self) -> None:
        """Synchronise and raise NonPhysicalState if a kernel met one (DGError
        with DG_EMESH if a moving mesh failed to rebuild)."""
        C.check(C.lib().dg_check(self._h), "dg_check")

    def set_motion(self, motion: int) -> None:
        """Moving meshes: 1 moves the generators with the flow, 0 holds them."""
        C.check(C.lib().dg_set_mesh_motion(self._h, int(motion)), "dg_set_mesh_motion")

    def set_timing(self, on: bool) -> None:
        """Moving meshes: record HIP events around the four kernels of each step."""
        C.check(C.lib().dg_set_moving_timing(self._h, int(bool(on))), "dg_set_moving_timing")

    def kernel_times(self):
        """Moving meshes: (average ms of the limiter, half-step mesh, update and
        new-mesh kernels over the steps timed since the last call, step count)."""
        ms = np.zeros(4)
        ns = ctypes.c_int()
        C.check(C.lib().dg_moving_timing(self._h, _f64p(ms), ctypes.byref(ns)),
                "dg_moving_timing")
        return ms, ns.value

    def geometry(self) -> dict:
        """Moving meshes: host copy of the current generators, volumes,
        centroids (generator + offset, not wrapped) and neighbour rings."""
        n = self.ncells
        gen = np.empty((n, 2))
        vol = np.empty(n)
        cen = np.empty((n, 2))
        ring = np.empty((n, 16), dtype=np.int32)
        deg = np.empty(n, dtype=np.int32)
        i32 = ctypes.POINTER(ctypes.c_int32)
        C.check(C.lib().dg_mesh_geometry(self._h, _f64p(gen), _f64p(vol), _f64p(cen),
                                         ring.ctypes.data_as(i32), deg.ctypes.data_as(i32)),
                "dg_mesh_geometry")
        return {"generators": gen, "volume": vol, "centroid": cen, "ring": ring, "degree": deg}

    def close(self) -> None:
        if getattr(self, "_h", None):
            C.lib().dg_mesh_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def batch(sizes, boxes=None) -> dict:
    """Batch of periodic 2D Cartesian instances: sizes [(nx, ny), ...], boxes
    [(lo_x, lo_y, hi_x, hi_y), ...] (default: the unit square)."""
    return {"kind": "batch", "n": [tuple(int(v) for v in n) for n in sizes], "box": boxes}


def moving(mesh: dict) -> dict:
    """A moving Voronoi mesh from a face-list descriptor with generators (its
    generators and faces give the initial mesh; the library builds the rest)."""
    return {"kind": "moving", "generators": mesh["generators"], "face_cells": mesh["face_cells"],
            "face_shift": mesh["face_shift"], "box": mesh["box"]}


def cartesian(n, lo, hi) -> dict:
    return {"kind": "cartesian", "n": tuple(int(v) for v in n), "lo": tuple(lo), "hi": tuple(hi)}
