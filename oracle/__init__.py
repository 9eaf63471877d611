"""Plain FP64 CPU oracle of the centroidal-Taylor P1 DG scheme (Mocz et al. 2013).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, by ``__graft_entry__.smoke()`` and
by the ``cpu_baseline`` leg of ``bench.py``.  The product package never imports it.

The arithmetic lives in ``dg_oracle.cpp`` (C++17, OpenMP over cells, templated on
the scalar so that dual numbers give exact directional derivatives).  This module
only marshals NumPy arrays into it.  See the C++ header comment for what each entry
computes and which passage of the paper it follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dg_oracle.cpp")
_PORTABLE = os.path.join(_HERE, "libdgoracle.so")
_LIB = _PORTABLE  # the copy lib() loads

_dp = ctypes.POINTER(ctypes.c_double)
_i64p = ctypes.POINTER(ctypes.c_int64)


def build(force: bool = True) -> str:
    """Compile the oracle with g++ (no -march=native: the library travels)."""
    if force or not os.path.exists(_PORTABLE) or os.path.getmtime(_PORTABLE) < os.path.getmtime(_SRC):
        tmp = _PORTABLE + ".tmp"
        cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-shared", "-fPIC", _SRC, "-o", tmp]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _PORTABLE)
    return _PORTABLE


_lib = None
BUILD_FLAGS = "-O2 -std=c++17 -fopenmp"


def use_native_build(directory: str) -> bool:
    """Compile the oracle for this host's CPU (g++ -O3 -march=native, the flags a
    host timing of the oracle calls for) into ``directory`` and load that copy
    instead of the portable one.  Must run before the first oracle call; returns
    False (and keeps the portable build) if the compiler is unavailable."""
    global _LIB, BUILD_FLAGS
    if _lib is not None:
        return False
    path = os.path.join(directory, "libdgoracle_native.so")
    cmd = ["g++", "-O3", "-march=native", "-std=c++17", "-fopenmp", "-shared", "-fPIC", _SRC,
           "-o", path]
    try:
        subprocess.run(cmd, check=True, capture_output=True)
    except (OSError, subprocess.CalledProcessError):
        return False
    _LIB = path
    BUILD_FLAGS = "-O3 -march=native -std=c++17 -fopenmp"
    return True


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        L = ctypes.CDLL(_LIB)
        L.or_mesh_cartesian.restype = ctypes.c_void_p
        L.or_mesh_cartesian.argtypes = [ctypes.c_int, _i64p, _dp, _dp]
        L.or_mesh_facelist2d.restype = ctypes.c_void_p
        L.or_mesh_facelist2d.argtypes = [ctypes.c_int64, ctypes.c_int64, _dp, _dp, _dp, _dp,
                                         ctypes.POINTER(ctypes.c_int32), _dp, _dp, _dp,
                                         ctypes.POINTER(ctypes.c_int8)]
        L.or_mesh_free.argtypes = [ctypes.c_void_p]
        L.or_mesh_ncells.restype = ctypes.c_int64
        L.or_mesh_ncells.argtypes = [ctypes.c_void_p]
        L.or_ncoef.restype = ctypes.c_int
        L.or_ncoef.argtypes = [ctypes.c_int, ctypes.c_int]
        L.or_rhs.restype = ctypes.c_int
        L.or_rhs.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_double, _dp,
                             _dp]
        L.or_limit.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_double, _dp,
                               _dp]
        L.or_step.restype = ctypes.c_int
        L.or_step.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                              ctypes.c_double, _dp, ctypes.c_double, _dp]
        L.or_step_jvp.restype = ctypes.c_int
        L.or_step_jvp.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                  _dp, _dp, ctypes.c_double, _dp, _dp]
        L.or_step_branches.restype = ctypes.c_int
        L.or_step_branches.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_double, _dp,
                                       ctypes.c_double, _dp, ctypes.POINTER(ctypes.c_int)]
        L.or_step_mh.restype = ctypes.c_int
        L.or_step_mh.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                 _dp, ctypes.c_double, _dp]
        L.or_rhs_mh.restype = ctypes.c_int
        L.or_rhs_mh.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_double, _dp,
                                ctypes.c_double, _dp]
        L.or_predict_prim.argtypes = [ctypes.c_int, ctypes.c_double, _dp, _dp, ctypes.c_double,
                                      _dp, _dp]
        L.or_rhs_jvp.restype = ctypes.c_int
        L.or_rhs_jvp.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_double, _dp, _dp, _dp,
                                 _dp]
        L.or_cfl_dt.restype = ctypes.c_double
        L.or_cfl_dt.argtypes = [ctypes.c_void_p, ctypes.c_int, ctypes.c_double, _dp,
                                ctypes.c_double]
        L.or_flux.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, _dp, _dp, _dp]
        L.or_hll.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, _dp, _dp, _dp, _dp]
        L.or_hlld.argtypes = [ctypes.c_double, _dp, _dp, _dp, _dp]
        L.or_signal_speed.restype = ctypes.c_double
        L.or_signal_speed.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, _dp, _dp]
        L.or_exact_riemann.restype = ctypes.c_int
        L.or_exact_riemann.argtypes = [ctypes.c_int, ctypes.c_double, _dp, _dp, _dp, _dp, _dp,
                                       _dp]
        L.or_cell_geometry.argtypes = [ctypes.c_void_p, ctypes.c_int64, _dp, _dp, _dp,
                                       ctypes.POINTER(ctypes.c_int), _dp, _dp]
        L.or_gram_B.argtypes = [_dp, _dp]
        L.or_gram_B2.argtypes = [_dp, _dp]
        L.or_eval_B.argtypes = [_dp, _dp, _dp, _dp]
        L.or_divB.argtypes = [ctypes.c_void_p, _dp, _dp]
        L.or_num_threads.restype = ctypes.c_int
        L.or_set_num_threads.argtypes = [ctypes.c_int]
        L.or_moving_update.restype = ctypes.c_int
        L.or_moving_update.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_double, _dp, ctypes.c_double, _dp, _dp, _dp]
        L.or_cfl_dt_moving.restype = ctypes.c_double
        L.or_cfl_dt_moving.argtypes = [ctypes.c_void_p, ctypes.c_double, _dp, _dp,
                                       ctypes.c_double]
        _lib = L
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(_dp)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def num_threads() -> int:
    return lib().or_num_threads()


def set_num_threads(n: int) -> None:
    lib().or_set_num_threads(int(n))


class NonPhysical(RuntimeError):
    """A quadrature point carried rho <= 0, p <= 0 or a non-finite value."""


class Mesh:
    """A mesh as the oracle sees it.  Build with :meth:`cartesian` or :meth:`facelist`."""

    def __init__(self, handle: int, dim: int, ncells: int, keep=()):
        self._h = ctypes.c_void_p(handle)
        self.dim = dim
        self.ncells = ncells
        self._keep = keep

    @classmethod
    def cartesian(cls, n, lo, hi) -> "Mesh":
        dim = len(n)
        nn = np.array(list(n) + [1] * (3 - dim), dtype=np.int64)
        l = _f64(list(lo) + [0.0] * (3 - dim))
        h = _f64(list(hi) + [1.0] * (3 - dim))
        hd = lib().or_mesh_cartesian(dim, nn.ctypes.data_as(_i64p), _p(l), _p(h))
        return cls(hd, dim, int(np.prod(nn)))

    @classmethod
    def facelist(cls, d) -> "Mesh":
        """2D periodic face-list mesh from a descriptor dict (see ``workloads.voronoi``)."""
        box = _f64(d["box"])
        V = _f64(d["cell_volume"])
        c = _f64(d["cell_centroid"])
        M = _f64(d["cell_moments"])
        fc = np.ascontiguousarray(d["face_cells"], dtype=np.int32)
        A = _f64(d["face_area"])
        n = _f64(d["face_normal"])
        x = _f64(d["face_centroid"])
        s = np.ascontiguousarray(d["face_shift"], dtype=np.int8)
        hd = lib().or_mesh_facelist2d(len(V), len(A), _p(box), _p(V), _p(c), _p(M),
                                      fc.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                      _p(A), _p(n), _p(x),
                                      s.ctypes.data_as(ctypes.POINTER(ctypes.c_int8)))
        return cls(hd, 2, len(V), keep=(box, V, c, M, fc, A, n, x, s))

    def __del__(self):
        if getattr(self, "_h", None) is not None and _lib is not None:
            _lib.or_mesh_free(self._h)
            self._h = None

    def cell_geometry(self, e: int):
        V = ctypes.c_double()
        c = np.zeros(3)
        M = np.zeros(9)
        nq = ctypes.c_int()
        rq = np.zeros(24)
        wq = np.zeros(8)
        lib().or_cell_geometry(self._h, e, ctypes.byref(V), _p(c), _p(M), ctypes.byref(nq),
                               _p(rq), _p(wq))
        k = nq.value
        return V.value, c, M.reshape(3, 3), rq[:3 * k].reshape(k, 3), wq[:k]


def ncoef(dim: int, mhd: bool) -> int:
    return lib().or_ncoef(dim, int(mhd))


def _state(mesh: Mesh, U, mhd: bool) -> np.ndarray:
    U = _f64(U)
    assert U.size == ncoef(mesh.dim, mhd) * mesh.ncells, "state length mismatch"
    return U


_RIEMANN = {"hll": 0, "exact": 1}


def rhs(mesh: Mesh, U, gamma: float, mhd: bool = False, check: bool = True,
        flux: str = "hll") -> np.ndarray:
    """Semi-discrete DG right-hand side L(U), coefficient-major layout.
    flux: the Euler face flux, "hll" or "exact" (MHD always uses HLLD)."""
    U = _state(mesh, U, mhd)
    out = np.empty_like(U)
    rc = lib().or_rhs(mesh._h, int(mhd), _RIEMANN[flux], gamma, _p(U), _p(out))
    if rc and check:
        raise NonPhysical("non-physical state in L(U)")
    return out


_LIMITER = {False: 0, True: 1, "arepo": 1, "weno": 2}


def limit(mesh: Mesh, U, mhd: bool = False, kind: str = "arepo",
          gamma: float = 1.4) -> np.ndarray:
    """Slope limiter Pi(U), means unchanged: "arepo" scales the gradients by
    alpha; "weno" (Euler) blends the stencil and DG primitive slopes."""
    U = _state(mesh, U, mhd)
    out = np.empty_like(U)
    lib().or_limit(mesh._h, int(mhd), _LIMITER[kind], gamma, _p(U), _p(out))
    return out


def step(mesh: Mesh, U, dt: float, gamma: float, limiter: bool, mhd: bool = False,
         check: bool = True, flux: str = "hll") -> np.ndarray:
    """One SSP-RK2 step with the limiter at the start of each stage."""
    U = _state(mesh, U, mhd)
    out = np.empty_like(U)
    rc = lib().or_step(mesh._h, int(mhd), _RIEMANN[flux], _LIMITER[limiter], gamma, _p(U), dt,
                       _p(out))
    if rc and check:
        raise NonPhysical("non-physical state in step")
    return out


def step_branches(mesh: Mesh, U, dt: float, gamma: float, limiter: bool = True):
    """One SSP-RK2 step (2D Euler, box, HLL) and the branches it takes: int codes
    [2 stages, ncells, 12] (the limiter of the four variables, then HLL at the
    two Gauss points of the faces -x, +x, -y, +y).  Two steps took the same
    branches everywhere exactly when their codes are equal."""
    U = _state(mesh, U, False)
    out = np.empty_like(U)
    codes = np.zeros((2, mesh.ncells, 12), dtype=np.int32)
    rc = lib().or_step_branches(mesh._h, int(bool(limiter)), gamma, _p(U), dt, _p(out),
                                codes.ctypes.data_as(ctypes.POINTER(ctypes.c_int)))
    if rc == 2:
        raise ValueError("step_branches: 2D Euler on a box only")
    if rc:
        raise NonPhysical("non-physical state in step_branches")
    return out, codes


def step_jvp(mesh: Mesh, U, dU, dt: float, gamma: float, limiter: bool, mhd: bool = False):
    """(S(U), dS/dU . dU) by dual numbers."""
    U = _state(mesh, U, mhd)
    dU = _state(mesh, dU, mhd)
    out = np.empty_like(U)
    dout = np.empty_like(U)
    rc = lib().or_step_jvp(mesh._h, int(mhd), int(limiter), gamma, _p(U), _p(dU), dt, _p(out),
                           _p(dout))
    if rc:
        raise NonPhysical("non-physical state in step_jvp")
    return out, dout


def rhs_jvp(mesh: Mesh, U, dU, gamma: float, mhd: bool = False):
    U = _state(mesh, U, mhd)
    dU = _state(mesh, dU, mhd)
    out = np.empty_like(U)
    dout = np.empty_like(U)
    rc = lib().or_rhs_jvp(mesh._h, int(mhd), gamma, _p(U), _p(dU), _p(out), _p(dout))
    if rc:
        raise NonPhysical("non-physical state in rhs_jvp")
    return out, dout


def cfl_dt(mesh: Mesh, U, gamma: float, cfl: float, mhd: bool = False) -> float:
    U = _state(mesh, U, mhd)
    return lib().or_cfl_dt(mesh._h, int(mhd), gamma, _p(U), cfl)


def step_mh(mesh: Mesh, U, dt: float, gamma: float, limiter: bool,
            flux: str = "hll") -> np.ndarray:
    """One MUSCL-Hancock step (Euler): Ua = Pi(U), U' = Ua + dt L_MH(Ua; dt/2)."""
    U = _state(mesh, U, False)
    out = np.empty_like(U)
    if lib().or_step_mh(mesh._h, _RIEMANN[flux], _LIMITER[limiter], gamma, _p(U), dt, _p(out)):
        raise NonPhysical("non-physical state in the MUSCL-Hancock step")
    return out


def rhs_mh(mesh: Mesh, U, half_dt: float, gamma: float, flux: str = "hll") -> np.ndarray:
    """The MUSCL-Hancock operator: surface and volume terms of the half-step
    primitive prediction (no limiter)."""
    U = _state(mesh, U, False)
    out = np.empty_like(U)
    rc = lib().or_rhs_mh(mesh._h, _RIEMANN[flux], gamma, _p(U), half_dt, _p(out))
    if rc:
        raise NonPhysical("non-physical state in the MUSCL-Hancock operator")
    return out


def predict_prim(mean, grad, gamma: float, half_dt: float):
    """(primitive centroid values advanced by half_dt, primitive gradients
    [nvar x 3]) of one cell from its conserved mean and gradients."""
    mean = _f64(mean)
    dim = len(mean) - 2
    grad = _f64(grad).reshape(dim + 2, dim)
    prim = np.empty(dim + 2)
    gprim = np.empty((dim + 2) * 3)
    lib().or_predict_prim(dim, gamma, _p(mean), _p(grad), half_dt, _p(prim), _p(gprim))
    return prim, gprim.reshape(dim + 2, 3)[:, :dim]


def run(mesh: Mesh, U, nsteps: int, gamma: float, cfl: float, limiter: bool,
        mhd: bool = False, t_end: float | None = None, integrator: str = "rk2",
        flux: str = "hll"):
    """Advance nsteps (or until t_end) with the CFL step; returns (U, dt list).
    integrator: "rk2" (SSP-RK2) or "mh" (MUSCL-Hancock, Euler only); flux: the
    Euler face flux ("hll" or "exact")."""
    U = _f64(U).copy()
    dts = []
    t = 0.0
    for _ in range(nsteps if t_end is None else 10 ** 9):
        dt = cfl_dt(mesh, U, gamma, cfl, mhd)
        if t_end is not None:
            if t >= t_end * (1 - 1e-14):
                break
            dt = min(dt, t_end - t)
        if integrator == "mh":
            U = step_mh(mesh, U, dt, gamma, limiter, flux=flux)
        else:
            U = step(mesh, U, dt, gamma, limiter, mhd, flux=flux)
        dts.append(dt)
        t += dt
    return U, dts


def flux(u, n, gamma: float, mhd: bool = False) -> np.ndarray:
    u = _f64(u)
    n3 = _f64(list(n) + [0.0] * (3 - len(n)))
    dim = 3 if mhd else len(n)
    out = np.zeros(8)
    lib().or_flux(dim, int(mhd), gamma, _p(u), _p(n3), _p(out))
    return out[:len(u)]


def hll(uL, uR, n, gamma: float) -> np.ndarray:
    uL = _f64(uL)
    uR = _f64(uR)
    n3 = _f64(list(n) + [0.0] * (3 - len(n)))
    out = np.zeros(8)
    lib().or_hll(len(n), 0, gamma, _p(uL), _p(uR), _p(n3), _p(out))
    return out[:len(uL)]


def hlld(uL, uR, n, gamma: float) -> np.ndarray:
    uL = _f64(uL)
    uR = _f64(uR)
    n3 = _f64(n)
    out = np.zeros(8)
    lib().or_hlld(gamma, _p(uL), _p(uR), _p(n3), _p(out))
    return out


def signal_speed(u, n, gamma: float, mhd: bool = False) -> float:
    """Sound speed (Euler) or fast magnetosonic speed along the unit normal n
    (MHD) of one conserved state."""
    u = _f64(u)
    n3 = _f64(list(n) + [0.0] * (3 - len(n)))
    dim = 3 if mhd else len(n)
    return lib().or_signal_speed(dim, int(mhd), gamma, _p(u), _p(n3))


def exact_riemann(uL, uR, n, gamma: float):
    """Exact Euler Riemann solver along the unit normal n: (flux, (p*, u*),
    (rho, u_n, p) on the face).  Raises NonPhysical on vacuum generation."""
    uL = _f64(uL)
    uR = _f64(uR)
    n3 = _f64(list(n) + [0.0] * (3 - len(n)))
    out = np.zeros(8)
    star = np.zeros(2)
    face = np.zeros(3)
    if lib().or_exact_riemann(len(n), gamma, _p(uL), _p(uR), _p(n3), _p(out), _p(star),
                              _p(face)):
        raise NonPhysical("vacuum generation in the Riemann problem")
    return out[:len(uL)], star, face


def gram_B2(M) -> np.ndarray:
    """5x5 Gram matrix of the 2D B basis from the 2x2 second-moment matrix."""
    M = _f64(M).reshape(4)
    G = np.empty(25)
    lib().or_gram_B2(_p(M), _p(G))
    return G.reshape(5, 5)


def gram_B(M) -> np.ndarray:
    M = _f64(M).reshape(9)
    G = np.zeros(64)
    lib().or_gram_B(_p(M), _p(G))
    return G.reshape(8, 8)


def eval_B(bbar, a, r) -> np.ndarray:
    out = np.zeros(3)
    lib().or_eval_B(_p(_f64(bbar)), _p(_f64(a)), _p(_f64(r)), _p(out))
    return out


def divB(mesh: Mesh, U) -> np.ndarray:
    U = _state(mesh, U, True)
    out = np.zeros(mesh.ncells)
    lib().or_divB(mesh._h, _p(U), _p(out))
    return out
