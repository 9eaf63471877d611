"""Moving periodic 2D Voronoi mesh for the oracle (Sec. 2.3, 2D Euler).

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: imported by ``tests/``,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py``.

The mesh of each step is rebuilt from scratch from its generators: the Voronoi cell
of a generator is the region closer to it than to any other generator or periodic
image.  The Voronoi vertices are the circumcentres of the Delaunay triangles of the
generators and their periodic images (``scipy.spatial.Delaunay`` is the library
primitive); the face between two cells is the segment between the circumcentres of
the two triangles that share their Delaunay edge.  Areas, centroids and second moments
are the exact polygon moments (fan triangles from the generator), the mass matrix of
Sec. 2.2, which a moving mesh recomputes every step.

One step (``step``), MUSCL-Hancock as in Sec. 2.4 with the moving-mesh fluxes of
Sec. 2.3:
  1. the generators move with their cell's fluid velocity w_e (mean momentum over
     mean density, constant over the step; ``motion=0`` holds them still);
  2. the mesh of the generators at the half step t^{n+1/2} is built: its faces and
     cells carry the fluxes (the midpoint rule in time for moving faces, which keeps
     the swept volumes and moments second order);
  3. ``or_moving_update`` (C++) limits the state on the mesh of t^n and returns the new
     conserved totals Q0 = V ubar and the first moments Q1 about the cell's origin
     carried along with w_e, from the face-frame Riemann fluxes (the face velocity at
     each Gauss point) and the volume flux F - U w_e^T (``moving_cell`` in
     ``dg_oracle.cpp``);
  4. the generators advance by dt w_e (wrapped into the box) and the mesh of t^{n+1}
     is built; the new means are Q0 / V^{n+1}; the moments are moved to the new
     centroid, Q1 - (c^{n+1} - c^n - dt w_e) Q0, and the new gradients solve
     M^{n+1} g = that.

Faces shorter than 1e-10 times their generators' distance (four nearly cocircular
generators) are dropped.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.spatial as sps

from . import Mesh, NonPhysical, _LIMITER, _RIEMANN, _f64, _p, lib

_TINY_FACE = 1e-10


def voronoi(P, box):
    """Face-list descriptor (the keys ``Mesh.facelist`` reads, plus ``generators``)
    of the periodic Voronoi mesh of generators P[n, 2] in the box [0, box)."""
    P = _f64(P).reshape(-1, 2)
    n = len(P)
    box = _f64(box)
    h = math.sqrt(box[0] * box[1] / n)
    band = min(6.0 * h, 0.5 * min(box))
    pts, orig, shift = [P], [np.arange(n)], [np.zeros((n, 2), dtype=np.int64)]
    for sx in (-1, 0, 1):
        for sy in (-1, 0, 1):
            if sx == 0 and sy == 0:
                continue
            Q = P + np.array([sx, sy]) * box
            keep = ((Q[:, 0] > -band) & (Q[:, 0] < box[0] + band) &
                    (Q[:, 1] > -band) & (Q[:, 1] < box[1] + band))
            pts.append(Q[keep])
            orig.append(np.nonzero(keep)[0])
            shift.append(np.tile(np.array([sx, sy], dtype=np.int64), (int(keep.sum()), 1)))
    X = np.concatenate(pts)
    orig = np.concatenate(orig)
    shift = np.concatenate(shift)
    tri = sps.Delaunay(X)
    T = tri.simplices
    NB = tri.neighbors
    # circumcentre of every triangle
    a = X[T[:, 0]]
    b = X[T[:, 1]] - a
    c = X[T[:, 2]] - a
    bb = np.sum(b * b, axis=1)
    cc = np.sum(c * c, axis=1)
    D = 2.0 * (b[:, 0] * c[:, 1] - b[:, 1] * c[:, 0])
    CC = a + np.stack([(c[:, 1] * bb - b[:, 1] * cc) / D, (b[:, 0] * cc - c[:, 0] * bb) / D],
                      axis=1)
    # every interior edge once: the edge opposite vertex k of triangle t
    t, k = np.nonzero(NB >= 0)
    t2 = NB[t, k]
    once = t < t2
    t, k, t2 = t[once], k[once], t2[once]
    u = T[t, (k + 1) % 3]
    v = T[t, (k + 2) % 3]
    real = (u < n) | (v < n)
    u, v, t, t2 = u[real], v[real], t[real], t2[real]
    A_, B_ = orig[u], orig[v]
    su, sv = shift[u], shift[v]
    rel = sv - su
    swap = (A_ > B_) | ((A_ == B_) & ((rel[:, 0] < 0) | ((rel[:, 0] == 0) & (rel[:, 1] < 0))))
    L = np.where(swap, B_, A_)
    R = np.where(swap, A_, B_)
    sL = np.where(swap[:, None], sv, su)
    s = np.where(swap[:, None], -rel, rel)
    V0 = CC[t] - sL * box
    V1 = CC[t2] - sL * box
    key = np.stack([L, R, s[:, 0], s[:, 1]], axis=1)
    _, first = np.unique(key, axis=0, return_index=True)
    first = np.sort(first)
    L, R, s, V0, V1 = L[first], R[first], s[first], V0[first], V1[first]
    e = V1 - V0
    area = np.sqrt(np.sum(e * e, axis=1))
    dLR = P[R] + s * box - P[L]
    keep = area >= _TINY_FACE * np.sqrt(np.sum(dLR * dLR, axis=1))
    L, R, s, V0, V1, e, area, dLR = L[keep], R[keep], s[keep], V0[keep], V1[keep], e[keep], \
        area[keep], dLR[keep]
    nrm = np.stack([e[:, 1], -e[:, 0]], axis=1) / area[:, None]
    nrm = np.where((np.sum(nrm * dLR, axis=1) < 0)[:, None], -nrm, nrm)
    # polygon moments from the fan triangles (generator, V0, V1) of both cells
    vol = np.zeros(n)
    m1 = np.zeros((n, 2))
    m2 = np.zeros((n, 3))
    for cell, w0, w1 in ((L, V0, V1), (R, V0 - s * box, V1 - s * box)):
        e0 = w0 - P[cell]
        e1 = w1 - P[cell]
        ar = 0.5 * np.abs(e0[:, 0] * e1[:, 1] - e0[:, 1] * e1[:, 0])
        sm = e0 + e1
        np.add.at(vol, cell, ar)
        np.add.at(m1, cell, ar[:, None] * sm / 3.0)
        # int over the triangle (0, e0, e1) of x x^T = A/12 (e0 e0^T + e1 e1^T + s s^T)
        m2c = np.stack([e0[:, 0] ** 2 + e1[:, 0] ** 2 + sm[:, 0] ** 2,
                        e0[:, 0] * e0[:, 1] + e1[:, 0] * e1[:, 1] + sm[:, 0] * sm[:, 1],
                        e0[:, 1] ** 2 + e1[:, 1] ** 2 + sm[:, 1] ** 2], axis=1)
        np.add.at(m2, cell, (ar / 12.0)[:, None] * m2c)
    dc = m1 / vol[:, None]
    mom = np.stack([m2[:, 0] - vol * dc[:, 0] ** 2, m2[:, 1] - vol * dc[:, 0] * dc[:, 1],
                    m2[:, 2] - vol * dc[:, 1] ** 2], axis=1)
    return {
        "kind": "facelist", "box": (float(box[0]), float(box[1])), "generators": P.copy(),
        "cell_volume": vol, "cell_centroid": P + dc, "cell_moments": mom,
        "face_cells": np.stack([L, R], axis=1).astype(np.int32), "face_area": area,
        "face_normal": nrm, "face_centroid": 0.5 * (V0 + V1),
        "face_shift": s.astype(np.int8),
    }


def neighbours(d):
    """Sorted neighbour lists of every cell of a descriptor."""
    n = len(d["cell_volume"])
    out = [[] for _ in range(n)]
    for L, R in d["face_cells"]:
        out[L].append(int(R))
        out[R].append(int(L))
    return [sorted(x) for x in out]


def generator_velocity(U, n, motion=1):
    """w_e = mean momentum / mean density of every cell (motion=1), or zero."""
    U = _f64(U).reshape(12, n)
    if motion == 0:
        return np.zeros((n, 2))
    return np.ascontiguousarray(np.stack([U[3] / U[0], U[6] / U[0]], axis=1))


def cfl_dt(d, U, gamma, cfl, motion=1, mesh=None):
    """cfl * min_e 2 V_e / sum_f A_f (|(v_e - w_e) . n_f| + c_e)."""
    mesh = mesh if mesh is not None else Mesh.facelist(d)
    U = _f64(U)
    w = generator_velocity(U, mesh.ncells, motion)
    return lib().or_cfl_dt_moving(mesh._h, gamma, _p(U), _p(w), cfl)


def update(d0, dh, U, dt, gamma, limiter="weno", flux="exact", motion=1):
    """Q (conserved totals and first moments about the carried origin) of one
    moving step: ``d0`` the mesh at t^n, ``dh`` the mesh of the generators at the
    half step, from which the fluxes are taken.  Returns (Q, generator velocities)."""
    m0 = Mesh.facelist(d0)
    mh = Mesh.facelist(dh)
    U = _f64(U)
    n = m0.ncells
    assert U.size == 12 * n
    w = generator_velocity(U, n, motion)
    gen = _f64(dh["generators"])
    Q = np.empty_like(U)
    rc = lib().or_moving_update(m0._h, mh._h, _RIEMANN[flux], _LIMITER[limiter], gamma, _p(U),
                                dt, _p(gen), _p(w), _p(Q))
    if rc:
        raise NonPhysical("non-physical state in the moving-mesh step")
    return Q, w


def finish(d0, d1, Q, w, dt):
    """New state on the mesh d1 from the totals and moments Q of ``update``."""
    n = len(d1["cell_volume"])
    box = np.asarray(d1["box"])
    Q = Q.reshape(12, n)
    dc = d1["cell_centroid"] - d0["cell_centroid"]
    dc -= box * np.round(dc / box)
    delta = dc - dt * w
    V = d1["cell_volume"]
    Mxx, Mxy, Myy = d1["cell_moments"].T
    det = Mxx * Myy - Mxy * Mxy
    U = np.empty_like(Q)
    for v in range(4):
        q0 = Q[3 * v]
        qx = Q[3 * v + 1] - delta[:, 0] * q0
        qy = Q[3 * v + 2] - delta[:, 1] * q0
        U[3 * v] = q0 / V
        U[3 * v + 1] = (Myy * qx - Mxy * qy) / det
        U[3 * v + 2] = (Mxx * qy - Mxy * qx) / det
    return U.reshape(-1)


def move(P, w, dt, box):
    """Generators advanced by dt w and wrapped into [0, box)."""
    return np.mod(_f64(P) + dt * w, np.asarray(box))


def step(d, U, dt, gamma, limiter="weno", flux="exact", motion=1):
    """One moving-mesh MUSCL-Hancock step from the mesh ``d`` at t^n; returns
    (U^{n+1}, the mesh descriptor at t^{n+1})."""
    w = generator_velocity(U, len(d["cell_volume"]), motion)
    dh = voronoi(move(d["generators"], w, 0.5 * dt, d["box"]), d["box"])
    Q, w = update(d, dh, U, dt, gamma, limiter, flux, motion)
    d1 = voronoi(move(d["generators"], w, dt, d["box"]), d["box"])
    return finish(d, d1, Q, w, dt), d1


def run(d, U, nsteps, gamma, cfl, limiter="weno", flux="exact", motion=1, t_end=None):
    """Advance nsteps (or to t_end) with the moving-mesh CFL step; returns
    (U, final mesh descriptor, list of dt)."""
    U = _f64(U).copy()
    dts = []
    t = 0.0
    for _ in range(nsteps if t_end is None else 10 ** 9):
        dt = cfl_dt(d, U, gamma, cfl, motion)
        if t_end is not None:
            if t >= t_end * (1 - 1e-14):
                break
            dt = min(dt, t_end - t)
        U, d = step(d, U, dt, gamma, limiter, flux, motion)
        dts.append(dt)
        t += dt
    return U, d, dts
