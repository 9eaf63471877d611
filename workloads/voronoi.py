"""Periodic 2D Voronoi meshes (face lists built on the host) and their initial states.

A mesh is the Voronoi tessellation of seeded uniform generators in the periodic box,
relaxed by Lloyd iterations (generators moved to their cell centroids), with cells
renumbered along a Morton curve so that index-contiguous cells are spatially close.
Geometry is exact for the polygons: areas, centroids and second moments come from the
closed-form moments of the fan triangles (generator, edge endpoints).

Descriptor keys (the layout of ``include/dg.h``'s face-list descriptor):
``cell_volume[n]``, ``cell_centroid[n, 2]``, ``cell_moments[n, 3]`` = (Mxx, Mxy, Myy)
about the centroid, ``face_cells[m, 2]`` = (L, R) with the unit normal L -> R,
``face_area[m]``, ``face_normal[m, 2]``, ``face_centroid[m, 2]`` (edge midpoint in L's
frame), ``face_shift[m, 2]`` in {-1, 0, 1} (R's image next to L is centroid[R] +
shift * box), plus ``box`` and ``kind = "facelist"``.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.spatial as sps


def _morton(P, box, bits=16):
    scale = (1 << bits) - 1
    xi = np.clip((P[:, 0] / box[0] * scale).astype(np.int64), 0, scale)
    yi = np.clip((P[:, 1] / box[1] * scale).astype(np.int64), 0, scale)

    def spread(v):
        v = (v | (v << 16)) & 0x0000FFFF0000FFFF
        v = (v | (v << 8)) & 0x00FF00FF00FF00FF
        v = (v | (v << 4)) & 0x0F0F0F0F0F0F0F0F
        v = (v | (v << 2)) & 0x3333333333333333
        v = (v | (v << 1)) & 0x5555555555555555
        return v

    return spread(xi) | (spread(yi) << 1)


def _build(P, box):
    n = len(P)
    box = np.asarray(box, dtype=np.float64)
    full = n < 4000
    delta = 1.0 if full else 8.0 / math.sqrt(n)
    pts = [P]
    orig = [np.arange(n)]
    offs = [np.zeros((n, 2), dtype=np.int64)]
    for dx in (-1, 0, 1):
        for dy in (-1, 0, 1):
            if dx == 0 and dy == 0:
                continue
            Q = P + np.array([dx, dy]) * box
            if full:
                keep = np.ones(n, dtype=bool)
            else:
                keep = ((Q[:, 0] > -delta * box[0]) & (Q[:, 0] < (1 + delta) * box[0]) &
                        (Q[:, 1] > -delta * box[1]) & (Q[:, 1] < (1 + delta) * box[1]))
            pts.append(Q[keep])
            orig.append(np.nonzero(keep)[0])
            offs.append(np.tile(np.array([dx, dy], dtype=np.int64), (keep.sum(), 1)))
    X = np.concatenate(pts)
    orig = np.concatenate(orig)
    offs = np.concatenate(offs)
    vor = sps.Voronoi(X)
    rp = vor.ridge_points
    rv = np.asarray(vor.ridge_vertices)
    ok = (rv.min(axis=1) >= 0) & ((rp[:, 0] < n) | (rp[:, 1] < n))
    rp, rv = rp[ok], rv[ok]
    a, b = rp[:, 0], rp[:, 1]
    A, B = orig[a], orig[b]
    oa, ob = offs[a], offs[b]
    sh = ob - oa
    # canonical orientation: L < R, or L == R with the shift pointing "up"
    flip = (A > B) | ((A == B) & ((sh[:, 0] < 0) | ((sh[:, 0] == 0) & (sh[:, 1] < 0))))
    L = np.where(flip, B, A)
    R = np.where(flip, A, B)
    oL = np.where(flip[:, None], ob, oa)
    s = np.where(flip[:, None], -sh, sh)
    V0 = vor.vertices[rv[:, 0]] - oL * box
    V1 = vor.vertices[rv[:, 1]] - oL * box
    # one face per (L, R, shift)
    key = np.stack([L, R, s[:, 0], s[:, 1]], axis=1)
    _, first = np.unique(key, axis=0, return_index=True)
    first = np.sort(first)
    L, R, s, V0, V1 = L[first], R[first], s[first], V0[first], V1[first]
    # unit normal of the edge itself (so that sum_f A n (x_f - c)^T = V I holds
    # to roundoff for every polygon), oriented from L's generator towards R's image
    e = V1 - V0
    area = np.linalg.norm(e, axis=1)
    nrm = np.stack([e[:, 1], -e[:, 0]], axis=1) / np.maximum(area, 1e-300)[:, None]
    d = (P[R] + s * box) - P[L]
    nrm = np.where((np.sum(nrm * d, axis=1) < 0)[:, None], -nrm, nrm)
    keep = area > 1e-14 * math.sqrt(box[0] * box[1] / n)
    L, R, s, V0, V1, nrm, area = L[keep], R[keep], s[keep], V0[keep], V1[keep], nrm[keep], area[keep]
    mid = 0.5 * (V0 + V1)
    # fan-triangle moments about each cell's generator
    vol = np.zeros(n)
    m1 = np.zeros((n, 2))
    m2 = np.zeros((n, 3))
    for cell, v0, v1 in ((L, V0, V1), (R, V0 - s * box, V1 - s * box)):
        p = P[cell]
        e0, e1 = v0 - p, v1 - p
        ar = 0.5 * np.abs(e0[:, 0] * e1[:, 1] - e0[:, 1] * e1[:, 0])
        sm = e0 + e1
        np.add.at(vol, cell, ar)
        np.add.at(m1, cell, ar[:, None] * sm / 3.0)
        # int x x^T over a triangle with vertices 0, e0, e1 = A/12 (e0 e0^T + e1 e1^T + s s^T)
        xx = ar / 12.0 * (e0[:, 0] ** 2 + e1[:, 0] ** 2 + sm[:, 0] ** 2)
        xy = ar / 12.0 * (e0[:, 0] * e0[:, 1] + e1[:, 0] * e1[:, 1] + sm[:, 0] * sm[:, 1])
        yy = ar / 12.0 * (e0[:, 1] ** 2 + e1[:, 1] ** 2 + sm[:, 1] ** 2)
        np.add.at(m2, cell, np.stack([xx, xy, yy], axis=1))
    dc = m1 / vol[:, None]
    cen = P + dc
    mom = np.stack([m2[:, 0] - vol * dc[:, 0] ** 2, m2[:, 1] - vol * dc[:, 0] * dc[:, 1],
                    m2[:, 2] - vol * dc[:, 1] ** 2], axis=1)
    order = np.lexsort((R, L))
    return {
        "kind": "facelist", "box": (float(box[0]), float(box[1])),
        "generators": P, "cell_volume": vol, "cell_centroid": cen, "cell_moments": mom,
        "face_cells": np.stack([L, R], axis=1)[order].astype(np.int32),
        "face_area": area[order], "face_normal": nrm[order], "face_centroid": mid[order],
        "face_shift": s[order].astype(np.int8),
    }


def periodic_voronoi(n, seed=1004, lloyd=2, box=(1.0, 1.0)):
    """Voronoi mesh of n seeded uniform generators in the periodic box after
    ``lloyd`` Lloyd iterations, cells in Morton order."""
    rng = np.random.default_rng(seed)
    box = np.asarray(box, dtype=np.float64)
    P = rng.random((n, 2)) * box
    for _ in range(lloyd):
        m = _build(P, box)
        P = np.mod(m["cell_centroid"], box)
    P = P[np.argsort(_morton(P, box), kind="stable")]
    return _build(P, box)


def project_voronoi(fields, mesh, order=4):
    """P1 projection of ``fields(X, Y) -> list of conserved arrays`` on every
    polygon: each cell is split into fan triangles (centroid, edge endpoints),
    integrated with a degree-4 Dunavant rule; gradient = M^-1 (first moments)."""
    box = np.asarray(mesh["box"])
    n = len(mesh["cell_volume"])
    L = mesh["face_cells"][:, 0].astype(np.int64)
    R = mesh["face_cells"][:, 1].astype(np.int64)
    s = mesh["face_shift"].astype(np.float64)
    A = mesh["face_area"]
    nrm = mesh["face_normal"]
    mid = mesh["face_centroid"]
    t = np.stack([-nrm[:, 1], nrm[:, 0]], axis=1)
    V0 = mid - 0.5 * A[:, None] * t
    V1 = mid + 0.5 * A[:, None] * t
    cen = mesh["cell_centroid"]
    # Dunavant degree-4 rule on the reference triangle (barycentric, weights)
    bary = np.array([[0.108103018168070, 0.445948490915965, 0.445948490915965],
                     [0.445948490915965, 0.108103018168070, 0.445948490915965],
                     [0.445948490915965, 0.445948490915965, 0.108103018168070],
                     [0.816847572980459, 0.091576213509771, 0.091576213509771],
                     [0.091576213509771, 0.816847572980459, 0.091576213509771],
                     [0.091576213509771, 0.091576213509771, 0.816847572980459]])
    wts = np.array([0.223381589678011] * 3 + [0.109951743655322] * 3)
    mean = None
    first = None
    for cell, v0, v1 in ((L, V0, V1), (R, V0 - s * box, V1 - s * box)):
        c = cen[cell]
        ar = 0.5 * np.abs((v0 - c)[:, 0] * (v1 - c)[:, 1] - (v0 - c)[:, 1] * (v1 - c)[:, 0])
        for q in range(6):
            X = bary[q, 0] * c + bary[q, 1] * v0 + bary[q, 2] * v1
            vals = fields(X[:, 0], X[:, 1])
            if mean is None:
                mean = np.zeros((len(vals), n))
                first = np.zeros((len(vals), 2, n))
            w = wts[q] * ar
            r = X - c
            for k, v in enumerate(vals):
                np.add.at(mean[k], cell, w * v)
                np.add.at(first[k, 0], cell, w * v * r[:, 0])
                np.add.at(first[k, 1], cell, w * v * r[:, 1])
    V = mesh["cell_volume"]
    M = mesh["cell_moments"]
    det = M[:, 0] * M[:, 2] - M[:, 1] ** 2
    nv = mean.shape[0]
    U = np.zeros((nv * 3, n))
    for k in range(nv):
        U[3 * k] = mean[k] / V
        U[3 * k + 1] = (M[:, 2] * first[k, 0] - M[:, 1] * first[k, 1]) / det
        U[3 * k + 2] = (-M[:, 1] * first[k, 0] + M[:, 0] * first[k, 1]) / det
    return U.reshape(-1)


def c4_state(mesh, gamma=5.0 / 3.0):
    """Gaussian density bump rho = 1 + 0.5 exp(-|x - (1/2, 1/2)|^2 / 0.01), p = 1,
    v = 0 (nearest periodic image of the centre)."""

    def f(X, Y):
        dx = (X - 0.5 + 0.5) % 1.0 - 0.5
        dy = (Y - 0.5 + 0.5) % 1.0 - 0.5
        rho = 1.0 + 0.5 * np.exp(-(dx * dx + dy * dy) / 0.01)
        return [rho, 0.0 * X, 0.0 * X, 1.0 / (gamma - 1.0) + 0.0 * X]

    return project_voronoi(f, mesh)


def random_voronoi_state(mesh, gamma, seed, amp=0.1):
    """Smooth random state (a few Fourier modes per field) projected on the mesh."""
    rng = np.random.default_rng(seed)

    def series():
        k = rng.integers(-3, 4, (4, 2))
        k[np.all(k == 0, axis=1)] = [1, 0]
        return k, rng.uniform(0.5, 1.0, 4), rng.uniform(0, 2 * math.pi, 4)

    sr, su, sv, sp_ = series(), series(), series(), series()

    def ev(X, Y, s):
        k, a, ph = s
        return sum(a[m] * np.sin(2 * math.pi * (k[m][0] * X + k[m][1] * Y) + ph[m])
                   for m in range(4)) / 4.0

    def f(X, Y):
        rho = 1.0 + amp * ev(X, Y, sr)
        u, v = amp * ev(X, Y, su), amp * ev(X, Y, sv)
        p = 1.0 + amp * ev(X, Y, sp_)
        return [rho, rho * u, rho * v, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)]

    return project_voronoi(f, mesh)


def kh_voronoi_state(mesh, gamma=5.0 / 3.0, w0=0.1, sigma=0.5 / math.sqrt(2.0)):
    """The Kelvin-Helmholtz setup of Sec. 3.6 on a periodic unit box: p = 2.5;
    rho = 2, v_x = 0.5 in the strip |y - 1/2| < 1/4, rho = 1, v_x = -0.5 outside;
    v_y = w0 sin(4 pi x) (exp(-(y - 1/4)^2 / (2 sigma^2)) + exp(-(y - 3/4)^2 /
    (2 sigma^2))).  Readings of the printed text: gamma 5/3 (printed "5.3") and a
    Gaussian exp(-(y - y0)^2 / (2 sigma^2)) (the printed exponent carries an
    extra minus sign)."""

    def f(X, Y):
        inside = np.abs(Y - 0.5) < 0.25
        rho = np.where(inside, 2.0, 1.0)
        u = np.where(inside, 0.5, -0.5)
        v = w0 * np.sin(4 * math.pi * X) * (np.exp(-(Y - 0.25) ** 2 / (2 * sigma ** 2)) +
                                           np.exp(-(Y - 0.75) ** 2 / (2 * sigma ** 2)))
        p = 2.5 + 0.0 * X
        return [rho, rho * u, rho * v, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)]

    return project_voronoi(f, mesh)
