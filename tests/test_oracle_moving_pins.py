"""Pins of the oracle's moving Voronoi mesh (Sec. 2.3 with the MUSCL-Hancock step
of Sec. 2.4, 2D Euler).

* Geometry from its definition: every Voronoi vertex is equidistant from the three
  generators whose cells meet there and no generator (or periodic image) is closer;
  every face midpoint is equidistant from its two generators and closer to them than
  to any other; the cells tile the box; each polygon is closed (sum A n = 0) and
  satisfies the divergence theorem sum A n (x_f - c)^T = V I.
* Holding the generators still (motion 0) gives the static MUSCL-Hancock step exactly.
* A uniform flow stays uniform and the mesh translates with it.
* Galilean invariance: a run boosted by a constant velocity V0 (the mesh moves with
  the boosted flow) is the unboosted run shifted by V0 t, with every velocity shifted
  by V0 (the face-frame Riemann problems, the volume flux F - U w^T and the moment
  bookkeeping only see relative velocities).  The WENO-type limiter (on primitive
  variables) keeps this; the Arepo limiter, applied to conserved coefficients, does not.
* Mass, momentum and energy are conserved through steps that change the topology.
* Second-order convergence of the cell means on the isentropic vortex with the mesh
  moving with the flow (limiter off and WENO-type with the exact flux).
"""
import math

import numpy as np
import pytest

from workloads.cartesian import vortex_fields
from workloads.voronoi import periodic_voronoi, project_voronoi, random_voronoi_state

G14 = 1.4
G53 = 5.0 / 3.0


@pytest.fixture(scope="module")
def mv(oracle):
    from oracle import moving
    return moving


def _minimg(d, box):
    return d - box * np.round(d / box)


def test_geometry_from_definition(mv):
    rng = np.random.default_rng(5)
    box = np.array([1.3, 0.9])
    P = rng.random((150, 2)) * box
    d = mv.voronoi(P, box)
    imgs = np.concatenate([P + np.array([sx, sy]) * box for sx in (-1, 0, 1)
                           for sy in (-1, 0, 1)])
    L, R = d["face_cells"][:, 0], d["face_cells"][:, 1]
    s = d["face_shift"].astype(float)
    n, A, x = d["face_normal"], d["face_area"], d["face_centroid"]
    t = np.stack([-n[:, 1], n[:, 0]], axis=1)
    rR = P[R] + s * box
    for pts in (x - 0.5 * A[:, None] * t, x + 0.5 * A[:, None] * t, x):
        dist = np.sqrt(((pts[:, None, :] - imgs[None, :, :]) ** 2).sum(-1)).min(1)
        dL = np.linalg.norm(pts - P[L], axis=1)
        dR = np.linalg.norm(pts - rR, axis=1)
        assert np.allclose(dL, dR, rtol=0, atol=1e-12)
        assert np.all(dL <= dist + 1e-12)
    assert abs(d["cell_volume"].sum() - box.prod()) < 1e-13
    Vn = np.zeros((len(P), 2))
    VI = np.zeros((len(P), 2, 2))
    c = d["cell_centroid"]
    for cell, sg, xs in ((L, 1.0, x), (R, -1.0, x - s * box)):
        np.add.at(Vn, cell, sg * A[:, None] * n)
        np.add.at(VI, cell, sg * A[:, None, None] * n[:, :, None] * (xs - c[cell])[:, None, :])
    assert np.abs(Vn).max() < 1e-13
    assert np.allclose(VI, d["cell_volume"][:, None, None] * np.eye(2), rtol=0, atol=1e-13)
    # second moments about the centroid: symmetric positive definite
    M = d["cell_moments"]
    assert np.all(M[:, 0] > 0) and np.all(M[:, 0] * M[:, 2] - M[:, 1] ** 2 > 0)


@pytest.mark.parametrize("limiter", [False, "arepo", "weno"])
@pytest.mark.parametrize("flux", ["hll", "exact"])
def test_static_generators_give_static_step(oracle, mv, limiter, flux):
    m = periodic_voronoi(400, seed=8)
    d = mv.voronoi(m["generators"], (1.0, 1.0))
    U = random_voronoi_state(d, G53, seed=9, amp=0.3)
    om = oracle.Mesh.facelist(d)
    dt = oracle.cfl_dt(om, U, G53, 0.3)
    ref = oracle.step_mh(om, U, dt, G53, limiter, flux=flux)
    got, d1 = mv.step(d, U, dt, G53, limiter, flux, motion=0)
    assert np.array_equal(d1["generators"], d["generators"])
    e = np.abs(got - ref).reshape(12, -1)
    assert e[0::3].max() < 1e-14 and e[1::3].max() * 0.05 < 1e-14 and e[2::3].max() * 0.05 < 1e-14


def test_uniform_flow(mv):
    n = 500
    d = mv.voronoi(periodic_voronoi(n, seed=3)["generators"], (1.0, 1.0))
    U = np.zeros((12, n))
    U[0], U[3], U[6] = 1.3, 1.3 * 0.7, 1.3 * -0.4
    U[9] = 2.0 / (G14 - 1) + 0.5 * 1.3 * (0.49 + 0.16)
    U = U.reshape(-1)
    d0, t, V = d, 0.0, U
    for _ in range(3):
        dt = mv.cfl_dt(d, V, G14, 0.3)
        V, d = mv.step(d, V, dt, G14, "weno", "exact")
        t += dt
    h = 1.0 / math.sqrt(n)
    e = np.abs(V - U).reshape(12, n) * np.array([1.0, h, h] * 4)[:, None]
    assert e.max() < 1e-12 * np.abs(U).max()
    shift = _minimg(d["generators"] - d0["generators"] - np.array([0.7, -0.4]) * t, 1.0)
    assert np.abs(shift).max() < 1e-14
    assert np.abs(d["cell_volume"] - d0["cell_volume"]).max() < 1e-15


def _boost(U, V, n):
    """Conserved P1 state seen by an observer moving with -V (velocities + V)."""
    U = U.reshape(12, n).copy()
    for c in range(3):
        r, mx, my = U[c].copy(), U[3 + c].copy(), U[6 + c].copy()
        U[9 + c] = U[9 + c] + mx * V[0] + my * V[1] + 0.5 * r * (V @ V)
        U[3 + c] = mx + r * V[0]
        U[6 + c] = my + r * V[1]
    return U.reshape(-1)


@pytest.mark.parametrize("limiter,flux", [("weno", "exact"), (False, "hll"), ("weno", "hll")])
def test_galilean_invariance(mv, limiter, flux):
    n = 600
    d = mv.voronoi(periodic_voronoi(n, seed=3)["generators"], (1.0, 1.0))
    U0 = random_voronoi_state(d, G53, seed=7, amp=0.3)
    V0 = np.array([0.37, -0.21])
    Ua, da = U0.copy(), d
    Ub, db = _boost(U0, V0, n), d
    t = 0.0
    for _ in range(6):
        dt = mv.cfl_dt(da, Ua, G53, 0.3)
        Ua, da = mv.step(da, Ua, dt, G53, limiter, flux)
        Ub, db = mv.step(db, Ub, dt, G53, limiter, flux)
        t += dt
    h = 1.0 / math.sqrt(n)
    e = np.abs(_boost(Ub, -V0, n) - Ua).reshape(12, n) * np.array([1.0, h, h] * 4)[:, None]
    assert e.max() < 1e-11, e.max(1)
    assert np.abs(_minimg(db["generators"] - da["generators"] - V0 * t, 1.0)).max() < 1e-13
    assert np.abs(Ua - U0).max() > 0.05  # the flow did evolve


def test_arepo_limiter_is_not_galilean_invariant(mv):
    """The Arepo limiter acts on conserved coefficients (momentum, total energy),
    which a boost changes: a documented property of that reading."""
    n = 600
    d = mv.voronoi(periodic_voronoi(n, seed=3)["generators"], (1.0, 1.0))
    U0 = random_voronoi_state(d, G53, seed=7, amp=0.3)
    V0 = np.array([0.37, -0.21])
    dt = mv.cfl_dt(d, U0, G53, 0.3)
    Ua, _ = mv.step(d, U0, dt, G53, "arepo", "exact")
    Ub, _ = mv.step(d, _boost(U0, V0, n), dt, G53, "arepo", "exact")
    assert np.abs(_boost(Ub, -V0, n) - Ua).max() > 1e-6


def test_scale_invariance(mv):
    """The Euler equations are invariant under x -> lam x, t -> lam t: the same
    generators and state in a box scaled by lam, stepped with dt scaled by lam,
    give the same cell values (gradients scaled by 1/lam) and a scaled mesh.  A
    non-square box with a non-unit scale exercises every periodic image."""
    n, box, lam = 600, np.array([1.3, 0.8]), 7.0
    P = periodic_voronoi(n, seed=19, box=tuple(box))["generators"]
    d1 = mv.voronoi(P, box)
    dL = mv.voronoi(P * lam, box * lam)
    U1 = random_voronoi_state(d1, G53, seed=20, amp=0.3)
    UL = U1.reshape(12, n).copy()
    UL[1::3] /= lam
    UL[2::3] /= lam
    UL = UL.reshape(-1)
    for _ in range(4):
        dt = mv.cfl_dt(d1, U1, G53, 0.3)
        U1, d1 = mv.step(d1, U1, dt, G53, "weno", "exact")
        UL, dL = mv.step(dL, UL, lam * dt, G53, "weno", "exact")
    A, B = U1.reshape(12, n), UL.reshape(12, n)
    h = math.sqrt(box.prod() / n)
    e = max(np.abs(A[0::3] - B[0::3]).max(),
            h * np.abs(A[1::3] - lam * B[1::3]).max(), h * np.abs(A[2::3] - lam * B[2::3]).max())
    assert e < 1e-11 * np.abs(A).max(), e
    assert np.abs(dL["generators"] - lam * d1["generators"]).max() < 1e-12 * lam


def test_conservation_through_topology_changes(mv):
    n = 800
    d = mv.voronoi(periodic_voronoi(n, seed=4)["generators"], (1.0, 1.0))

    def shear(X, Y):
        rho = 1.0 + 0.5 * (np.abs(Y - 0.5) < 0.25)
        u = 0.8 * np.tanh((0.25 - np.abs(Y - 0.5)) / 0.05)
        v = 0.1 * np.sin(2 * math.pi * X)
        p = 2.5 + 0.0 * X
        return [rho, rho * u, rho * v, p / (G53 - 1) + 0.5 * rho * (u * u + v * v)]

    U = project_voronoi(shear, d)
    tot0 = (U.reshape(12, n)[0::3] * d["cell_volume"]).sum(1)
    nb0 = mv.neighbours(d)
    changed = 0
    for _ in range(8):
        dt = mv.cfl_dt(d, U, G53, 0.3)
        U, d = mv.step(d, U, dt, G53, "weno", "exact")
    nb1 = mv.neighbours(d)
    changed = sum(a != b for a, b in zip(nb0, nb1))
    tot1 = (U.reshape(12, n)[0::3] * d["cell_volume"]).sum(1)
    assert changed > 20
    assert np.all(np.abs(tot1 - tot0) <= 1e-13 * np.abs(tot0).max())


@pytest.mark.parametrize("limiter,min_order", [(False, 1.9), ("weno", 1.7)])
def test_vortex_second_order(mv, limiter, min_order):
    errs = []
    for N in (256, 1024, 4096):
        m = periodic_voronoi(N, seed=11, box=(10.0, 10.0))
        d = mv.voronoi(m["generators"], (10.0, 10.0))
        U0 = project_voronoi(vortex_fields(0.0, G14), d)
        U1, d1, _ = mv.run(d, U0, 0, G14, 0.3, limiter, "exact", t_end=1.0)
        ex = project_voronoi(vortex_fields(1.0, G14), d1).reshape(12, -1)[0]
        errs.append(np.sum(np.abs(U1.reshape(12, -1)[0] - ex) * d1["cell_volume"]) / 100.0)
    orders = [math.log(errs[i] / errs[i + 1]) / math.log(2) for i in range(2)]
    assert min(orders) >= min_order, (errs, orders)
