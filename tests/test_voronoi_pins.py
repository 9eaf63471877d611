"""Pins of the oracle on periodic Voronoi meshes (face lists) and checks of the mesh
generator's geometry."""
import math

import numpy as np
import pytest

import workloads as W
from workloads.voronoi import periodic_voronoi, project_voronoi, random_voronoi_state

G14 = 1.4
G53 = 5.0 / 3.0


@pytest.fixture(scope="module")
def meshes():
    return {n: periodic_voronoi(n, seed=11) for n in (40, 400, 3000)}


def test_generator_geometry(meshes):
    for n, m in meshes.items():
        V = m["cell_volume"]
        assert abs(V.sum() - 1.0) < 1e-13
        assert len(m["face_area"]) == 3 * n  # Euler's formula on the torus
        L, R = m["face_cells"][:, 0], m["face_cells"][:, 1]
        An = m["face_area"][:, None] * m["face_normal"]
        clo = np.zeros((n, 2))
        np.add.at(clo, L, An)
        np.add.at(clo, R, -An)
        assert np.abs(clo).max() < 1e-15
        M = m["cell_moments"]
        assert np.all(M[:, 0] > 0) and np.all(M[:, 0] * M[:, 2] - M[:, 1] ** 2 > 0)
        # second moments against an independent quadrature of x x^T over the
        # polygons (degree-4 triangle rule about the centroid)
        mom = project_voronoi(lambda X, Y: [np.ones_like(X)], m)
        assert np.allclose(mom.reshape(3, -1)[0], 1.0, atol=1e-13)


def test_principal_axis_rule_exact_on_quadratics(oracle, meshes):
    """The oracle's 4-point volume rule reproduces the cell volume, the zero
    first moments and the second-moment matrix, hence every quadratic."""
    m = meshes[400]
    om = oracle.Mesh.facelist(m)
    for e in range(0, 400, 37):
        V, c, M, rq, wq = om.cell_geometry(e)
        assert abs(wq.sum() - V) < 1e-15 * V
        assert np.abs((wq[:, None] * rq).sum(0)).max() < 1e-18
        mm = np.einsum("q,qi,qj->ij", wq, rq[:, :2], rq[:, :2])
        ref = np.array([[m["cell_moments"][e, 0], m["cell_moments"][e, 1]],
                        [m["cell_moments"][e, 1], m["cell_moments"][e, 2]]])
        assert np.abs(mm - ref).max() <= 1e-13 * np.abs(ref).max()


def test_free_stream_voronoi(oracle, meshes):
    """A uniform state has L(U) = 0 on any closed polygonal mesh.  The gradient
    equations amplify the roundoff of absolute coordinates by 12/(V h^2), so the
    check is on L h^2 / |F|."""
    for n, m in meshes.items():
        om = oracle.Mesh.facelist(m)
        U = np.zeros((12, n))
        U[0], U[3], U[6], U[9] = 1.3, 0.4, -0.2, 2.5
        L = oracle.rhs(om, U.reshape(-1), G53).reshape(12, -1)
        h2 = m["cell_volume"].min()
        F = 3.0  # flux scale of this state
        assert np.abs(L[0::3]).max() * math.sqrt(h2) / F < 1e-14
        assert np.abs(L).max() * h2 / F < 1e-12


def test_conservation_voronoi_limited(oracle, meshes):
    m = meshes[400]
    om = oracle.Mesh.facelist(m)
    U = random_voronoi_state(m, G53, seed=5, amp=0.3)
    V = m["cell_volume"]
    tot0 = (U.reshape(12, -1)[0::3] * V).sum(1)
    ref = (np.abs(U.reshape(12, -1)[0::3]) * V).sum(1)
    for _ in range(5):
        U = oracle.step(om, U, 2e-3, G53, True)
    tot1 = (U.reshape(12, -1)[0::3] * V).sum(1)
    assert np.all(np.abs(tot1 - tot0) <= 1e-13 * ref)


def test_vortex_converges_on_voronoi(oracle):
    """Advected isentropic vortex on Lloyd-relaxed periodic Voronoi meshes of
    [0,10]^2: the L1 error of the density means falls at (close to) second
    order as the mean spacing halves."""
    errs, hs = [], []
    for n in (256, 1024, 4096):
        m = periodic_voronoi(n, seed=3, box=(10.0, 10.0))
        om = oracle.Mesh.facelist(m)
        U0 = project_voronoi(W.vortex_fields(0.0, G14), m)
        U1, _ = oracle.run(om, U0, 0, G14, 0.3, False, t_end=0.5)
        ex = project_voronoi(W.vortex_fields(0.5, G14), m).reshape(12, -1)[0]
        V = m["cell_volume"]
        errs.append(np.sum(np.abs(U1.reshape(12, -1)[0] - ex) * V) / V.sum())
        hs.append(math.sqrt(100.0 / n))
    orders = [math.log(errs[i] / errs[i + 1]) / math.log(hs[i] / hs[i + 1]) for i in range(2)]
    assert min(orders) >= 1.6, (errs, orders)


def test_limiter_bounds_voronoi(oracle, meshes):
    """After limiting, the linear extrapolation to every face centroid lies
    within the min/max of the cell's and its neighbours' means."""
    m = meshes[400]
    n = 400
    om = oracle.Mesh.facelist(m)
    U = random_voronoi_state(m, G53, seed=8, amp=0.3).reshape(12, -1)
    U[1::3] *= 5.0
    U[2::3] *= -4.0
    Ul = oracle.limit(om, U.reshape(-1)).reshape(12, -1)
    L, R = m["face_cells"][:, 0], m["face_cells"][:, 1]
    c = m["cell_centroid"]
    x = m["face_centroid"]
    s = m["face_shift"].astype(float)
    for v in range(4):
        mean = U[3 * v]
        hi = mean.copy()
        lo = mean.copy()
        np.maximum.at(hi, L, mean[R])
        np.maximum.at(hi, R, mean[L])
        np.minimum.at(lo, L, mean[R])
        np.minimum.at(lo, R, mean[L])
        for cell, r in ((L, x - c[L]), (R, x - s - c[R])):
            ext = Ul[3 * v][cell] + Ul[3 * v + 1][cell] * r[:, 0] + Ul[3 * v + 2][cell] * r[:, 1]
            tol = 1e-12 * (np.abs(mean).max() + 1)
            assert np.all(ext <= hi[cell] + tol) and np.all(ext >= lo[cell] - tol)
