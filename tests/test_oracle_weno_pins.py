"""Pins of the oracle's WENO-type limiter (Sec. 2.5: for each primitive variable,
the stencil slope limited as in the Arepo limiter and the unlimited DG slope,
blended with weights (eps + o_k)^(-1/2) from the oscillation factors o_k).

* a linear primitive field is left unchanged (both candidates are exact);
* one cell with a perturbed DG slope in a linear 1D profile, and one at a
  local maximum where the stencil slope is limited to zero: the result equals
  the blend computed by hand from the printed definitions (face-centroid
  increments, the neighbours' means, exponent 1/2, eps the machine epsilon);
* mirror symmetry x -> -x;
* the cell means are unchanged;
* second-order convergence on the isentropic vortex and the paper's acoustic
  wave with the WENO-limited scheme, and L1 convergence on the paper's Sod
  tube.
"""
import math

import numpy as np
import pytest

import workloads as W

G14 = 1.4
G53 = 5.0 / 3.0
EPS = 2.220446049250313e-16


def _order(errs):
    return [math.log(errs[i] / errs[i + 1]) / math.log(2) for i in range(len(errs) - 1)]


def _from_primitive(w, gw, g):
    """Conserved means and gradients of cells from primitive centroid values
    w[4, ncell] and gradients gw[4, 2, ncell] (chain rule)."""
    rho, vx, vy, p = w
    U = np.zeros((12, w.shape[1]))
    U[0] = rho
    U[3] = rho * vx
    U[6] = rho * vy
    U[9] = p / (g - 1) + 0.5 * rho * (vx * vx + vy * vy)
    for d in range(2):
        gr, gvx, gvy, gp = gw[0, d], gw[1, d], gw[2, d], gw[3, d]
        U[1 + d] = gr
        U[4 + d] = vx * gr + rho * gvx
        U[7 + d] = vy * gr + rho * gvy
        U[10 + d] = gp / (g - 1) + 0.5 * (vx * vx + vy * vy) * gr + rho * (vx * gvx + vy * gvy)
    return U


def test_linear_primitive_field_is_unchanged(oracle):
    n, lo, hi = (12, 10), (0.0, 0.0), (1.2, 0.7)
    h = ((hi[0] - lo[0]) / n[0], (hi[1] - lo[1]) / n[1])
    xc = lo[0] + h[0] * (np.arange(n[0]) + 0.5)
    yc = lo[1] + h[1] * (np.arange(n[1]) + 0.5)
    X, Y = np.meshgrid(xc, yc)
    X, Y = X.reshape(-1), Y.reshape(-1)
    w0 = np.array([1.0, 0.3, -0.2, 1.5])
    G = np.array([[0.2, -0.1], [0.5, 0.3], [-0.4, 0.2], [0.3, 0.6]])
    w = w0[:, None] + G[:, 0:1] * X + G[:, 1:2] * Y
    gw = np.repeat(G[:, :, None], X.size, axis=2)
    U = _from_primitive(w, gw, G14)
    m = oracle.Mesh.cartesian(n, lo, hi)
    out = oracle.limit(m, U.reshape(-1), kind="weno", gamma=G14).reshape(12, -1)
    interior = ((np.arange(X.size) % n[0]) % (n[0] - 1) != 0) & \
               ((np.arange(X.size) // n[0]) % (n[1] - 1) != 0)
    assert np.allclose(out[:, interior], U[:, interior], rtol=0, atol=1e-12)
    assert np.array_equal(out[0::3], U[0::3])


@pytest.mark.parametrize("K", [0.5, -0.3, 0.1])
def test_closed_form_one_cell(oracle, K):
    """rho linear in x (slope a) at rest under uniform pressure; cell i0's DG
    density slope replaced by K.  For rho the stencil candidate is a with
    o_s = 2 a h and the DG candidate K with o_dg = |K| h + 2 |a h - K h / 2|;
    the y-faces and the other variables contribute nothing."""
    nx, a = 16, 0.1
    h = 1.0 / nx
    xc = h * (np.arange(nx) + 0.5)
    w = np.array([1.0 + a * xc, 0 * xc, 0 * xc, 1.0 + 0 * xc])
    gw = np.zeros((4, 2, nx))
    gw[0, 0] = a
    U = _from_primitive(w, gw, G14)
    i0 = 7
    U[1, i0] = K
    m = oracle.Mesh.cartesian((nx, 1), (0.0, 0.0), (1.0, h))
    out = oracle.limit(m, U.reshape(-1), kind="weno", gamma=G14).reshape(12, -1)
    o_s = 2 * a * h
    o_dg = abs(K) * h + 2 * abs(a * h - K * h / 2)
    ws, wd = (EPS + o_s) ** -0.5, (EPS + o_dg) ** -0.5
    expect = (ws * a + wd * K) / (ws + wd)
    assert abs(out[1, i0] - expect) <= 1e-14
    assert np.all(out[[2, 4, 5, 7, 8, 10, 11], i0] == 0.0)


@pytest.mark.parametrize("K", [0.8, -0.5])
def test_closed_form_limited_stencil(oracle, K):
    """Cell i0 a local density maximum (1.3 between 1.0 and 1.2, all other
    cells 1.0): the stencil slope 0.1/h is limited to 0 (D = 0), so o_s =
    |1.0 - 1.3| + |1.2 - 1.3| and the result is the DG slope K weighted
    against zero."""
    nx = 16
    h = 1.0 / nx
    i0 = 7
    rho = np.ones(nx)
    rho[i0], rho[i0 + 1] = 1.3, 1.2
    w = np.array([rho, 0 * rho, 0 * rho, 1.0 + 0 * rho])
    U = _from_primitive(w, np.zeros((4, 2, nx)), G14)
    U[1, i0] = K
    m = oracle.Mesh.cartesian((nx, 1), (0.0, 0.0), (1.0, h))
    out = oracle.limit(m, U.reshape(-1), kind="weno", gamma=G14).reshape(12, -1)
    o_s = 0.3 + 0.1
    o_dg = abs(K) * h + abs(1.2 - 1.3 - K * h / 2) + abs(1.0 - 1.3 + K * h / 2)
    ws, wd = (EPS + o_s) ** -0.5, (EPS + o_dg) ** -0.5
    assert abs(out[1, i0] - wd * K / (ws + wd)) <= 1e-14


def test_mirror_symmetry(oracle):
    n = (14, 9)
    U = W.random_p1_state(n, (0.0, 0.0), (1.0, 1.0), G53, seed=21, amp=0.3).reshape(12, *n[::-1])
    U = U.copy()
    U[1::3] *= 3.0
    U[2::3] *= 3.0
    m = oracle.Mesh.cartesian(n, (0.0, 0.0), (1.0, 1.0))
    out = oracle.limit(m, U.reshape(-1), kind="weno", gamma=G53).reshape(12, *n[::-1])
    # mirror x -> -x: reverse the columns; every d/dx flips, and so does every
    # coefficient of m_x (whose d/dx therefore keeps its sign)
    s = np.ones(12)
    for v in range(4):
        s[3 * v + 1] = -1.0
    s[3:6] *= -1.0
    Um = (U * s[:, None, None])[:, :, ::-1]
    outm = oracle.limit(m, Um.reshape(-1), kind="weno", gamma=G53).reshape(12, *n[::-1])
    back = (outm[:, :, ::-1]) * s[:, None, None]
    assert np.allclose(back, out, rtol=0, atol=1e-13 * np.abs(out).max())


def test_means_unchanged(oracle):
    n = (10, 8)
    U = W.random_p1_state(n, (0.0, 0.0), (1.0, 1.0), G53, seed=22, amp=0.3)
    m = oracle.Mesh.cartesian(n, (0.0, 0.0), (1.0, 1.0))
    out = oracle.limit(m, U, kind="weno", gamma=G53).reshape(12, -1)
    assert np.array_equal(out[0::3], U.reshape(12, -1)[0::3])


def test_smooth_second_order(oracle):
    errs = []
    for n in [16, 32, 64]:
        shape = (n, n)
        m = oracle.Mesh.cartesian(shape, (0, 0), (10, 10))
        U0 = W.project_cartesian(W.vortex_fields(0.0, G14), shape, (0, 0), (10, 10))
        U1, _ = oracle.run(m, U0, 0, G14, 0.3, "weno", t_end=1.0)
        ex = W.project_cartesian(W.vortex_fields(1.0, G14), shape, (0, 0), (10, 10),
                                 nq=6).reshape(12, -1)[0]
        errs.append(np.abs(U1.reshape(12, -1)[0] - ex).mean())
    assert min(_order(errs)) >= 1.8, (errs, _order(errs))
    errs = []
    for n in [16, 32, 64]:
        U0 = W.acoustic_state(n, axis=1)
        m = oracle.Mesh.cartesian((2, n), (0, 0), (1, 1))
        U1, _ = oracle.run(m, U0, 0, G53, 0.3, "weno", t_end=1.0)
        errs.append(np.abs(U1.reshape(12, -1)[0] - U0.reshape(12, -1)[0]).mean())
    assert min(_order(errs)) >= 1.7, (errs, _order(errs))


def test_sod_converges(oracle):
    """The paper's Sod tube on a periodic [-1, 1] (left state for |x| < 1/2),
    WENO limiter and the exact flux (the paper's moving-DG defaults), t = 0.2:
    the L1 density distance to a 1024-cell run falls with resolution."""
    def run(n):
        h = 2.0 / n
        x = -1.0 + h * (np.arange(n) + 0.5)
        U = np.zeros((12, n))
        U[0] = np.where(np.abs(x) < 0.5, 1.0, 0.25)
        U[9] = np.where(np.abs(x) < 0.5, 1.0, 0.1795) / (G14 - 1)
        m = oracle.Mesh.cartesian((n, 1), (-1.0, 0.0), (1.0, h))
        U1, _ = oracle.run(m, U.reshape(-1), 0, G14, 0.3, "weno", t_end=0.2, flux="exact")
        return U1.reshape(12, n)[0]
    fine = run(1024)
    errs = []
    for n in [64, 128, 256]:
        coarse = fine.reshape(n, -1).mean(1)
        errs.append(np.abs(run(n) - coarse).mean())
    assert errs[-1] < 0.01 and min(_order(errs)) > 0.5, (errs, _order(errs))
