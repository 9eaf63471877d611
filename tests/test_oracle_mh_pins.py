"""Pins of the oracle's MUSCL-Hancock integrator (Sec. 2.4): the half-step
primitive prediction and the one-pass update.

* exact advected isentropic vortex and the paper's acoustic wave: second-order
  convergence of the density means;
* free-stream preservation and conservation over limited steps;
* with zero gradients the prediction is the identity (no time derivative), so
  the step reduces to the forward-Euler update with the semi-discrete operator
  (an independently pinned routine);
* the primitive gradients equal numerical derivatives of the conserved-to-
  primitive map along the cell's linear conserved field;
* the predicted time derivative equals the exact time derivative of the
  isentropic vortex's primitive fields at a point (finite differences in time
  of the exact solution).
"""
import math

import numpy as np
import pytest

import workloads as W

G14 = 1.4
G53 = 5.0 / 3.0


def _order(errs, ns):
    return [math.log(errs[i] / errs[i + 1]) / math.log(ns[i + 1] / ns[i])
            for i in range(len(errs) - 1)]


@pytest.mark.parametrize("vel,aspect", [((1.0, 1.0), 1), ((1.0, -0.5), 2)])
def test_mh_vortex_second_order(oracle, vel, aspect):
    ns = [16, 32, 64]
    errs = []
    for n in ns:
        shape = (n, n * aspect)
        m = oracle.Mesh.cartesian(shape, (0, 0), (10, 10))
        U0 = W.project_cartesian(W.vortex_fields(0.0, G14, vel=vel), shape, (0, 0), (10, 10))
        U1, _ = oracle.run(m, U0, 0, G14, 0.3, False, t_end=1.0, integrator="mh")
        ex = W.project_cartesian(W.vortex_fields(1.0, G14, vel=vel), shape, (0, 0), (10, 10),
                                 nq=6).reshape(12, -1)[0]
        errs.append(np.abs(U1.reshape(12, -1)[0] - ex).mean())
    orders = _order(errs, ns)
    assert min(orders) >= 1.8, (errs, orders)


@pytest.mark.parametrize("axis", [0, 1])
def test_mh_acoustic_wave_second_order(oracle, axis):
    ns = [16, 32, 64]
    errs = []
    for n in ns:
        U0 = W.acoustic_state(n, axis=axis)
        shape = (n, 2) if axis == 0 else (2, n)
        m = oracle.Mesh.cartesian(shape, (0, 0), (1, 1))
        U1, _ = oracle.run(m, U0, 0, G53, 0.3, False, t_end=1.0, integrator="mh")
        errs.append(np.abs(U1.reshape(12, -1)[0] - U0.reshape(12, -1)[0]).mean())
    orders = _order(errs, ns)
    assert min(orders) >= 1.8, (errs, orders)


def test_mh_free_stream_and_conservation(oracle):
    n = (12, 10)
    m = oracle.Mesh.cartesian(n, (0, 0), (1, 1))
    U = np.zeros((12, 120))
    U[0], U[3], U[6], U[9] = 1.3, 0.4, -0.2, 2.5
    U1 = oracle.step_mh(m, U.reshape(-1), 0.01, G14, True).reshape(12, -1)
    assert np.abs(U1 - U).max() < 1e-14
    U = W.random_p1_state(n, (0, 0), (1, 1), G14, seed=4, amp=0.3)
    V = 1.0 / 120
    tot0 = U.reshape(12, -1)[0::3].sum(1) * V
    ref = np.abs(U.reshape(12, -1)[0::3]).sum(1) * V
    for _ in range(10):
        U = oracle.step_mh(m, U, 0.004, G14, True)
    tot1 = U.reshape(12, -1)[0::3].sum(1) * V
    assert np.all(np.abs(tot1 - tot0) <= 1e-13 * ref)


def test_mh_zero_gradients_reduce_to_forward_euler(oracle):
    """Piecewise-constant data: no time derivative in the prediction, so the
    step is U + dt L(U) with the semi-discrete operator (up to the rounding of
    the conserved -> primitive -> conserved round trip)."""
    n = (9, 7)
    m = oracle.Mesh.cartesian(n, (0, 0), (1, 1))
    U = W.random_p1_state(n, (0, 0), (1, 1), G14, seed=5, amp=0.3).reshape(12, -1).copy()
    U[1::3] = 0.0
    U[2::3] = 0.0
    U = U.reshape(-1)
    dt = 0.002
    got = oracle.step_mh(m, U, dt, G14, False)
    ref = U + dt * oracle.rhs(m, U, G14)
    scale = np.abs(ref.reshape(12, -1)[0::3]).max()
    assert np.abs(got - ref).max() < 1e-13 * scale


def _prim(u, gamma):
    rho = u[0]
    v = u[1:-1] / rho
    p = (gamma - 1.0) * (u[-1] - 0.5 * rho * (v * v).sum())
    return np.concatenate([[rho], v, [p]])


@pytest.mark.parametrize("dim", [2, 3])
def test_predicted_gradients_are_derivatives_of_the_primitive_map(oracle, dim):
    rng = np.random.default_rng(6 + dim)
    for _ in range(5):
        rho = rng.uniform(0.5, 2.0)
        v = rng.uniform(-1, 1, dim)
        p = rng.uniform(0.5, 2.0)
        mean = np.concatenate([[rho], rho * v, [p / (G53 - 1) + 0.5 * rho * (v * v).sum()]])
        grad = rng.uniform(-1, 1, (dim + 2, dim))
        w, gw = oracle.predict_prim(mean, grad, G53, 0.0)
        assert np.allclose(w, _prim(mean, G53), rtol=0, atol=1e-14)
        h = 1e-6
        for d in range(dim):
            fd = (_prim(mean + h * grad[:, d], G53) - _prim(mean - h * grad[:, d], G53)) / (2 * h)
            assert np.allclose(gw[:, d], fd, rtol=1e-7, atol=1e-8), (d, gw[:, d], fd)


def test_predicted_time_derivative_matches_exact_vortex(oracle):
    """At points of the advected isentropic vortex, (w(h) - w(0)) / h of the
    prediction (computed from the exact point values and gradients) equals
    the exact time derivative of the primitive fields."""
    vel = (0.7, -0.4)
    f0 = W.vortex_fields(0.0, G14, vel=vel)

    def cons(t, x, y):
        return np.array(W.vortex_fields(t, G14, vel=vel)(np.array([x]), np.array([y])))[:, 0]

    for (x, y) in [(5.3, 4.6), (4.1, 5.9), (6.0, 5.2)]:
        u = cons(0.0, x, y)
        e = 1e-6
        grad = np.stack([(cons(0.0, x + e, y) - cons(0.0, x - e, y)) / (2 * e),
                         (cons(0.0, x, y + e) - cons(0.0, x, y - e)) / (2 * e)], axis=1)
        w0, _ = oracle.predict_prim(u, grad, G14, 0.0)
        hstep = 1e-3
        w1, _ = oracle.predict_prim(u, grad, G14, hstep)
        dwdt = (w1 - w0) / hstep
        te = 1e-5
        exact = (_prim(cons(te, x, y), G14) - _prim(cons(-te, x, y), G14)) / (2 * te)
        assert np.allclose(dwdt, exact, rtol=1e-5, atol=1e-7), (dwdt, exact)
    del f0
