"""Pins of the oracle's 2D ideal MHD (Sec. 2.2: the 2D locally divergence-free
basis V1..V5 for (B_x, B_y), B_z in the Taylor basis; HLLD on in-plane
normals).

* the Gram matrix of V3..V5 is the paper's printed 3x3 mass matrix;
* a uniform state is stationary; conserved totals are constant;
* projecting a linear divergence-free field recovers its coefficients
  exactly, and every cell polynomial is divergence-free;
* the Stokes divergence of a projected smooth field falls as h^2;
* the circularly polarised Alfven wave (an exact nonlinear solution with
  in-plane and out-of-plane field) converges at second order.
"""
import math

import numpy as np
import pytest

import workloads as W

G53 = 5.0 / 3.0


def _order(errs, ns):
    return [math.log(errs[i] / errs[i + 1]) / math.log(ns[i + 1] / ns[i])
            for i in range(len(errs) - 1)]


def test_gram_matches_printed_matrix(oracle):
    rng = np.random.default_rng(1)
    for _ in range(4):
        A = rng.normal(size=(2, 2))
        M = A @ A.T + 0.1 * np.eye(2)   # int x x^T over a cell: symmetric positive
        mxx, mxy, myy = M[0, 0], M[0, 1], M[1, 1]
        G = oracle.gram_B2(M)
        printed = np.array([[myy, 0.0, mxy], [0.0, mxx, -mxy], [mxy, -mxy, mxx + myy]])
        assert np.allclose(G[:3, :3], printed, rtol=0, atol=1e-14)
        assert np.allclose(G[3:, 3:], M, rtol=0, atol=1e-14)
        assert np.abs(G[:3, 3:]).max() == 0.0


def test_free_stream_and_conservation(oracle):
    n = (9, 7)
    m = oracle.Mesh.cartesian(n, (0.0, 0.0), (1.0, 0.7))
    U = np.zeros((23, 63))
    U[0], U[3], U[6], U[9], U[12] = 1.2, 0.3, -0.2, 0.1, 3.0
    U[15], U[16], U[17] = 0.4, -0.3, 0.2
    L = oracle.rhs(m, U.reshape(-1), G53, mhd=True)
    assert np.abs(L).max() < 1e-11
    U = W.random_p1_state(n, (0.0, 0.0), (1.0, 0.7), G53, seed=2, amp=0.2, mhd=True)
    V = 0.7 / 63
    A = U.reshape(23, -1)
    tot0 = np.concatenate([A[0:15:3], A[15:18]]).sum(1) * V
    ref = np.abs(np.concatenate([A[0:15:3], A[15:18]])).sum(1) * V
    for _ in range(8):
        U = oracle.step(m, U, 0.002, G53, True, mhd=True)
    A = U.reshape(23, -1)
    tot1 = np.concatenate([A[0:15:3], A[15:18]]).sum(1) * V
    assert np.all(np.abs(tot1 - tot0) <= 1e-13 * np.maximum(ref, 1e-300) + 1e-16)


def test_linear_divergence_free_field_is_exact(oracle):
    """B = (b + a1 y + a3 x, c + a2 x - a3 y, d + e x + f y) lies in the span of
    the basis: its projection returns the coefficients, and the cell
    polynomials carry zero divergence (dB_x/dx = a3 = -dB_y/dy)."""
    a1, a2, a3, bz_x, bz_y = 0.3, -0.7, 0.45, 0.2, -0.1

    def f(X, Y):
        B = [0.5 + a1 * (Y - 0.5) + a3 * (X - 0.5), -0.2 + a2 * (X - 0.5) - a3 * (Y - 0.5),
             0.1 + bz_x * (X - 0.5) + bz_y * (Y - 0.5)]
        return W.cartesian._mhd_conserved(1.0 + 0.0 * X, [0.0 * X] * 3, 1.0 + 0.0 * X, B, G53)

    U = W.project_cartesian(f, (6, 5), (0.0, 0.0), (1.0, 1.0), mhd=True).reshape(23, -1)
    assert np.allclose(U[18], a1, atol=1e-13)
    assert np.allclose(U[19], a2, atol=1e-13)
    assert np.allclose(U[20], a3, atol=1e-13)
    assert np.allclose(U[21], bz_x, atol=1e-13)
    assert np.allclose(U[22], bz_y, atol=1e-13)


def test_stokes_divergence_second_order(oracle):
    """(1/V) sum_faces B_n A of a projected smooth solenoidal field (the face
    average of both extrapolations) falls at second order."""
    errs, ns = [], [24, 48, 96]
    for n in ns:
        U = W.random_p1_state((n, n), (0.0, 0.0), (1.0, 1.0), G53, seed=3, amp=0.1, mhd=True,
                              bamp=0.05)
        m = oracle.Mesh.cartesian((n, n), (0.0, 0.0), (1.0, 1.0))
        errs.append(np.abs(oracle.divB(m, U)).mean())
    orders = _order(errs, ns)
    assert min(orders) >= 1.8, (errs, orders)


def test_alfven_wave_2d_second_order(oracle):
    """After half a period the exact solution is the initial one shifted by
    half a wavelength; the L1 error of the out-of-plane field B_z falls at
    second order."""
    ns = [16, 32, 64]
    errs = []
    T = 1.0 / math.sqrt(2)
    for n in ns:
        U0 = W.alfven2d_state(n)
        m = oracle.Mesh.cartesian((n, n), (0.0, 0.0), (1.0, 1.0))
        U1, _ = oracle.run(m, U0, 0, G53, 0.3, False, mhd=True, t_end=0.5 * T)
        ex = W.alfven2d_state(n, t=0.5 * T)
        errs.append(np.abs(U1.reshape(23, -1)[17] - ex.reshape(23, -1)[17]).mean())
    orders = _order(errs, ns)
    assert min(orders) >= 1.8, (errs, orders)


def test_orszag_tang_runs_and_conserves(oracle):
    """The paper's Orszag-Tang setup advances with the limiter on, stays
    physical and conserves mass, momentum, energy and mean field.  (The
    rotor's disc edge, a 10:1 density jump spun at Mach ~2, gives negative
    pressure at quadrature points under the conserved-variable limiter in the
    first stage: the method has no positivity safeguard, so it is not run.)"""
    n = 32
    U = W.orszag_tang_state(n)
    m = oracle.Mesh.cartesian((n, n), (0.0, 0.0), (1.0, 1.0))
    A0 = U.reshape(23, -1)
    tot0 = np.concatenate([A0[0:15:3], A0[15:18]]).sum(1)
    U1, dts = oracle.run(m, U, 20, G53, 0.3, True, mhd=True)
    A1 = U1.reshape(23, -1)
    tot1 = np.concatenate([A1[0:15:3], A1[15:18]]).sum(1)
    scale = np.abs(np.concatenate([A0[0:15:3], A0[15:18]])).sum(1)
    assert np.all(np.abs(tot1 - tot0) <= 1e-12 * np.maximum(scale, 1.0))
    assert np.all(np.isfinite(U1)) and len(dts) == 20
