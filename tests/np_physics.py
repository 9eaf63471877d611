"""Textbook Euler and ideal-MHD physics in NumPy for the oracle pins.

Written from the conservation laws (Sec. 2.1) in units with mu0 = 1
(p_total = p + B^2/2, E = p/(gamma - 1) + rho v^2/2 + B^2/2), independently of
the oracle.  Works on complex arrays too, so complex-step derivatives of the
flux give its Jacobian to machine precision.
"""
import math

import numpy as np


def pressure(u, gamma, mhd):
    if mhd:
        rho, m, E, B = u[0], u[1:4], u[4], u[5:8]
        return (gamma - 1.0) * (E - 0.5 * (m @ m) / rho - 0.5 * (B @ B))
    dim = len(u) - 2
    rho, m, E = u[0], u[1:1 + dim], u[1 + dim]
    return (gamma - 1.0) * (E - 0.5 * (m @ m) / rho)


def flux(u, n, gamma, mhd):
    """Physical flux F(U) . n of the Euler or ideal-MHD equations."""
    p = pressure(u, gamma, mhd)
    if not mhd:
        dim = len(u) - 2
        rho, v = u[0], u[1:1 + dim] / u[0]
        nn = np.asarray(n)[:dim]
        vn = v @ nn
        return np.concatenate([[rho * vn], rho * v * vn + p * nn, [(u[1 + dim] + p) * vn]])
    rho, v, E, B = u[0], u[1:4] / u[0], u[4], u[5:8]
    n = np.asarray(n)
    vn, Bn = v @ n, B @ n
    pT = p + 0.5 * (B @ B)
    return np.concatenate([[rho * vn], rho * v * vn + pT * n - B * Bn,
                           [(E + pT) * vn - Bn * (v @ B)], B * vn - v * Bn])


def hll(uL, uR, n, gamma):
    """HLL with the Davis speed estimates (the Euler Riemann solver of the build)."""
    dim = len(uL) - 2
    nn = np.asarray(n)[:dim]
    FL, FR = flux(uL, n, gamma, False), flux(uR, n, gamma, False)
    vL, vR = uL[1:1 + dim] @ nn / uL[0], uR[1:1 + dim] @ nn / uR[0]
    cL = math.sqrt(gamma * pressure(uL, gamma, False) / uL[0])
    cR = math.sqrt(gamma * pressure(uR, gamma, False) / uR[0])
    SL, SR = min(vL - cL, vR - cR), max(vL + cL, vR + cR)
    if SL >= 0:
        return FL
    if SR <= 0:
        return FR
    return (SR * FL - SL * FR + SL * SR * (uR - uL)) / (SR - SL)


def flux_jacobian(u, n, gamma, mhd):
    """dF(U).n/dU by complex-step differentiation (exact to rounding)."""
    u = np.asarray(u, dtype=np.float64)
    k = len(u)
    J = np.zeros((k, k))
    h = 1e-30
    for j in range(k):
        uc = u.astype(np.complex128)
        uc[j] += 1j * h
        J[:, j] = flux(uc, n, gamma, mhd).imag / h
    return J


def mhd_state(rho, v, p, B, gamma):
    v, B = np.asarray(v, float), np.asarray(B, float)
    E = p / (gamma - 1.0) + 0.5 * rho * (v @ v) + 0.5 * (B @ B)
    return np.array([rho, *(rho * v), E, *B])


def euler_state(rho, v, p, gamma):
    v = np.asarray(v, float)
    return np.array([rho, *(rho * v), p / (gamma - 1.0) + 0.5 * rho * (v @ v)])
