"""GPU discrete adjoint of the 2D Euler Cartesian step against the oracle.

The oracle differentiates its own step forward with dual numbers (J v).  The
GPU adjoint gives J^T w.  Element by element, (J^T w)_i = <J e_i, w>, so every
sampled entry is checked against one oracle JVP of a unit vector.  Entries are
normalised per kind (means, gradients), whose adjoints differ by a factor h.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

G53 = 5.0 / 3.0
LO, HI = (0.0, 0.0), (1.0, 1.0)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _solver(n, limiter=True, precision="fp64"):
    from paper_1305_5536_amd.solver import Solver, cartesian
    return Solver(cartesian(n, LO, HI), precision=precision, limiter=limiter, gamma=G53)


def _state(n, seed, grad_scale=3.0, drift=0.0):
    """Smooth random state with steepened gradients (so that the limiter acts on
    part of the cells) and an optional uniform x drift (supersonic faces)."""
    U = W.random_p1_state(n, LO, HI, G53, seed=seed, amp=0.2).reshape(12, -1).copy()
    U[1::3] *= grad_scale
    U[2::3] *= grad_scale
    if drift:
        rho, mx, my, E = U[0], U[3], U[6], U[9]
        E_new = E + drift * mx + 0.5 * drift * drift * rho
        gE = (U[10] + drift * U[4] + 0.5 * drift * drift * U[1],
              U[11] + drift * U[5] + 0.5 * drift * drift * U[2])
        U[3] = mx + drift * rho
        U[4] = U[4] + drift * U[1]
        U[5] = U[5] + drift * U[2]
        U[9], U[10], U[11] = E_new, gE[0], gE[1]
    return U.reshape(-1)


def _rel_by_kind(a, b):
    a = a.reshape(4, 3, -1)
    b = b.reshape(4, 3, -1)
    em = np.abs(a[:, 0] - b[:, 0]).max() / max(np.abs(b[:, 0]).max(), 1e-300)
    eg = np.abs(a[:, 1:] - b[:, 1:]).max() / max(np.abs(b[:, 1:]).max(), 1e-300)
    return max(em, eg)


def _columns(oracle, om, U, dt, limiter, idx, w):
    out = np.empty(len(idx))
    for j, i in enumerate(idx):
        e = np.zeros_like(U)
        e[i] = 1.0
        _, Je = oracle.step_jvp(om, U, e, dt, G53, limiter)
        out[j] = Je @ w
    return out


def _sample(ncells, n, rng, count=96):
    """All entries when small, else a sample that includes the last row and
    column of cells (the ragged tile tail) and every coefficient."""
    ndof = 12 * ncells
    if ndof <= 720:
        return np.arange(ndof)
    nx, ny = n
    tail = [(ny - 1) * nx + x for x in range(nx)] + [y * nx + nx - 1 for y in range(ny)]
    cells = np.concatenate([rng.choice(tail, count // 2), rng.integers(0, ncells, count // 2)])
    ks = rng.integers(0, 12, count)
    return ks * ncells + cells


@pytest.mark.parametrize("limiter", [False, True])
@pytest.mark.parametrize("n", [(8, 6), (40, 36), (17, 33), (1, 5), (3, 1)])
def test_adjoint_entries_match_oracle(oracle, torch_cuda, n, limiter):
    ncells = n[0] * n[1]
    om = oracle.Mesh.cartesian(n, LO, HI)
    U0 = _state(n, seed=100 + n[0])
    if limiter and ncells >= 48:
        assert (oracle.limit(om, U0) != U0).any()  # the limiter acts somewhere
    dt = oracle.cfl_dt(om, U0, G53, 0.3)
    rng = np.random.default_rng(7)
    w = rng.standard_normal(12 * ncells)
    s = _solver(n, limiter=limiter)
    lam = s.adjoint_step(s.to_device(U0), dt, s.to_device(w)).cpu().numpy()
    s.check()
    idx = _sample(ncells, n, rng)
    ref = _columns(oracle, om, U0, dt, limiter, idx, w)
    full_ref = np.zeros(12 * ncells)
    full_got = np.zeros(12 * ncells)
    full_ref[idx] = ref
    full_got[idx] = lam[idx]
    err = _rel_by_kind(full_got, full_ref)
    assert err < 1e-12, err


@pytest.mark.parametrize("limiter", [False, True])
def test_adjoint_supersonic_faces(oracle, torch_cuda, limiter):
    """A uniform x drift of Mach ~1.6 makes every x face take the upwind branch
    of HLL (S_L >= 0), the y faces the two-wave branch."""
    n = (24, 20)
    om = oracle.Mesh.cartesian(n, LO, HI)
    U0 = _state(n, seed=5, drift=2.0)
    dt = oracle.cfl_dt(om, U0, G53, 0.3)
    rng = np.random.default_rng(8)
    w = rng.standard_normal(U0.size)
    s = _solver(n, limiter=limiter)
    lam = s.adjoint_step(s.to_device(U0), dt, s.to_device(w)).cpu().numpy()
    idx = _sample(n[0] * n[1], n, rng)
    ref = _columns(oracle, om, U0, dt, limiter, idx, w)
    a, b = np.zeros_like(lam), np.zeros_like(lam)
    a[idx], b[idx] = lam[idx], ref
    assert _rel_by_kind(a, b) < 1e-12


@pytest.mark.parametrize("limiter", [False, True])
def test_adjoint_dot_product(oracle, torch_cuda, limiter):
    """<J v, w> (oracle, dual numbers) = <v, J^T w> (GPU) on a mesh of 7 x 5
    adjoint tiles with ragged edges, for three random directions."""
    n = (100, 70)
    om = oracle.Mesh.cartesian(n, LO, HI)
    U0 = _state(n, seed=11)
    dt = oracle.cfl_dt(om, U0, G53, 0.3)
    rng = np.random.default_rng(9)
    s = _solver(n, limiter=limiter)
    U = s.to_device(U0)
    for _ in range(3):
        v = rng.standard_normal(U0.size)
        w = rng.standard_normal(U0.size)
        _, Jv = oracle.step_jvp(om, U0, v, dt, G53, limiter)
        lam = s.adjoint_step(U, dt, s.to_device(w)).cpu().numpy()
        a, b = Jv @ w, v @ lam
        assert abs(a - b) <= 1e-12 * max(np.abs(Jv * w).sum(), 1e-300), (a, b)


@pytest.mark.parametrize("limiter,grad_scale", [(False, 1.0), (True, 3.0)])
def test_adjoint_central_difference(torch_cuda, limiter, grad_scale):
    """Central difference of <w, S(U)> in FP64 through the GPU forward step.
    The step is only piecewise smooth (the limiter's branches, the min/max of
    the wave speeds), so the difference step is small (1e-7 of each entry),
    and the error is measured against sum_i |v_i lam_i|, the size of the terms
    of the inner product (which cancel heavily for a random w)."""
    n = (64, 48)
    U0 = _state(n, seed=12, grad_scale=grad_scale)
    s = _solver(n, limiter=limiter)
    U = s.to_device(U0)
    dt = s.cfl_dt(U, 0.3).item()
    rng = np.random.default_rng(10)
    v = rng.standard_normal(U0.size) * np.abs(U0)
    w = s.to_device(rng.standard_normal(U0.size))
    lam = s.adjoint_step(U, dt, w).cpu().numpy()
    g = float(v @ lam)
    scale = float(np.abs(v * lam).sum())
    eps = 1e-7

    def J(x):
        return float((s.step(s.to_device(x), dt) * w).sum())

    fd = (J(U0 + eps * v) - J(U0 - eps * v)) / (2 * eps)
    assert abs(fd - g) <= 1e-8 * scale, (fd, g, scale)


def test_adjoint_fp32_error_stated(torch_cuda):
    n = (64, 48)
    U0 = _state(n, seed=13)
    rng = np.random.default_rng(11)
    w = rng.standard_normal(U0.size)
    s64, s32 = _solver(n), _solver(n, precision="fp32")
    dt = s64.cfl_dt(s64.to_device(U0), 0.3).item()
    a = s64.adjoint_step(s64.to_device(U0), dt, s64.to_device(w)).cpu().numpy()
    b = s32.adjoint_step(s32.to_device(U0), dt, s32.to_device(w)).double().cpu().numpy()
    err = _rel_by_kind(b, a)
    print("FP32 adjoint step, relative error by kind vs FP64:", err)
    assert err < 1e-4


def test_adjoint_given_v1_is_bitwise_recompute(torch_cuda):
    n = (40, 36)
    U0 = _state(n, seed=14)
    s = _solver(n)
    U = s.to_device(U0)
    dt = s.cfl_dt(U, 0.3).item()
    w = s.to_device(np.random.default_rng(12).standard_normal(U0.size))
    V1 = s.empty()
    s.stage1(U, dt, V1)
    a = s.adjoint_step(U, dt, w, V1=V1)
    b = s.adjoint_step(U, dt, w)
    assert torch_cuda.equal(a, b)


def test_adjoint_argument_errors(torch_cuda):
    from paper_1305_5536_amd.capi import DGError
    from paper_1305_5536_amd.solver import Solver, cartesian
    n = (16, 16)
    s = _solver(n)
    U = s.to_device(_state(n, seed=15))
    with pytest.raises(DGError):
        s.adjoint_step(U, 1e-3, U, out=U)
    # not built: the exact Riemann solver
    sx = Solver(cartesian(n, LO, HI), gamma=G53, flux="exact")
    with pytest.raises(DGError):
        sx.adjoint_step(sx.to_device(_state(n, seed=15)), 1e-3, sx.empty().fill_(0.0))
