"""GPU discrete adjoint of the 2D ideal-MHD Cartesian step (HLLD flux on the
face-averaged normal field, the limiter of Sec. 2.5 with one alpha for B)
against the oracle.

The oracle differentiates its own step forward with dual numbers (J v); the GPU
adjoint gives J^T w.  Entry by entry, (J^T w)_i = <J e_i, w>, checked against
one oracle JVP of a unit vector per entry (every entry on meshes of a few
cells, including one-cell-wide directions where a cell is its own neighbour,
a sample on larger ones), per kind of coefficient (hydro means, hydro
gradients, field means, field linear coefficients).
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

G53 = 5.0 / 3.0
NC = 23
LO, HI = (0.0, 0.0), (1.0, 1.0)
KINDS = (list(range(0, 15, 3)), [k for k in range(15) if k % 3], [15, 16, 17],
         list(range(18, 23)))


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _solver(n, limiter=True, precision="fp64"):
    from paper_1305_5536_amd.solver import Solver, cartesian
    return Solver(cartesian(n, LO, HI), physics="mhd", precision=precision, limiter=limiter,
                  gamma=G53)


def _state(n, seed, grad_scale=2.5):
    """Smooth random MHD state with steepened hydro gradients and field
    coefficients, so that the limiter acts on part of the cells."""
    U = W.random_p1_state(n, LO, HI, G53, seed=seed, amp=0.3, mhd=True,
                          bamp=0.05).reshape(NC, -1).copy()
    for v in range(5):
        U[3 * v + 1:3 * v + 3] *= grad_scale
    U[18:] *= grad_scale
    return U.reshape(-1)


def _rel_by_kind(a, b):
    a = a.reshape(NC, -1)
    b = b.reshape(NC, -1)
    out = 0.0
    for ks in KINDS:
        scale = np.abs(b[ks]).max()
        if scale > 0:
            out = max(out, np.abs(a[ks] - b[ks]).max() / scale)
    return out


def _columns(oracle, om, U, dt, limiter, idx, w):
    out = np.empty(len(idx))
    for j, i in enumerate(idx):
        e = np.zeros_like(U)
        e[i] = 1.0
        _, Je = oracle.step_jvp(om, U, e, dt, G53, limiter, mhd=True)
        out[j] = Je @ w
    return out


def _sample(ncells, n, rng, count=120):
    ndof = NC * ncells
    if ndof <= 600:
        return np.arange(ndof)
    nx, ny = n
    tail = [(ny - 1) * nx + x for x in range(nx)] + [y * nx + nx - 1 for y in range(ny)]
    cells = np.concatenate([rng.choice(tail, count // 2), rng.integers(0, ncells, count // 2)])
    ks = rng.integers(0, NC, count)
    return ks * ncells + cells


@pytest.mark.parametrize("limiter", [False, True])
@pytest.mark.parametrize("n", [(4, 3), (1, 5), (3, 1), (2, 2), (12, 10)])
def test_mhd_adjoint_entries_match_oracle(oracle, torch_cuda, n, limiter):
    ncells = n[0] * n[1]
    om = oracle.Mesh.cartesian(n, LO, HI)
    U0 = _state(n, seed=200 + 7 * n[0] + n[1])
    if limiter and ncells >= 12:
        assert (oracle.limit(om, U0, mhd=True) != U0).any()  # the limiter acts somewhere
    dt = oracle.cfl_dt(om, U0, G53, 0.3, mhd=True)
    rng = np.random.default_rng(17)
    w = rng.standard_normal(NC * ncells)
    s = _solver(n, limiter=limiter)
    lam = s.adjoint_step(s.to_device(U0), dt, s.to_device(w)).cpu().numpy()
    s.check()
    idx = _sample(ncells, n, rng)
    ref = _columns(oracle, om, U0, dt, limiter, idx, w)
    got, want = np.zeros(NC * ncells), np.zeros(NC * ncells)
    got[idx], want[idx] = lam[idx], ref
    err = _rel_by_kind(got, want)
    print(f"2D MHD adjoint {n} limiter {limiter}: {len(idx)} entries, max error by kind {err:.2e}")
    assert err < 1e-12, err


@pytest.mark.parametrize("limiter", [False, True])
def test_mhd_adjoint_dot_product(oracle, torch_cuda, limiter):
    """<J v, w> (oracle, dual numbers) = <v, J^T w> (GPU) on a 40 x 30 mesh for
    three random directions."""
    n = (40, 30)
    om = oracle.Mesh.cartesian(n, LO, HI)
    U0 = _state(n, seed=31)
    dt = oracle.cfl_dt(om, U0, G53, 0.3, mhd=True)
    rng = np.random.default_rng(19)
    s = _solver(n, limiter=limiter)
    U = s.to_device(U0)
    for _ in range(3):
        v = rng.standard_normal(U0.size)
        w = rng.standard_normal(U0.size)
        _, Jv = oracle.step_jvp(om, U0, v, dt, G53, limiter, mhd=True)
        lam = s.adjoint_step(U, dt, s.to_device(w)).cpu().numpy()
        a, b = Jv @ w, v @ lam
        assert abs(a - b) <= 1e-12 * np.abs(Jv * w).sum(), (a, b)
    s.check()


def test_mhd_adjoint_central_difference(torch_cuda):
    """Without the limiter the step is smooth where no HLLD wave region
    changes: a central difference of the GPU step (eps 1e-6) agrees with the
    adjoint to the difference's truncation error."""
    n = (24, 20)
    U0 = _state(n, seed=37, grad_scale=1.0)
    s = _solver(n, limiter=False)
    U = s.to_device(U0)
    dt = s.cfl_dt(U, 0.3).item()
    rng = np.random.default_rng(23)
    v = s.to_device(rng.standard_normal(U0.size) * np.abs(U0))
    w = s.to_device(rng.standard_normal(U0.size))
    eps = 1e-6
    fd = float(((s.step(U + eps * v, dt) - s.step(U - eps * v, dt)) * w).sum()) / (2 * eps)
    ad = float((s.adjoint_step(U, dt, w) * v).sum())
    print(f"2D MHD central difference {fd:.12e} vs adjoint {ad:.12e}")
    assert abs(fd - ad) <= 1e-7 * abs(ad)


def test_mhd_adjoint_given_v1_and_fp32(torch_cuda):
    """A given stage-1 output gives the same bits as the recomputed one; the
    FP32 adjoint's error against FP64 is stated."""
    n = (30, 22)
    U0 = _state(n, seed=41)
    s = _solver(n)
    U = s.to_device(U0)
    dt = s.cfl_dt(U, 0.3).item()
    w = np.random.default_rng(29).standard_normal(U0.size)
    V1 = s.empty()
    s.stage1(U, dt, V1)
    a = s.adjoint_step(U, dt, s.to_device(w), V1=V1)
    b = s.adjoint_step(U, dt, s.to_device(w))
    assert torch_cuda.equal(a, b)
    s32 = _solver(n, precision="fp32")
    c = s32.adjoint_step(s32.to_device(U0), dt, s32.to_device(w)).double().cpu().numpy()
    err = _rel_by_kind(c, a.cpu().numpy())
    print(f"2D MHD adjoint FP32 vs FP64, max relative error by kind: {err:.2e}")
    assert err < 1e-2
