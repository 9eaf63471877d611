"""GPU discrete adjoint of the 2D Euler step on a static face-list (periodic
Voronoi) mesh against the oracle (HLL, the limiter of Sec. 2.5 or none).

The oracle differentiates its own step forward with dual numbers (J v); the GPU
adjoint gives J^T w.  Entry by entry, (J^T w)_i = <J e_i, w>: every entry on a
12-cell mesh (cells with repeated neighbours across the periodic box), a
sample on larger meshes, per kind of coefficient (means, gradients); the
dot-product test on 5000 cells; a central difference of the limiter-free step.
"""
import numpy as np
import pytest

from workloads.voronoi import periodic_voronoi, random_voronoi_state

pytestmark = pytest.mark.gpu

G53 = 5.0 / 3.0


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def meshes():
    return {n: periodic_voronoi(n, seed=61) for n in (12, 40, 300, 5000)}


def _solver(mesh, limiter=True, precision="fp64"):
    from paper_1305_5536_amd.solver import Solver
    return Solver(mesh, precision=precision, limiter=limiter, gamma=G53)


def _state(mesh, seed, grad_scale=3.0):
    """Smooth random state with steepened gradients, so that the limiter acts
    on part of the cells."""
    U = random_voronoi_state(mesh, G53, seed=seed, amp=0.2).reshape(12, -1).copy()
    U[1::3] *= grad_scale
    U[2::3] *= grad_scale
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


@pytest.mark.parametrize("limiter", [False, True])
@pytest.mark.parametrize("n", [12, 40, 300])
def test_facelist_adjoint_entries_match_oracle(oracle, torch_cuda, meshes, n, limiter):
    m = meshes[n]
    om = oracle.Mesh.facelist(m)
    U0 = _state(m, seed=300 + n)
    if limiter:
        assert (oracle.limit(om, U0) != U0).any()  # the limiter acts somewhere
    dt = oracle.cfl_dt(om, U0, G53, 0.3)
    rng = np.random.default_rng(n)
    w = rng.standard_normal(U0.size)
    s = _solver(m, limiter=limiter)
    lam = s.adjoint_step(s.to_device(U0), dt, s.to_device(w)).cpu().numpy()
    s.check()
    idx = np.arange(U0.size) if U0.size <= 500 else rng.choice(U0.size, 150, replace=False)
    ref = _columns(oracle, om, U0, dt, limiter, idx, w)
    got, want = np.zeros(U0.size), np.zeros(U0.size)
    got[idx], want[idx] = lam[idx], ref
    err = _rel_by_kind(got, want)
    print(f"face-list adjoint, {n} cells, limiter {limiter}: {len(idx)} entries, "
          f"max error by kind {err:.2e}")
    assert err < 1e-12, err


@pytest.mark.parametrize("limiter", [False, True])
def test_facelist_adjoint_dot_product(oracle, torch_cuda, meshes, limiter):
    """<J v, w> (oracle) = <v, J^T w> (GPU) on 5000 cells, three directions."""
    m = meshes[5000]
    om = oracle.Mesh.facelist(m)
    U0 = _state(m, seed=71)
    dt = oracle.cfl_dt(om, U0, G53, 0.3)
    rng = np.random.default_rng(73)
    s = _solver(m, limiter=limiter)
    U = s.to_device(U0)
    for _ in range(3):
        v = rng.standard_normal(U0.size)
        w = rng.standard_normal(U0.size)
        _, Jv = oracle.step_jvp(om, U0, v, dt, G53, limiter)
        lam = s.adjoint_step(U, dt, s.to_device(w)).cpu().numpy()
        a, b = Jv @ w, v @ lam
        assert abs(a - b) <= 1e-12 * np.abs(Jv * w).sum(), (a, b)
    s.check()


def test_facelist_adjoint_central_difference_and_fp32(torch_cuda, meshes):
    """Limiter off: a central difference of the GPU step (eps 1e-6) agrees with
    the adjoint to its truncation error; a given stage-1 output gives the same
    bits as the recomputed one; the FP32 adjoint's error is stated."""
    m = meshes[300]
    U0 = _state(m, seed=79, grad_scale=1.0)
    s = _solver(m, limiter=False)
    U = s.to_device(U0)
    dt = s.cfl_dt(U, 0.3).item()
    rng = np.random.default_rng(83)
    v = s.to_device(rng.standard_normal(U0.size) * np.abs(U0))
    w = s.to_device(rng.standard_normal(U0.size))
    eps = 1e-6
    fd = float(((s.step(U + eps * v, dt) - s.step(U - eps * v, dt)) * w).sum()) / (2 * eps)
    ad = float((s.adjoint_step(U, dt, w) * v).sum())
    print(f"face-list central difference {fd:.12e} vs adjoint {ad:.12e}")
    assert abs(fd - ad) <= 1e-7 * abs(ad)
    sl = _solver(m)
    U = sl.to_device(_state(m, seed=89))
    V1 = sl.empty()
    sl.stage1(U, dt, V1)
    a = sl.adjoint_step(U, dt, w, V1=V1)
    assert torch_cuda.equal(a, sl.adjoint_step(U, dt, w))
    s32 = _solver(m, precision="fp32")
    c = s32.adjoint_step(s32.to_device(U.cpu().numpy()), dt,
                         s32.to_device(w.cpu().numpy())).double().cpu().numpy()
    err = _rel_by_kind(c, a.cpu().numpy())
    print(f"face-list adjoint FP32 vs FP64, max relative error by kind: {err:.2e}")
    assert err < 1e-2
