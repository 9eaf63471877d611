"""GPU parity of the 2D Euler face-list (static Voronoi) path against the oracle."""
import math

import numpy as np
import pytest

from workloads.voronoi import c4_state, periodic_voronoi, random_voronoi_state

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
    return {n: periodic_voronoi(n, seed=21) for n in (12, 300, 5000)}


def _solver(mesh, limiter=True, precision="fp64"):
    from paper_1305_5536_amd.solver import Solver
    return Solver(mesh, precision=precision, limiter=limiter, gamma=G53)


def field_errors(A, B, mesh, U=None):
    """Per-field error; each field's scale is floored at the density scale so
    that fields that vanish in exact arithmetic (the momentum of a state at
    rest) are not measured as roundoff over roundoff."""
    h = math.sqrt(mesh["cell_volume"].min())
    A = A.reshape(12, -1)
    B = B.reshape(12, -1)
    errs = []
    for v in range(4):
        k = 3 * v
        scale = max(np.abs(B[k]).max(), np.abs(B[0]).max())
        if U is not None:
            scale = max(scale, np.abs(U.reshape(12, -1)[0::3]).max() / h)
        d = max(np.abs(A[k] - B[k]).max(), h * np.abs(A[k + 1:k + 3] - B[k + 1:k + 3]).max())
        errs.append(d / scale)
    return np.array(errs)


@pytest.mark.parametrize("n", [12, 300, 5000])
def test_rhs_matches_oracle(oracle, torch_cuda, meshes, n):
    m = meshes[n]
    U0 = random_voronoi_state(m, G53, seed=n, amp=0.2)
    s = _solver(m, limiter=False)
    got = s.rhs(s.to_device(U0)).cpu().numpy()
    s.check()
    ref = oracle.rhs(oracle.Mesh.facelist(m), U0, G53)
    errs = field_errors(got, ref, m, U=U0)
    assert errs.max() < 1e-13, errs


@pytest.mark.parametrize("n", [12, 300, 5000])
def test_limit_matches_oracle(oracle, torch_cuda, meshes, n):
    m = meshes[n]
    U0 = random_voronoi_state(m, G53, seed=n + 1, amp=0.3).reshape(12, -1)
    U0[1::3] *= 4.0
    U0[2::3] *= -3.0
    U0 = U0.reshape(-1)
    s = _solver(m)
    got = s.limit(s.to_device(U0)).cpu().numpy()
    ref = oracle.limit(oracle.Mesh.facelist(m), U0)
    assert np.abs(got - ref).max() <= 1e-13 * np.abs(ref).max()


@pytest.mark.parametrize("limiter", [False, True])
@pytest.mark.parametrize("n", [300, 5000])
def test_step_matches_oracle(oracle, torch_cuda, meshes, n, limiter):
    m = meshes[n]
    om = oracle.Mesh.facelist(m)
    U0 = random_voronoi_state(m, G53, seed=7, amp=0.3)
    dt = oracle.cfl_dt(om, U0, G53, 0.3)
    ref = oracle.step(om, U0, dt, G53, limiter)
    s = _solver(m, limiter=limiter)
    U = s.to_device(U0)
    got = s.step(U, dt).cpu().numpy()
    s.check()
    assert field_errors(got, ref, m).max() < 1e-13
    V1, out = s.empty(), s.empty()
    s.stage1(U, dt, V1)
    s.stage2(U, V1, dt, out)
    assert torch_cuda.equal(out, s.step(U, dt))


def test_cfl_matches_oracle(oracle, torch_cuda, meshes):
    m = meshes[300]
    U0 = random_voronoi_state(m, G53, seed=9, amp=0.3)
    s = _solver(m)
    U = s.to_device(U0)
    dt = s.cfl_dt(U, 0.3).item()
    ref = oracle.cfl_dt(oracle.Mesh.facelist(m), U0, G53, 0.3)
    assert abs(dt - ref) <= 1e-13 * ref
    V1, out = s.empty(), s.empty()
    nxt = torch_cuda.empty(1, dtype=torch_cuda.float64, device="cuda")
    s.stage1(U, dt, V1)
    s.stage2(U, V1, dt, out, cfl=0.3, dt_next=nxt)
    assert nxt.item() == s.cfl_dt(out, 0.3).item()


def test_c4_recipe_100_steps_small(oracle, torch_cuda):
    """The C4 recipe (Gaussian density bump at rest, limiter on) on a 20k-cell
    Lloyd-relaxed Voronoi mesh: 100 steps on the oracle's dt schedule agree to
    1e-11 per field; the FP32 error is stated."""
    m = periodic_voronoi(20000, seed=1004)
    U0 = c4_state(m)
    om = oracle.Mesh.facelist(m)
    ref, dts = oracle.run(om, U0, 100, G53, 0.3, True)
    for prec, tol in (("fp64", 1e-11), ("fp32", 1e-3)):
        s = _solver(m, precision=prec)
        U = s.to_device(U0)
        V = s.empty()
        for dt in dts:
            s.step(U, dt, out=V)
            U, V = V, U
        s.check()
        errs = field_errors(U.double().cpu().numpy(), ref, m)
        print(f"C4(20k cells) {prec} per-field error after 100 steps:", errs)
        assert errs.max() < tol, (prec, errs)


def test_dynamic_state_100_steps(oracle, torch_cuda):
    """A moving smooth random state on a 5000-cell Voronoi mesh, limiter on:
    100 steps on the oracle's dt schedule agree to 1e-11 per field."""
    m = periodic_voronoi(5000, seed=33)
    U0 = random_voronoi_state(m, G53, seed=34, amp=0.3)
    om = oracle.Mesh.facelist(m)
    ref, dts = oracle.run(om, U0, 100, G53, 0.3, True)
    s = _solver(m)
    U = s.to_device(U0)
    V = s.empty()
    for dt in dts:
        s.step(U, dt, out=V)
        U, V = V, U
    s.check()
    errs = field_errors(U.cpu().numpy(), ref, m)
    print("Voronoi 5000 cells, moving state, FP64 per-field error after 100 steps:", errs)
    assert errs.max() < 1e-11, errs


def test_bad_face_list_is_rejected(torch_cuda, meshes):
    from paper_1305_5536_amd.capi import DGError
    m = dict(meshes[12])
    m["face_area"] = m["face_area"].copy()
    m["face_area"][3] *= 1.5  # breaks the closure of two cells
    with pytest.raises(DGError):
        _solver(m)
