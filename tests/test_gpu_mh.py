"""GPU MUSCL-Hancock step (dg_step_mh, Sec. 2.4) against the oracle's, through
the C ABI: single steps on ragged meshes, 100-step runs on the oracle's step
schedule, batches, graph-captured runs, and the unsupported mesh kinds."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

G14 = 1.4
G53 = 5.0 / 3.0


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _solver(n, lo, hi, gamma, limiter=True, precision="fp64"):
    from paper_1305_5536_amd.solver import Solver, cartesian
    return Solver(cartesian(n, lo, hi), precision=precision, limiter=limiter, gamma=gamma)


def field_errors(A, B, h):
    """err_k = max(|d mean_k|, h |d grad_k|) / max|mean_k| (scale floored at the
    density scale)."""
    A = A.reshape(12, -1)
    B = B.reshape(12, -1)
    out = []
    for v in range(4):
        k = 3 * v
        scale = max(np.abs(B[k]).max(), np.abs(B[0]).max())
        d = max(np.abs(A[k] - B[k]).max(), h * np.abs(A[k + 1:k + 3] - B[k + 1:k + 3]).max())
        out.append(d / scale)
    return np.array(out)


@pytest.mark.parametrize("limiter", [False, True])
@pytest.mark.parametrize("n", [(100, 70), (61, 9), (1, 5), (3, 1), (130, 4)])
def test_mh_step_matches_oracle(oracle, torch_cuda, n, limiter):
    lo, hi = (0.0, 0.0), (1.0, 1.0)
    U0 = W.random_p1_state(n, lo, hi, G53, seed=70 + n[0], amp=0.3).reshape(12, -1).copy()
    U0[1::3] *= 2.0
    U0[2::3] *= 2.0
    U0 = U0.reshape(-1)
    om = oracle.Mesh.cartesian(n, lo, hi)
    dt = oracle.cfl_dt(om, U0, G53, 0.3)
    ref = oracle.step_mh(om, U0, dt, G53, limiter)
    s = _solver(n, lo, hi, G53, limiter)
    got = s.step_mh(s.to_device(U0), dt).cpu().numpy()
    s.check()
    h = min((hi[0] - lo[0]) / n[0], (hi[1] - lo[1]) / n[1])
    assert field_errors(got, ref, h).max() < 1e-13


def test_mh_vortex_100_steps(oracle, torch_cuda):
    """C1 recipe (vortex 64^2, no limiter) with the MUSCL-Hancock integrator:
    100 steps on the oracle's schedule agree to 1e-11 per field."""
    n, lo, hi = (64, 64), (0.0, 0.0), (10.0, 10.0)
    U0 = W.c1_state(64)
    om = oracle.Mesh.cartesian(n, lo, hi)
    ref, dts = oracle.run(om, U0, 100, G14, 0.3, False, integrator="mh")
    for prec, tol in (("fp64", 1e-11), ("fp32", 1e-4)):
        s = _solver(n, lo, hi, G14, limiter=False, precision=prec)
        U = s.to_device(U0)
        V = s.empty()
        for dt in dts:
            s.step_mh(U, dt, out=V)
            U, V = V, U
        s.check()
        e = field_errors(U.double().cpu().numpy(), ref, 10.0 / 64)
        print(f"MUSCL-Hancock vortex 64^2 {prec}, 100 steps, per-field error: {e}")
        assert e.max() < tol, (prec, e)


def test_mh_shear_100_steps_small(oracle, torch_cuda):
    """C2 recipe at 128^2 (limiter on) with the MUSCL-Hancock integrator."""
    n, lo, hi = (128, 128), (0.0, 0.0), (1.0, 1.0)
    U0 = W.c2_state(128)
    om = oracle.Mesh.cartesian(n, lo, hi)
    ref, dts = oracle.run(om, U0, 100, G53, 0.3, True, integrator="mh")
    for prec, tol in (("fp64", 1e-11), ("fp32", 1e-3)):
        s = _solver(n, lo, hi, G53, precision=prec)
        U = s.to_device(U0)
        V = s.empty()
        for dt in dts:
            s.step_mh(U, dt, out=V)
            U, V = V, U
        s.check()
        e = field_errors(U.double().cpu().numpy(), ref, 1.0 / 128)
        print(f"MUSCL-Hancock shear 128^2 {prec}, 100 steps, per-field error: {e}")
        assert e.max() < tol, (prec, e)


def test_mh_sod_100_steps(oracle, torch_cuda):
    """The paper's Sod tube (Sec. 3.2) along x on a periodic [-1, 1] (left
    state for |x| < 1/2), HLL, limiter on: 100 steps on the oracle's schedule.
    Ahead of the rarefactions the slopes decay into the denormal range, where
    the limiter's ratio D/dm must stay finite."""
    n = 256
    h = 2.0 / n
    x = -1.0 + h * (np.arange(n) + 0.5)
    U = np.zeros((12, n))
    U[0] = np.where(np.abs(x) < 0.5, 1.0, 0.25)
    U[9] = np.where(np.abs(x) < 0.5, 1.0, 0.1795) / (G14 - 1.0)
    U0 = U.reshape(-1)
    om = oracle.Mesh.cartesian((n, 1), (-1.0, 0.0), (1.0, h))
    ref, dts = oracle.run(om, U0, 100, G14, 0.3, True, integrator="mh")
    s = _solver((n, 1), (-1.0, 0.0), (1.0, h), G14)
    Ug = s.to_device(U0)
    V = s.empty()
    for dt in dts:
        s.step_mh(Ug, dt, out=V)
        Ug, V = V, Ug
    s.check()
    e = field_errors(Ug.cpu().numpy(), ref, h)
    assert e.max() < 1e-11, e


def test_mh_fused_cfl_and_graph_run(torch_cuda):
    torch = torch_cuda
    n, lo, hi = (96, 80), (0.0, 0.0), (1.0, 1.0)
    U0 = W.random_p1_state(n, lo, hi, G53, seed=77, amp=0.3)
    s = _solver(n, lo, hi, G53)
    U = s.to_device(U0)
    dt = s.cfl_dt(U, 0.3)
    hist = [dt.clone()]
    Uc = U.clone()
    for _ in range(6):
        nxt = torch.empty_like(dt)
        Uc = s.step_mh(Uc, dt, cfl=0.3, dt_next=nxt)
        assert nxt.item() == s.cfl_dt(Uc, 0.3).item()
        dt = nxt
        hist.append(dt.clone())
    for graph in (False, True):
        out, dth = s.run(U, 6, cfl=0.3, graph=graph, integrator="mh")
        assert torch.equal(out, Uc)
        assert torch.equal(dth, torch.cat(hist))
    s.check()


def test_mh_batch_equals_single(torch_cuda):
    from paper_1305_5536_amd.solver import Solver, batch
    sizes = [(64, 64), (17, 33), (130, 4), (1, 5)]
    states = [W.random_p1_state(n, (0, 0), (1, 1), G53, seed=80 + i, amp=0.3)
              for i, n in enumerate(sizes)]
    b = Solver(batch(sizes), gamma=G53)
    U = b.pack(states)
    dt = b.cfl_dt(U, 0.3)
    got = b.unpack(b.step_mh(U, dt))
    for i, n in enumerate(sizes):
        s = _solver(n, (0, 0), (1, 1), G53)
        ref = s.step_mh(s.to_device(states[i]), dt[i].item()).cpu().numpy()
        assert np.array_equal(got[i], ref), n


def test_mh_unsupported_meshes(torch_cuda):
    from paper_1305_5536_amd.capi import DGError
    from paper_1305_5536_amd.solver import Solver, cartesian
    s3 = Solver(cartesian((4, 4, 4), (0, 0, 0), (1, 1, 1)), physics="mhd", gamma=G53)
    with pytest.raises(DGError):
        s3.step_mh(s3.empty().fill_(1.0), 1e-3)
    s = _solver((8, 8), (0, 0), (1, 1), G53)
    U = s.to_device(W.random_p1_state((8, 8), (0, 0), (1, 1), G53, seed=1))
    with pytest.raises(DGError):
        s.step_mh(U, 1e-3, out=U)
