"""dg_cfl_dt_static, the CFL step for callers that cannot allocate: through the
C ABI it gives dg_cfl_dt's result bit for bit on two calls in a row (the second
on a smaller mesh, so the shared static array holds the first call's partials),
refuses meshes above its static limit and other mesh kinds."""
import ctypes

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

G53 = 5.0 / 3.0


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_static_cfl_matches_cfl(torch_cuda, precision):
    torch = torch_cuda
    from paper_1305_5536_amd import capi as C
    from paper_1305_5536_amd.solver import Solver, _stream, cartesian
    lib = C.lib()
    for n, seed in (((300, 260), 3), ((64, 48), 4)):  # the second call is smaller
        s = Solver(cartesian(n, (0.0, 0.0), (1.0, 0.7)), precision=precision, gamma=G53)
        U = s.to_device(W.random_p1_state(n, (0.0, 0.0), (1.0, 0.7), G53, seed=seed, amp=0.3))
        want = s.cfl_dt(U, 0.3)
        got = torch.full((1,), -1.0, dtype=torch.float64, device=U.device)
        st = lib.dg_cfl_dt_static(s._h, U.data_ptr(), 0.3, got.data_ptr(), _stream())
        assert st == C.DG_OK, C.last_error()
        torch.cuda.synchronize()
        print(f"{precision} {n}: static {got.item()!r} handle {want.item()!r}")
        assert got.item() == want.item(), (n, got.item(), want.item())
        s.check()
        s.close()


def test_static_cfl_limits(torch_cuda):
    torch = torch_cuda
    from paper_1305_5536_amd import capi as C
    from paper_1305_5536_amd.solver import Solver, _stream, batch, cartesian
    lib = C.lib()
    dt = torch.zeros(1, dtype=torch.float64, device="cuda")
    # 2^25 + 5792 cells: one row of cells above the limit
    big = Solver(cartesian((5792, 5794), (0.0, 0.0), (1.0, 1.0)), precision="fp32", gamma=G53)
    assert big.ncells > 1 << 25
    assert lib.dg_cfl_dt_static(big._h, dt.data_ptr(), 0.3, dt.data_ptr(), _stream()) == \
        C.DG_EINVAL
    assert b"static scratch limit" in lib.dg_last_error()
    big.close()
    b = Solver(batch([(8, 8), (4, 4)]), precision="fp64", gamma=G53)
    assert lib.dg_cfl_dt_static(b._h, dt.data_ptr(), 0.3, dt.data_ptr(), _stream()) == \
        C.DG_EUNSUPPORTED
    b.close()
    assert dt.item() == 0.0
