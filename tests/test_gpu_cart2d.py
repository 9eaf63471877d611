"""GPU parity of the 2D Euler Cartesian path against the CPU oracle (through the C ABI).

Tolerances: single calls agree to 1e-12 of the field scale (different rounding
order only); 100-step runs to 1e-11 relative per field, with the per-field error
err_k = max_e max(|d mean_k|, h |d grad_k|_inf) / max_e |mean_k|.
"""
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


def field_errors(A, B, n, lo, hi, nvar=4, U=None):
    """Per-field relative error of A against the reference B (means and h-scaled
    gradients, normalised by the largest mean of the field).  With U given the
    arguments are right-hand sides L(U), whose natural size is max|U| c / h
    over all conserved fields (c ~ 1 here), and that is the scale."""
    dim = len(n)
    h = min((hi[d] - lo[d]) / n[d] for d in range(dim))
    A = A.reshape(nvar * (1 + dim), -1)
    B = B.reshape(nvar * (1 + dim), -1)
    Us = None if U is None else U.reshape(nvar * (1 + dim), -1)
    errs = []
    for v in range(nvar):
        k = v * (1 + dim)
        scale = max(np.abs(B[k]).max(), 1e-300)
        if Us is not None:
            scale = max(scale, np.abs(Us[0::1 + dim]).max() / h)
        d = np.abs(A[k] - B[k]).max()
        for c in range(1, 1 + dim):
            d = max(d, h * np.abs(A[k + c] - B[k + c]).max())
        errs.append(d / scale)
    return np.array(errs)


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


SHAPES = [(100, 70), (61, 9), (1, 5), (3, 1), (130, 4), (64, 64)]


@pytest.mark.parametrize("n", SHAPES)
def test_rhs_matches_oracle(oracle, torch_cuda, n):
    lo, hi = (0.0, -0.5), (1.3, 1.0)
    U0 = W.random_p1_state(n, lo, hi, G14, seed=hash(n) % 1000, amp=0.25)
    s = _solver(n, lo, hi, G14, limiter=False)
    got = s.rhs(s.to_device(U0)).cpu().numpy()
    s.check()
    ref = oracle.rhs(oracle.Mesh.cartesian(n, lo, hi), U0, G14)
    # The gradient equations subtract O(|F|) surface and volume sums that are
    # then scaled by 12/(V h^2): compare gradients in the h-scaled norm.
    errs = field_errors(got, ref, n, lo, hi, U=U0)
    assert errs.max() < 1e-13, (n, errs)


@pytest.mark.parametrize("n", SHAPES)
def test_limit_matches_oracle(oracle, torch_cuda, n):
    lo, hi = (0.0, 0.0), (1.0, 2.0)
    U0 = W.random_p1_state(n, lo, hi, G14, seed=3, amp=0.3).reshape(12, -1)
    U0[1::3] *= 4.0  # steep gradients so the limiter is active
    U0[2::3] *= -3.0
    U0 = U0.reshape(-1)
    s = _solver(n, lo, hi, G14)
    got = s.limit(s.to_device(U0)).cpu().numpy()
    ref = oracle.limit(oracle.Mesh.cartesian(n, lo, hi), U0)
    assert _rel(got, ref) < 1e-13
    assert np.array_equal(got.reshape(12, -1)[0::3], U0.reshape(12, -1)[0::3])


@pytest.mark.parametrize("limiter", [False, True])
@pytest.mark.parametrize("n", [(100, 70), (61, 9), (2, 3)])
def test_step_matches_oracle(oracle, torch_cuda, n, limiter):
    lo, hi = (0.0, 0.0), (1.0, 1.0)
    U0 = W.random_p1_state(n, lo, hi, G53, seed=5, amp=0.3)
    om = oracle.Mesh.cartesian(n, lo, hi)
    dt = oracle.cfl_dt(om, U0, G53, 0.3)
    ref = oracle.step(om, U0, dt, G53, limiter)
    s = _solver(n, lo, hi, G53, limiter=limiter)
    got = s.step(s.to_device(U0), dt).cpu().numpy()
    s.check()
    assert field_errors(got, ref, n, lo, hi).max() < 1e-13


def test_step_is_composition_of_limit_and_rhs(torch_cuda):
    """dg_step equals Ua = Pi(U); V1 = Ua + dt L(Ua); Ub = Pi(V1);
    U' = Ua/2 + (Ub + dt L(Ub))/2 built from dg_limit and dg_rhs."""
    n, lo, hi = (90, 33), (0.0, 0.0), (1.0, 1.0)
    U0 = W.random_p1_state(n, lo, hi, G53, seed=8, amp=0.3)
    s = _solver(n, lo, hi, G53, limiter=True)
    s_nolim = _solver(n, lo, hi, G53, limiter=False)
    U = s.to_device(U0)
    dt = 1e-3
    Ua = s.limit(U)
    V1 = Ua + dt * s_nolim.rhs(Ua)
    Ub = s.limit(V1)
    comp = 0.5 * Ua + 0.5 * (Ub + dt * s_nolim.rhs(Ub))
    got = s.step(U, dt)
    assert _rel(got.cpu().numpy(), comp.cpu().numpy()) < 1e-14


def test_c1_vortex_100_steps(oracle, torch_cuda):
    """The 64x64 isentropic vortex (gamma 1.4, no limiter), 100 steps on the
    oracle's CFL-0.3 dt schedule: 1e-11 relative per field."""
    n, lo, hi = (64, 64), (0.0, 0.0), (10.0, 10.0)
    U0 = W.c1_state(64)
    om = oracle.Mesh.cartesian(n, lo, hi)
    ref, dts = oracle.run(om, U0, 100, G14, 0.3, False)
    s = _solver(n, lo, hi, G14, limiter=False)
    U = s.to_device(U0)
    V = s.empty()
    for dt in dts:
        s.step(U, dt, out=V)
        U, V = V, U
    s.check()
    errs = field_errors(U.cpu().numpy(), ref, n, lo, hi)
    print("C1 FP64 per-field error after 100 steps:", errs)
    assert errs.max() < 1e-11


def test_c2_shear_100_steps_small(oracle, torch_cuda):
    """The shear-layer recipe (gamma 5/3, limiter on) at 128x128, 100 steps on
    the oracle's dt schedule."""
    n, lo, hi = (128, 128), (0.0, 0.0), (1.0, 1.0)
    U0 = W.c2_state(128)
    om = oracle.Mesh.cartesian(n, lo, hi)
    ref, dts = oracle.run(om, U0, 100, G53, 0.3, True)
    s = _solver(n, lo, hi, G53, limiter=True)
    U = s.to_device(U0)
    V = s.empty()
    for dt in dts:
        s.step(U, dt, out=V)
        U, V = V, U
    s.check()
    errs = field_errors(U.cpu().numpy(), ref, n, lo, hi)
    print("C2(128^2) FP64 per-field error after 100 steps:", errs)
    assert errs.max() < 1e-11
    # FP32 run on the same schedule: error stated per field
    s32 = _solver(n, lo, hi, G53, limiter=True, precision="fp32")
    U = s32.to_device(U0)
    V = s32.empty()
    for dt in dts:
        s32.step(U, dt, out=V)
        U, V = V, U
    s32.check()
    e32 = field_errors(U.double().cpu().numpy(), ref, n, lo, hi)
    print("C2(128^2) FP32 per-field error after 100 steps:", e32)
    assert e32.max() < 1e-3


def test_in_place_step_and_determinism(torch_cuda):
    n, lo, hi = (200, 37), (0.0, 0.0), (1.0, 1.0)
    U0 = W.random_p1_state(n, lo, hi, G53, seed=9, amp=0.3)
    s = _solver(n, lo, hi, G53)
    a = s.to_device(U0)
    b = s.step(a.clone(), 1e-3)
    c = s.step(a.clone(), 1e-3)
    assert torch_cuda.equal(b, c)
    s.step(a, 1e-3, out=a)
    assert torch_cuda.equal(a, b)


def test_cfl_dt_matches_oracle(oracle, torch_cuda):
    n, lo, hi = (77, 50), (0.0, 0.0), (2.0, 1.0)
    U0 = W.random_p1_state(n, lo, hi, G14, seed=10, amp=0.3)
    s = _solver(n, lo, hi, G14)
    dt = s.cfl_dt(s.to_device(U0), 0.3).item()
    ref = oracle.cfl_dt(oracle.Mesh.cartesian(n, lo, hi), U0, G14, 0.3)
    assert abs(dt - ref) <= 1e-14 * ref


def test_device_dt_step(oracle, torch_cuda):
    n, lo, hi = (64, 64), (0.0, 0.0), (1.0, 1.0)
    U0 = W.random_p1_state(n, lo, hi, G53, seed=12, amp=0.2)
    s = _solver(n, lo, hi, G53)
    U = s.to_device(U0)
    dt = s.cfl_dt(U, 0.3)
    a = s.step(U, dt)
    b = s.step(U, dt.item())
    assert torch_cuda.equal(a, b)


def test_nonphysical_state_is_reported(torch_cuda):
    from paper_1305_5536_amd.capi import NonPhysicalState
    n, lo, hi = (16, 16), (0.0, 0.0), (1.0, 1.0)
    U0 = W.random_p1_state(n, lo, hi, G14, seed=1, amp=0.1).reshape(12, -1)
    U0[0, 37] = -1.0  # negative density in one cell
    s = _solver(n, lo, hi, G14, limiter=False)
    s.rhs(s.to_device(U0.reshape(-1)))
    with pytest.raises(NonPhysicalState):
        s.check()
    s.check()  # the flag was cleared


def test_bad_arguments_are_rejected(torch_cuda):
    from paper_1305_5536_amd.capi import DGError
    s = _solver((8, 8), (0, 0), (1, 1), G14)
    with pytest.raises(ValueError):
        s.rhs(torch_cuda.zeros(10, dtype=torch_cuda.float64, device="cuda"))
    U = torch_cuda.ones(s.state_len, dtype=torch_cuda.float64, device="cuda")
    import ctypes
    from paper_1305_5536_amd import capi as C
    st = C.lib().dg_rhs(s._h, ctypes.c_void_p(U.data_ptr()), ctypes.c_void_p(U.data_ptr()), None)
    assert st == C.DG_EINVAL
    with pytest.raises(DGError):
        C.check(st, "dg_rhs")


def test_stages_with_device_dt_and_fused_cfl(oracle, torch_cuda):
    """dg_stage1 + dg_stage2 equal dg_step (the fused step kernel) to rounding;
    the fused CFL minimum of stage 2 equals dg_cfl_dt of the new state (and the
    oracle's)."""
    n, lo, hi = (150, 90), (0.0, 0.0), (1.0, 1.0)
    U0 = W.random_p1_state(n, lo, hi, G53, seed=13, amp=0.3)
    s = _solver(n, lo, hi, G53)
    U = s.to_device(U0)
    dt = s.cfl_dt(U, 0.3)
    V1 = s.empty()
    Un = s.empty()
    dt_next = torch_cuda.empty(1, dtype=torch_cuda.float64, device="cuda")
    s.stage1(U, dt, V1)
    s.stage2(U, V1, dt, Un, cfl=0.3, dt_next=dt_next)
    ref = s.step(U, dt.item())
    assert field_errors(Un.cpu().numpy(), ref.cpu().numpy(), n, lo, hi).max() < 1e-14
    assert dt_next.item() == s.cfl_dt(Un, 0.3).item()
    o = oracle.cfl_dt(oracle.Mesh.cartesian(n, lo, hi), Un.cpu().numpy(), G53, 0.3)
    assert abs(dt_next.item() - o) <= 1e-14 * o
    # dt_next may alias dt
    s.stage2(U, V1, dt, Un, cfl=0.3, dt_next=dt)
    assert dt.item() == dt_next.item()


def test_limiter_with_denormal_slopes(oracle, torch_cuda):
    """Nearly flat cells: slopes and mean differences in the denormal range.
    The limiter's D/dm stays finite and equals the oracle's (IEEE division)."""
    n, lo, hi = (16, 8), (0.0, 0.0), (1.0, 1.0)
    U = np.zeros((12, 128))
    U[0], U[9] = 1.0, 2.5
    rng = np.random.default_rng(8)
    for k in (1, 2, 4, 5, 7, 8, 10, 11):
        U[k] = rng.choice([0.0, 3e-310, -2e-312, 1e-300, 5e-320], 128)
    U[0] += rng.choice([0.0, 1e-16, 2.2e-16], 128)
    # a strictly rising x-momentum of denormal size: D / dm is a ratio of two
    # denormals (about 0.1)
    U[3] = np.tile(np.arange(16), 8) * 1e-312
    U[4] = 3e-310
    U0 = U.reshape(-1)
    s = _solver(n, lo, hi, G14)
    got = s.limit(s.to_device(U0)).cpu().numpy()
    ref = oracle.limit(oracle.Mesh.cartesian(n, lo, hi), U0)
    assert np.all(np.isfinite(got))
    # element-wise, with an absolute floor of a few thousand denormal ulps
    assert np.all(np.abs(got - ref) <= 1e-13 * np.abs(ref) + 1e-320)
    assert np.all(np.isfinite(s.step(s.to_device(U0), 1e-3).cpu().numpy()))
    s.check()


def test_results_do_not_depend_on_tiling(torch_cuda):
    """Every cell and face uses the same arithmetic whatever the rows per wave:
    outputs are bitwise identical across tilings (including ragged tiles)."""
    n, lo, hi = (130, 77), (0.0, 0.0), (1.0, 1.0)
    U0 = W.random_p1_state(n, lo, hi, G53, seed=14, amp=0.3)
    s = _solver(n, lo, hi, G53)
    U = s.to_device(U0)
    outs = []
    for rows in (1, 3, 7, 16, 77, 0):
        s.tiling = rows
        assert s.tiling == (rows if rows else s.tiling)
        outs.append((s.step(U, 1e-3), s.rhs(U)))
    for a, b in outs[1:]:
        assert torch_cuda.equal(a, outs[0][0])
        assert torch_cuda.equal(b, outs[0][1])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_tile_rows_environment_replaces_every_default(monkeypatch, torch_cuda, precision):
    """DG_TILE_ROWS replaces the library default of every Cartesian stage
    kernel (2D Euler, 2D MHD, 3D planes, batches) at creation and after tiling = 0; an
    explicit tiling still wins.  Results stay those of any other tiling."""
    from paper_1305_5536_amd.solver import Solver, batch, cartesian
    monkeypatch.setenv("DG_TILE_ROWS", "7")
    n2, n3 = (96, 40), (20, 9, 30)
    meshes = [
        (cartesian(n2, (0.0, 0.0), (1.0, 1.0)), "euler"),
        (cartesian(n2, (0.0, 0.0), (1.0, 1.0)), "mhd"),
        (cartesian(n3, (0.0,) * 3, (1.0,) * 3), "mhd"),
        (batch([(30, 20), (17, 9)]), "euler"),
    ]
    for mesh, physics in meshes:
        s = Solver(mesh, physics=physics, precision=precision, gamma=G53)
        assert s.tiling == 7, (physics, mesh)
        s.tiling = 5
        assert s.tiling == 5
        s.tiling = 0
        assert s.tiling == 7
    monkeypatch.delenv("DG_TILE_ROWS")
    s = _solver(n2, (0.0, 0.0), (1.0, 1.0), G53, precision=precision)
    default = s.tiling
    s.tiling = 7
    U = s.to_device(W.random_p1_state(n2, (0.0, 0.0), (1.0, 1.0), G53, seed=16, amp=0.2))
    a = s.step(U, 1e-3)
    s.tiling = 0
    assert s.tiling == default
    assert torch_cuda.equal(a, s.step(U, 1e-3))


def test_autotuner_picks_a_candidate(tmp_path, monkeypatch, torch_cuda):
    from paper_1305_5536_amd.autotune import autotune
    monkeypatch.setenv("DG_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    n, lo, hi = (256, 256), (0.0, 0.0), (1.0, 1.0)
    s = _solver(n, lo, hi, G53)
    U = s.to_device(W.random_p1_state(n, lo, hi, G53, seed=15, amp=0.2))
    r = autotune(s, U, n, candidates=(4, 8, 16), reps=3)
    assert r["rows"] in (4, 8, 16) and s.tiling == r["rows"]
    # second call hits the cache
    s.tiling = 0
    r2 = autotune(s, U, n, candidates=(4, 8, 16), reps=3)
    assert r2["rows"] == r["rows"] and s.tiling == r["rows"]


FUSED_SHAPES = [(1, 5), (3, 1), (2, 3), (61, 9), (57, 13), (113, 40), (130, 77), (224, 20)]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("limiter", [False, True])
@pytest.mark.parametrize("n", FUSED_SHAPES)
def test_fused_step_equals_two_stages(torch_cuda, n, limiter, precision):
    """On 2D Euler dg_step runs both stages in one kernel (stage-1 rows pass to
    stage 2 in registers; 56 output columns per wave; four extra stage-1 rows
    per strip).  It equals dg_stage1 + dg_stage2 to rounding (the same
    arithmetic; the compiler may contract the row update's products into FMAs
    differently: 1e-14 of the field scale in FP64, 1e-5 in FP32, where the
    face sums cancel to a few tens of ulps of the field scale), on meshes
    narrower than a wave, ragged strips and single rows, and dg_step_cfl's CFL
    step equals stage 2's to the same bound; in place it gives the same bits."""
    lo, hi = (0.0, 0.0), (1.0, 1.3)
    U0 = W.random_p1_state(n, lo, hi, G53, seed=n[0] * 1000 + n[1], amp=0.3)
    s = _solver(n, lo, hi, G53, limiter=limiter, precision=precision)
    U = s.to_device(U0)
    dt = s.cfl_dt(U, 0.3)
    V1, ref, got = s.empty(), s.empty(), s.empty()
    f64 = dict(dtype=torch_cuda.float64, device="cuda")
    d_ref, d_got = torch_cuda.empty(1, **f64), torch_cuda.empty(1, **f64)
    s.stage1(U, dt, V1)
    s.stage2(U, V1, dt, ref, cfl=0.3, dt_next=d_ref)
    s.step(U, dt, out=got, cfl=0.3, dt_next=d_got)
    s.check()
    tol = 1e-14 if precision == "fp64" else 1e-5
    errs = field_errors(got.double().cpu().numpy(), ref.double().cpu().numpy(), n, lo, hi)
    assert errs.max() < tol, errs
    assert abs(d_got.item() - d_ref.item()) <= tol * d_ref.item()
    # in place, with the next step size written over the current one
    s.step(U, dt, out=U, cfl=0.3, dt_next=dt)
    assert torch_cuda.equal(U, got) and dt.item() == d_got.item()


def test_fused_step_matches_oracle_over_strips_and_rows(oracle, torch_cuda):
    """A mesh of several 56-column strips with a ragged last strip and rows per
    wave that leave a short last tile: 20 fused steps against the oracle."""
    n, lo, hi = (150, 47), (0.0, 0.0), (1.5, 0.47)
    U0 = W.random_p1_state(n, lo, hi, G53, seed=31, amp=0.3)
    om = oracle.Mesh.cartesian(n, lo, hi)
    ref, dts = oracle.run(om, U0, 20, G53, 0.3, True)
    s = _solver(n, lo, hi, G53, limiter=True)
    s.tiling = 10
    U = s.to_device(U0)
    dt = torch_cuda.tensor([dts[0]], dtype=torch_cuda.float64, device="cuda")
    V = s.empty()
    for k in range(20):
        # the kernel's own CFL step drives the run; it must agree with the oracle's
        assert abs(dt.item() - dts[k]) <= 1e-13 * dts[k]
        dt.fill_(dts[k])
        s.step(U, dt, out=V, cfl=0.3, dt_next=dt)
        U, V = V, U
    s.check()
    errs = field_errors(U.cpu().numpy(), ref, n, lo, hi)
    assert errs.max() < 1e-12, errs


def test_fused_step_reports_nonphysical_state(torch_cuda):
    from paper_1305_5536_amd.capi import NonPhysicalState
    n, lo, hi = (70, 20), (0.0, 0.0), (1.0, 1.0)
    U0 = W.random_p1_state(n, lo, hi, G14, seed=2, amp=0.1).reshape(12, -1)
    s = _solver(n, lo, hi, G14, limiter=False)
    s.step(s.to_device(U0.reshape(-1)), 1e-4)
    s.check()  # a physical state raises nothing (halo lanes are masked)
    U0[9, 12 * 70 + 69] = -1.0  # negative energy in the last column of row 12
    s.step(s.to_device(U0.reshape(-1)), 1e-4)
    with pytest.raises(NonPhysicalState):
        s.check()


def test_run_two_stage_flag_steps_with_the_stage_pair(torch_cuda):
    """dg_run with DG_RUN_TWO_STAGE steps with the stage-1/stage-2 kernels: its
    states and step sizes equal those of stage1 + stage2 called one at a time
    and of the run that keeps the stage-1 outputs, bit for bit, graph-captured
    or not; the flag is refused together with MUSCL-Hancock."""
    from paper_1305_5536_amd import capi as C
    n, lo, hi = (70, 33), (0.0, 0.0), (1.0, 1.0)
    U0 = W.random_p1_state(n, lo, hi, G53, seed=35, amp=0.3)
    s = _solver(n, lo, hi, G53)
    U = s.to_device(U0)
    dt = s.cfl_dt(U, 0.3)
    A, V1, B = U.clone(), s.empty(), s.empty()
    for _ in range(5):
        s.stage1(A, dt, V1)
        s.stage2(A, V1, dt, B, cfl=0.3, dt_next=dt)
        A, B = B, A
    v1 = [s.empty() for _ in range(5)]
    kept, hist_kept = s.run(U, 5, cfl=0.3, v1_keep=v1, graph=False)
    for graph in (False, True, True):
        out, hist = s.run(U, 5, cfl=0.3, graph=graph, two_stage=True)
        torch_cuda.cuda.synchronize()
        assert torch_cuda.equal(out, A), graph
        assert torch_cuda.equal(out, kept), graph
        assert torch_cuda.equal(hist, hist_kept), graph
        assert hist[5].item() == dt.item(), graph
    with pytest.raises(C.DGError):
        s.run(U, 2, cfl=0.3, graph=False, two_stage=True, integrator="mh")
    s.check()


def test_run_uses_the_fused_step(torch_cuda):
    """dg_run on a 2D Euler mesh steps with the fused kernel (graph-captured,
    replayed twice) and equals dg_step_cfl one call at a time bit for bit, and
    the two-stage path that keeps the stage-1 outputs to rounding."""
    n, lo, hi = (90, 40), (0.0, 0.0), (1.0, 1.0)
    U0 = W.random_p1_state(n, lo, hi, G53, seed=33, amp=0.3)
    s = _solver(n, lo, hi, G53)
    U = s.to_device(U0)
    dt = s.cfl_dt(U, 0.3)
    A, B = U.clone(), s.empty()
    for _ in range(6):
        s.step(A, dt, out=B, cfl=0.3, dt_next=dt)
        A, B = B, A
    v1 = [s.empty() for _ in range(6)]
    two, hist2 = s.run(U, 6, cfl=0.3, v1_keep=v1, graph=False)
    out = s.empty()
    hist = torch_cuda.empty(7, dtype=torch_cuda.float64, device="cuda")
    for rep in range(3):  # capture, then two replays of the cached graph
        out.zero_()
        s.run(U, 6, cfl=0.3, out=out, dt_hist=hist, graph=True)
        torch_cuda.cuda.synchronize()
        assert torch_cuda.equal(out, A), rep
        assert hist[6].item() == dt.item(), rep
        assert field_errors(out.cpu().numpy(), two.cpu().numpy(), n, lo, hi).max() < 1e-13
        assert torch_cuda.allclose(hist, hist2, rtol=1e-13, atol=0)
    s.check()
