"""GPU batched stepper: a batch of uneven 2D Euler instances must give, per
instance, exactly what a single-mesh handle gives (same arithmetic per cell,
so bit for bit), and agree with the oracle; dg_run (plain and hipGraph
replays, checkpoints, kept stage-1 outputs) must equal the step-by-step
launches."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

G53 = 5.0 / 3.0
SIZES = [(64, 64), (1, 5), (3, 1), (61, 9), (130, 4), (100, 70), (96, 128), (17, 33)]


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _states(sizes, seed0=300, amp=0.2, grad_scale=2.0):
    out = []
    for i, n in enumerate(sizes):
        U = W.random_p1_state(n, (0.0, 0.0), (1.0, 1.0), G53, seed=seed0 + i, amp=amp)
        U = U.reshape(12, -1).copy()
        U[1::3] *= grad_scale
        U[2::3] *= grad_scale
        out.append(U.reshape(-1))
    return out


def _batch(sizes, limiter=True, precision="fp64"):
    from paper_1305_5536_amd.solver import Solver, batch
    return Solver(batch(sizes), precision=precision, limiter=limiter, gamma=G53)


def _single(n, limiter=True, precision="fp64"):
    from paper_1305_5536_amd.solver import Solver, cartesian
    return Solver(cartesian(n, (0.0, 0.0), (1.0, 1.0)), precision=precision, limiter=limiter,
                  gamma=G53)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("limiter", [False, True])
def test_batch_equals_single_meshes(torch_cuda, limiter, precision):
    torch = torch_cuda
    states = _states(SIZES)
    b = _batch(SIZES, limiter, precision)
    U = b.pack(states)
    dtb = b.cfl_dt(U, 0.3)
    got = {"rhs": b.unpack(b.rhs(U)), "limit": b.unpack(b.limit(U)),
           "step": b.unpack(b.step(U, dtb))}
    V1, out, nxt = b.empty(), b.empty(), torch.empty_like(dtb)
    b.stage1(U, dtb, V1)
    b.stage2(U, V1, dtb, out, cfl=0.3, dt_next=nxt)
    got["stage2"] = b.unpack(out)
    b.check()
    for i, n in enumerate(SIZES):
        s = _single(n, limiter, precision)
        u = s.to_device(states[i])
        dt = s.cfl_dt(u, 0.3)
        assert dt.item() == dtb[i].item(), (n, dt.item(), dtb[i].item())
        # the single mesh's two stage kernels (its dg_step fuses both stages
        # into one kernel, equal to these to rounding only)
        v1, ref_step = s.empty(), s.empty()
        s.stage1(u, dt, v1)
        s.stage2(u, v1, dt, ref_step)
        assert np.array_equal(got["rhs"][i], s.rhs(u).double().cpu().numpy()), n
        assert np.array_equal(got["limit"][i], s.limit(u).double().cpu().numpy()), n
        assert np.array_equal(got["step"][i], ref_step.double().cpu().numpy()), n
        assert np.array_equal(got["stage2"][i], ref_step.double().cpu().numpy()), n
        assert nxt[i].item() == s.cfl_dt(ref_step, 0.3).item(), n


def test_batch_matches_oracle(oracle, torch_cuda):
    sizes = [(24, 20), (7, 31), (40, 12)]
    states = _states(sizes, seed0=500)
    b = _batch(sizes)
    U = b.pack(states)
    dts = []
    refs = []
    for i, n in enumerate(sizes):
        om = oracle.Mesh.cartesian(n, (0.0, 0.0), (1.0, 1.0))
        dts.append(oracle.cfl_dt(om, states[i], G53, 0.3))
        refs.append(oracle.step(om, states[i], dts[i], G53, True))
    dt = torch_cuda.tensor(dts, dtype=torch_cuda.float64, device=b.device)
    got = b.unpack(b.step(U, dt))
    for i in range(len(sizes)):
        scale = np.abs(refs[i].reshape(12, -1)[0::3]).max()
        assert np.abs(got[i] - refs[i]).max() < 1e-13 * scale


@pytest.mark.parametrize("wpb,grid", [(1, 0), (2, 0), (4, 7), (1, 1000), (2, 33)])
def test_launch_shape_does_not_change_results(torch_cuda, wpb, grid):
    states = _states(SIZES, seed0=600)
    b = _batch(SIZES)
    U = b.pack(states)
    dt = b.cfl_dt(U, 0.3)
    ref = b.step(U, dt)
    b.launch = (wpb, grid)
    assert b.launch == (wpb, grid)
    for rows in (1, 5, 64):
        b.tiling = rows
        assert torch_cuda.equal(b.step(U, dt), ref), (wpb, grid, rows)
        assert torch_cuda.equal(b.cfl_dt(U, 0.3), dt)


@pytest.mark.parametrize("graph", [False, True])
def test_run_equals_step_loop(torch_cuda, graph):
    torch = torch_cuda
    states = _states(SIZES, seed0=700)
    b = _batch(SIZES, precision="fp32")
    U0 = b.pack(states)
    nsteps = 9
    # step loop with the fused CFL of stage 2
    dt = b.cfl_dt(U0, 0.3)
    hist = [dt.clone()]
    U = U0.clone()
    V1, W2 = b.empty(), b.empty()
    for _ in range(nsteps):
        nxt = torch.empty_like(dt)
        b.stage1(U, dt, V1)
        b.stage2(U, V1, dt, W2, cfl=0.3, dt_next=nxt)
        U, W2 = W2, U
        dt = nxt
        hist.append(dt.clone())
    ref_hist = torch.cat(hist)
    ck = [b.empty() for _ in range((nsteps - 1) // 3)]
    v1k = [b.empty() for _ in range(nsteps)]
    for rep in range(3 if graph else 1):
        for c in ck + v1k:
            c.fill_(-1.0)  # eager work between replays
        out, dth = b.run(U0, nsteps, cfl=0.3, ckpt_every=3, ckpts=ck, v1_keep=v1k, graph=graph)
        torch.cuda.synchronize()
        assert torch.equal(out, U), rep
        assert torch.equal(dth, ref_hist), rep
        # checkpoints: the states after steps 3 and 6; v1_keep[n] = stage 1 of step n
        Uc = U0.clone()
        for n in range(nsteps):
            V = b.empty()
            b.stage1(Uc, dth[n * b.ninst:(n + 1) * b.ninst], V)
            assert torch.equal(V, v1k[n]), (rep, n)
            Uc = b.step(Uc, dth[n * b.ninst:(n + 1) * b.ninst])
            if (n + 1) % 3 == 0 and n + 1 < nsteps:
                assert torch.equal(Uc, ck[(n + 1) // 3 - 1]), (rep, n)
    # fixed-step replay of the recorded history gives the same final state
    out2, _ = b.run(U0, nsteps, cfl=0.0, dt_hist=dth[:nsteps * b.ninst].clone(), graph=graph)
    assert torch.equal(out2, U)
    b.check()


def test_run_on_other_mesh_kinds(torch_cuda):
    """dg_run on a single 2D mesh, a 3D MHD mesh and a Voronoi mesh equals the
    step loop with the same step sizes."""
    torch = torch_cuda
    from paper_1305_5536_amd.solver import Solver, cartesian
    from workloads.voronoi import periodic_voronoi, random_voronoi_state
    cases = []
    s2 = _single((50, 40))
    cases.append((s2, s2.to_device(_states([(50, 40)])[0])))
    s3 = Solver(cartesian((8, 6, 5), (0, 0, 0), (1, 1, 1)), physics="mhd", gamma=G53)
    U3 = W.random_p1_state((8, 6, 5), (0, 0, 0), (1, 1, 1), G53, seed=3, amp=0.1, mhd=True)
    cases.append((s3, s3.to_device(U3)))
    m = periodic_voronoi(400, seed=4)
    sv = Solver(m, gamma=G53)
    cases.append((sv, sv.to_device(random_voronoi_state(m, G53, seed=5, amp=0.2))))
    for s, U0 in cases:
        out, dth = s.run(U0, 4, cfl=0.3, graph=True)
        U = U0.clone()
        for n in range(4):
            U = s.step(U, dth[n:n + 1])
        assert torch.equal(out, U)
        s.check()


def test_batch_adjoint_equals_single(torch_cuda):
    states = _states(SIZES, seed0=800)
    b = _batch(SIZES)
    U = b.pack(states)
    dt = b.cfl_dt(U, 0.3)
    rng = np.random.default_rng(3)
    lams = [rng.standard_normal(s.size) for s in states]
    got = b.unpack(b.adjoint_step(U, dt, b.pack(lams)))
    for i, n in enumerate(SIZES):
        s = _single(n)
        ref = s.adjoint_step(s.to_device(states[i]), dt[i].item(), s.to_device(lams[i]))
        assert np.array_equal(got[i], ref.cpu().numpy()), n


def test_batch_arguments(torch_cuda):
    from paper_1305_5536_amd.capi import DGError
    from paper_1305_5536_amd.solver import Solver, batch
    with pytest.raises(DGError):
        Solver(batch([(4, 4), (0, 3)]), gamma=G53)
    b = _batch([(8, 8), (5, 9)])
    with pytest.raises(DGError):
        b.launch = (3, 0)
    U = b.pack(_states([(8, 8), (5, 9)]))
    with pytest.raises(DGError):
        b.run(U, 1, cfl=0.3, out=U)


def test_batch_autotuner(torch_cuda, tmp_path, monkeypatch):
    from paper_1305_5536_amd import autotune
    monkeypatch.setenv("DG_AUTOTUNE_CACHE", str(tmp_path / "tune.json"))
    sizes = [(64, 64), (96, 96), (130, 40)]
    b = _batch(sizes, precision="fp32")
    U = b.pack(_states(sizes, seed0=900))
    e = autotune.autotune_batch(b, U, sizes, reps=2)
    assert e["rows"] in autotune.BATCH_ROWS and e["wpb"] in autotune.BATCH_WPB
    assert e["grid"] in autotune.BATCH_GRID
    assert b.tiling == e["rows"] and b.launch == (e["wpb"], e["grid"])
    b2 = _batch(sizes, precision="fp32")
    assert autotune.autotune_batch(b2, U, sizes)["rows"] == e["rows"]  # from the cache
    assert b2.launch == (e["wpb"], e["grid"])


def test_batch_handle_entry_points(torch_cuda, tmp_path):
    """dg_batch_create / offset / run / adjoint_step / destroy through the C ABI:
    a batch built from single meshes computes exactly what a batch mesh
    (kind 2) of the same instances computes, with and without a launch file."""
    import ctypes
    from paper_1305_5536_amd import capi as C
    from paper_1305_5536_amd.solver import _stream
    torch = torch_cuda
    lib = C.lib()
    sizes = [(64, 64), (61, 9), (100, 70), (17, 33), (3, 1)]
    states = _states(sizes, seed0=700)
    singles = [_single(n) for n in sizes]
    ref = _batch(sizes)
    hs = (ctypes.c_void_p * len(sizes))(*[s._h.value for s in singles])
    launch = tmp_path / "launch.txt"
    launch.write_text("8 2 2048\n")
    for cache in (None, str(launch).encode()):
        bh = ctypes.c_void_p()
        assert lib.dg_batch_create(hs, len(sizes), cache, ctypes.byref(bh)) == C.DG_OK, \
            C.last_error()
        try:
            assert lib.dg_batch_mesh(bh) is not None
            for i in range(len(sizes) + 1):
                assert lib.dg_batch_offset(bh, i) == ref.offsets[i]
            assert lib.dg_batch_offset(bh, len(sizes) + 1) == -1
            for nsteps in (1, 3):
                U0 = ref.pack(states)
                U = U0.clone()
                hist = torch.empty((nsteps + 1) * len(sizes), dtype=torch.float64,
                                   device=U.device)
                assert lib.dg_batch_run(bh, U.data_ptr(), 0.3, hist.data_ptr(), nsteps,
                                        _stream()) == C.DG_OK, C.last_error()
                want, want_hist = ref.run(U0, nsteps, cfl=0.3)
                torch.cuda.synchronize()
                assert torch.equal(U, want), nsteps
                assert torch.equal(hist, want_hist), nsteps
            U = ref.pack(states)
            dt = ref.cfl_dt(U, 0.3)
            lam = torch.randn_like(U)
            got = torch.empty_like(U)
            assert lib.dg_batch_adjoint_step(bh, U.data_ptr(), dt.data_ptr(), lam.data_ptr(),
                                             got.data_ptr(), _stream()) == C.DG_OK
            assert torch.equal(got, ref.adjoint_step(U, dt, lam))
            assert lib.dg_check(lib.dg_batch_mesh(bh)) == C.DG_OK
        finally:
            lib.dg_batch_destroy(bh)
    # malformed launch file, mixed configurations, wrong mesh kinds
    bad = tmp_path / "bad.txt"
    bad.write_text("eight\n")
    bh = ctypes.c_void_p()
    assert lib.dg_batch_create(hs, len(sizes), str(bad).encode(), ctypes.byref(bh)) == C.DG_EINVAL
    assert not bh.value
    other = _single((8, 8), limiter=False)
    mixed = (ctypes.c_void_p * 2)(singles[0]._h.value, other._h.value)
    assert lib.dg_batch_create(mixed, 2, None, ctypes.byref(bh)) == C.DG_EINVAL
    assert lib.dg_batch_create(hs, 0, None, ctypes.byref(bh)) == C.DG_EINVAL
    for s in singles + [other]:
        s.close()
    ref.close()
