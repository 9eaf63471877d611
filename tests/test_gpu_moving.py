"""GPU moving Voronoi mesh (Sec. 2.3, 2D Euler, MUSCL-Hancock of Sec. 2.4) against
the oracle's moving mesh, through the C ABI (mesh kind 3, dg_step_mh):

* the mesh the GPU builds (walking each cell's faces among its previous 2-ring) against
  the oracle's (Delaunay circumcentres, rebuilt from scratch): the same neighbours,
  volumes and centroids; also after steps that change the topology;
* the limiters (Arepo, WENO-type) on the moving mesh;
* single steps with the generators moving and held still, HLL and exact fluxes,
  every limiter;
* 100 FP64 steps of the isentropic vortex, of a shear layer (WENO-type limiter and
  exact flux; also the Arepo limiter with HLL) and of the paper's Sod tube (shocks,
  contact, rarefactions) on the oracle's time-step schedule at 1e-11 per field (FP32
  error stated);
* the CFL step, conservation, and the refused calls and descriptors.
"""
import math

import numpy as np
import pytest

from workloads.cartesian import vortex_fields
from workloads.voronoi import periodic_voronoi, project_voronoi, random_voronoi_state

pytestmark = pytest.mark.gpu

G14 = 1.4
G53 = 5.0 / 3.0


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def mv(oracle):
    from oracle import moving
    return moving


def _solver(d, limiter="weno", flux="exact", gamma=G53, precision="fp64", motion=1):
    from paper_1305_5536_amd.solver import Solver, moving
    s = Solver(moving(d), precision=precision, limiter=limiter, gamma=gamma, flux=flux)
    if motion != 1:
        s.set_motion(motion)
    return s


def field_errors(A, B, h):
    A = A.reshape(12, -1)
    B = B.reshape(12, -1)
    out = []
    for v in range(4):
        k = 3 * v
        dd = max(np.abs(A[k] - B[k]).max(), h * np.abs(A[k + 1:k + 3] - B[k + 1:k + 3]).max())
        out.append(dd / max(np.abs(B[k]).max(), np.abs(B[0]).max()))
    return np.array(out)


def compare_mesh(geo, d, tol=1e-13):
    n = len(d["cell_volume"])
    box = np.asarray(d["box"])
    assert np.abs(geo["generators"] - d["generators"]).max() <= 1e-15 * box.max()
    assert np.abs(geo["volume"] - d["cell_volume"]).max() <= tol * d["cell_volume"].max()
    dc = geo["centroid"] - d["cell_centroid"]
    dc -= box * np.round(dc / box)
    assert np.abs(dc).max() <= tol * box.max()
    nb = [[] for _ in range(n)]
    for L, R in d["face_cells"]:
        nb[L].append(int(R))
        nb[R].append(int(L))
    for i in range(n):
        got = sorted(geo["ring"][i, :geo["degree"][i]].tolist())
        assert got == sorted(nb[i]), (i, got, sorted(nb[i]))


@pytest.mark.parametrize("n,lloyd,box", [(1000, 2, (1.0, 1.0)), (500, 0, (1.3, 0.8)),
                                         (64, 1, (1.0, 1.0))])
def test_initial_mesh(mv, torch_cuda, n, lloyd, box):
    d = mv.voronoi(periodic_voronoi(n, seed=40 + n, lloyd=lloyd, box=box)["generators"], box)
    s = _solver(d)
    compare_mesh(s.geometry(), d)
    s.check()


@pytest.mark.parametrize("kind", ["arepo", "weno"])
def test_limit(oracle, mv, torch_cuda, kind):
    d = mv.voronoi(periodic_voronoi(800, seed=5)["generators"], (1.0, 1.0))
    U = random_voronoi_state(d, G53, seed=6, amp=0.3).reshape(12, -1)
    U[1::3] *= 3.0
    U[2::3] *= 3.0
    U = U.reshape(-1)
    ref = oracle.limit(oracle.Mesh.facelist(d), U, kind=kind, gamma=G53)
    s = _solver(d, limiter=kind)
    e = field_errors(s.limit(s.to_device(U)).cpu().numpy(), ref, 1.0 / math.sqrt(800))
    assert e.max() < 1e-13, e
    s.check()


@pytest.mark.parametrize("motion", [1, 0])
@pytest.mark.parametrize("limiter", [False, "arepo", "weno"])
@pytest.mark.parametrize("flux", ["hll", "exact"])
def test_one_step(mv, torch_cuda, motion, limiter, flux):
    n = 700
    d = mv.voronoi(periodic_voronoi(n, seed=9, lloyd=1)["generators"], (1.0, 1.0))
    U = random_voronoi_state(d, G53, seed=10, amp=0.3)
    dt = mv.cfl_dt(d, U, G53, 0.3, motion)
    ref, d1 = mv.step(d, U, dt, G53, limiter, flux, motion)
    s = _solver(d, limiter=limiter, flux=flux, motion=motion)
    got = s.step_mh(s.to_device(U), dt).cpu().numpy()
    s.check()
    e = field_errors(got, ref, 1.0 / math.sqrt(n))
    # generator positions are absolute coordinates in the box: their rounding
    # (eps L) enters the gradients through the moment shift amplified by L / h,
    # so one step agrees to ~1e-13 rather than to eps
    assert e.max() < 1e-12, e
    compare_mesh(s.geometry(), d1)


def _run(s, U0, dts):
    U = s.to_device(U0)
    V = s.empty()
    for dt in dts:
        s.step_mh(U, dt, out=V)
        U, V = V, U
    s.check()
    return U.double().cpu().numpy()


def _shear(X, Y):
    rho = 1.0 + 0.5 * (np.abs(Y - 0.5) < 0.25)
    u = 0.5 * np.tanh((0.25 - np.abs(Y - 0.5)) / 0.05)
    v = 0.05 * np.sin(2 * math.pi * X)
    p = 2.5 + 0.0 * X
    return [rho, rho * u, rho * v, p / (G53 - 1) + 0.5 * rho * (u * u + v * v)]


@pytest.mark.parametrize("case", ["vortex", "shear"])
def test_100_steps(mv, torch_cuda, case):
    if case == "vortex":
        n, box, g = 4096, (10.0, 10.0), G14
        d = mv.voronoi(periodic_voronoi(n, seed=11, box=box)["generators"], box)
        U0 = project_voronoi(vortex_fields(0.0, g), d)
    else:
        n, box, g = 4096, (1.0, 1.0), G53
        d = mv.voronoi(periodic_voronoi(n, seed=12, box=box)["generators"], box)
        U0 = project_voronoi(_shear, d)
    ref, d1, dts = mv.run(d, U0, 100, g, 0.3, "weno", "exact")
    h = math.sqrt(box[0] * box[1] / n)
    for prec, tol in (("fp64", 1e-11), ("fp32", 1e-3)):
        s = _solver(d, gamma=g, precision=prec)
        got = _run(s, U0, dts)
        e = field_errors(got, ref, h)
        print(f"moving mesh, {case} {n} cells, WENO + exact, {prec}, 100 steps: {e}")
        assert e.max() < tol, (prec, e)
        if prec == "fp64":
            compare_mesh(s.geometry(), d1, tol=1e-11)
            nb0, nb1 = mv.neighbours(d), mv.neighbours(d1)
            assert sum(a != b for a, b in zip(nb0, nb1)) > 50  # the topology did change


def test_100_steps_arepo_hll(mv, torch_cuda):
    """The other limiter and flux over many steps: the Arepo limiter on conserved
    coefficients with the HLL flux, on the shear layer (topology changing)."""
    n, box = 4096, (1.0, 1.0)
    d = mv.voronoi(periodic_voronoi(n, seed=14, box=box)["generators"], box)
    U0 = project_voronoi(_shear, d)
    ref, d1, dts = mv.run(d, U0, 100, G53, 0.3, "arepo", "hll")
    h = math.sqrt(box[0] * box[1] / n)
    for prec, tol in (("fp64", 1e-11), ("fp32", 1e-3)):
        s = _solver(d, limiter="arepo", flux="hll", gamma=G53, precision=prec)
        got = _run(s, U0, dts)
        e = field_errors(got, ref, h)
        print(f"moving mesh, shear {n} cells, Arepo limiter + HLL, {prec}, 100 steps: {e}")
        assert e.max() < tol, (prec, e)
        if prec == "fp64":
            compare_mesh(s.geometry(), d1, tol=1e-11)


def _sod(X, Y):
    """The paper's Sod tube (Sec. 3.2) on a periodic [0, 2): (rho, p) = (1, 1) for
    abs(x - 1) < 1/2, (0.25, 0.1795) elsewhere, at rest; gamma 1.4."""
    inside = np.abs(X - 1.0) < 0.5
    rho = np.where(inside, 1.0, 0.25)
    p = np.where(inside, 1.0, 0.1795)
    return [rho, 0.0 * X, 0.0 * X, p / (G14 - 1)]


def test_sod_100_steps(mv, torch_cuda):
    """Shocks, contacts and rarefactions on the moving mesh: the generators
    compress behind the shocks and spread in the rarefactions."""
    n, box = 2048, (2.0, 0.25)
    d = mv.voronoi(periodic_voronoi(n, seed=13, box=box)["generators"], box)
    U0 = project_voronoi(_sod, d)
    ref, d1, dts = mv.run(d, U0, 100, G14, 0.3, "weno", "exact")
    h = math.sqrt(box[0] * box[1] / n)
    for prec, tol in (("fp64", 1e-11), ("fp32", 1e-3)):
        s = _solver(d, gamma=G14, precision=prec)
        got = _run(s, U0, dts)
        e = field_errors(got, ref, h)
        print(f"moving mesh, Sod {n} cells, WENO + exact, {prec}, 100 steps: {e}")
        assert e.max() < tol, (prec, e)
        if prec == "fp64":
            compare_mesh(s.geometry(), d1, tol=1e-11)
    # the waves moved the generators enough to change the neighbours of many cells
    assert sum(a != b for a, b in zip(mv.neighbours(d), mv.neighbours(d1))) > 100


def test_cfl(mv, torch_cuda):
    torch = torch_cuda
    d = mv.voronoi(periodic_voronoi(900, seed=13)["generators"], (1.0, 1.0))
    U = random_voronoi_state(d, G53, seed=14, amp=0.3)
    for motion in (1, 0):
        s = _solver(d, motion=motion)
        u = s.to_device(U)
        got = float(s.cfl_dt(u, 0.3).cpu())
        ref = mv.cfl_dt(d, U, G53, 0.3, motion)
        assert abs(got - ref) <= 1e-14 * ref
        # fused into the step: the CFL step of the new state on the new mesh
        dt = torch.tensor([ref], dtype=torch.float64, device=s.device)
        nxt = torch.empty(1, dtype=torch.float64, device=s.device)
        out = s.step_mh(u, dt, cfl=0.3, dt_next=nxt)
        U1, d1 = mv.step(d, U, ref, G53, "weno", "exact", motion)
        assert abs(float(nxt.cpu()) - mv.cfl_dt(d1, U1, G53, 0.3, motion)) <= 1e-13 * ref
        assert abs(float(s.cfl_dt(out, 0.3).cpu()) - float(nxt.cpu())) <= 1e-15 * ref
        s.check()


def test_conservation(mv, torch_cuda):
    n = 2000
    d = mv.voronoi(periodic_voronoi(n, seed=15)["generators"], (1.0, 1.0))
    U0 = project_voronoi(_shear, d)
    s = _solver(d)
    U = s.to_device(U0)
    V = s.empty()
    tot0 = (U0.reshape(12, n)[0::3] * d["cell_volume"]).sum(1)
    for _ in range(30):
        dt = float(s.cfl_dt(U, 0.3).cpu())
        s.step_mh(U, dt, out=V)
        U, V = V, U
    s.check()
    geo = s.geometry()
    tot1 = (U.cpu().numpy().reshape(12, n)[0::3] * geo["volume"]).sum(1)
    assert np.all(np.abs(tot1 - tot0) <= 1e-13 * np.abs(tot0).max()), tot1 - tot0
    assert abs(geo["volume"].sum() - 1.0) < 1e-13


def test_refused(mv, torch_cuda):
    from paper_1305_5536_amd.capi import DGError
    from paper_1305_5536_amd.solver import Solver, moving
    d = mv.voronoi(periodic_voronoi(200, seed=16)["generators"], (1.0, 1.0))
    s = _solver(d)
    U = s.to_device(random_voronoi_state(d, G53, seed=17, amp=0.1))
    for call in (lambda: s.step(U, 1e-3), lambda: s.rhs(U), lambda: s.run(U, 2, cfl=0.3)):
        with pytest.raises(DGError):
            call()
    with pytest.raises(DGError):
        Solver(moving(d), physics="mhd", gamma=G53)
    small = mv.voronoi(periodic_voronoi(40, seed=18)["generators"], (1.0, 1.0))
    with pytest.raises(DGError):
        _solver(small)
    broken = dict(d)
    keep = np.all(d["face_cells"] != 0, axis=1)  # cell 0 loses every face
    broken["face_cells"] = d["face_cells"][keep]
    broken["face_shift"] = d["face_shift"][keep]
    with pytest.raises(DGError):
        _solver(broken)
    outside = dict(d)
    outside["generators"] = d["generators"] + 1.0
    with pytest.raises(DGError):
        _solver(outside)
    # the static Cartesian mesh has no generator motion
    from paper_1305_5536_amd.solver import cartesian
    c = Solver(cartesian((8, 8), (0, 0), (1, 1)), gamma=G53)
    with pytest.raises(DGError):
        c.set_motion(0)


def test_kernel_timing(mv, torch_cuda):
    """dg_set_moving_timing / dg_moving_timing: four positive averages over the
    timed steps, a fresh record after each read, and results unchanged."""
    d = mv.voronoi(periodic_voronoi(500, seed=21)["generators"], (1.0, 1.0))
    U0 = random_voronoi_state(d, G53, seed=22, amp=0.2)
    dt = mv.cfl_dt(d, U0, G53, 0.3)
    a, b = _solver(d), _solver(d)
    ua, ub = a.to_device(U0), b.to_device(U0)
    b.set_timing(True)
    ra = a.step_mh(ua, dt)
    rb = b.step_mh(ub, dt)
    b.step_mh(rb, dt)
    ms, n = b.kernel_times()
    assert n == 2 and np.all(ms > 0), (ms, n)
    ms, n = b.kernel_times()
    assert n == 0 and np.all(ms == 0)
    b.set_timing(False)
    a.check()
    b.check()
    U1, _ = mv.step(d, U0, dt, G53, "weno", "exact")
    # the first timed step of b computes what a's untimed step does
    b2 = _solver(d)
    b2.set_timing(True)
    assert np.array_equal(b2.step_mh(b2.to_device(U0), dt).cpu().numpy(), ra.cpu().numpy())
    assert field_errors(ra.cpu().numpy(), U1, 1.0 / math.sqrt(500)).max() < 1e-12
    from paper_1305_5536_amd.capi import DGError
    from paper_1305_5536_amd.solver import Solver, cartesian
    c = Solver(cartesian((8, 8), (0, 0), (1, 1)), gamma=G53)
    with pytest.raises(DGError):
        c.set_timing(True)


@pytest.mark.parametrize("cap", [None, "4"])
def test_high_degree_cell(mv, torch_cuda, monkeypatch, cap):
    """A generator ringed by 16 close neighbours (the most a ring holds), with the
    walk's candidate list in LDS and, with DG_MOVING_CANDIDATES=4, with every cell's
    candidates streamed from the rings instead: the mesh and a step match the
    oracle either way."""
    if cap is not None:
        monkeypatch.setenv("DG_MOVING_CANDIDATES", cap)
    rng = np.random.default_rng(23)
    n0 = 700
    P = periodic_voronoi(n0, seed=24)["generators"]
    c = np.array([0.5, 0.5])
    h = 1.0 / math.sqrt(n0)
    keep = np.linalg.norm(P - c, axis=1) > 2.2 * h
    ang = 2 * math.pi * (np.arange(16) + rng.uniform(-0.05, 0.05, 16)) / 16
    ring = c + 1.0 * h * np.stack([np.cos(ang), np.sin(ang)], 1)
    P = np.concatenate([P[keep], c[None], ring])
    d = mv.voronoi(P, (1.0, 1.0))
    ic = int(np.sum(keep))
    assert len(mv.neighbours(d)[ic]) == 16
    s = _solver(d)
    compare_mesh(s.geometry(), d)
    U = random_voronoi_state(d, G53, seed=25, amp=0.2)
    dt = mv.cfl_dt(d, U, G53, 0.3)
    ref, d1 = mv.step(d, U, dt, G53, "weno", "exact")
    got = s.step_mh(s.to_device(U), dt).cpu().numpy()
    s.check()
    assert field_errors(got, ref, h).max() < 1e-12
    compare_mesh(s.geometry(), d1)
