"""The largest Cartesian meshes the library accepts (ncells x ncoef just below
2^31, the limit of its 32-bit cell indexing), run through the same entry points
and launch shapes as every other size.

The state varies along x only (smooth fields plus two density jumps, so the
limiter acts), so every row (2D) or (y, z) row (3D) of the result must be the
same.  Each kernel computes a cell from its own and its neighbours' values with
the same arithmetic wherever the cell sits (results are bitwise independent of
the tiling), so every row of the large mesh must equal, bit for bit, the result
on a mesh of the same x extent with two cells along the other axes and the same
spacings; that small mesh is checked against the oracle (without the limiter at
1e-13; with it at 1e-13 for Euler and, for MHD, where B_x is constant and the
field's common alpha acts on rounding noise, at ten times the oracle's own
one-ulp sensitivity).  A 32-bit overflow in any address or index would break
the row equality.

Device memory: up to about 105 GB (five or six states of 17 GB); the test is
skipped on a GPU with less free memory.
"""
import math

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

G53 = 5.0 / 3.0
LIMIT = 1 << 31


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _fields(mhd):
    """Conserved fields that depend on x only; B_x constant (div B = 0)."""
    def f(*X):
        x = X[0]
        rho = (1.0 + 0.2 * np.sin(2 * math.pi * x) + 0.1 * np.cos(6 * math.pi * x)
               + np.where((x > 0.3) & (x < 0.7), 0.8, 0.0))
        vel = [0.3 + 0.2 * np.sin(4 * math.pi * x), 0.4 * np.cos(2 * math.pi * x)]
        if mhd or len(X) == 3:
            vel.append(-0.25 * np.sin(2 * math.pi * x + 0.5))
        p = 1.0 + 0.2 * np.cos(2 * math.pi * x + 1.0)
        ke = 0.5 * rho * sum(v * v for v in vel)
        out = [rho] + [rho * v for v in vel]
        if not mhd:
            return out + [p / (G53 - 1.0) + ke]
        B = [np.full_like(x, 0.5), 0.3 * np.sin(2 * math.pi * x), 0.2 * np.cos(2 * math.pi * x)]
        return out + [p / (G53 - 1.0) + ke + 0.5 * sum(b * b for b in B)] + B
    return f


def _field_error(A, B, ncoef, means, h):
    """max over coefficients of |A - B| (gradient-like coefficients scaled by h),
    relative to the largest mean."""
    A = A.reshape(ncoef, -1)
    B = B.reshape(ncoef, -1)
    w = np.full((ncoef, 1), h)
    w[means] = 1.0
    return (w * np.abs(A - B)).max() / np.abs(B[means]).max()


def _run_max_case(torch, n_max, physics, precision, oracle, means):
    from paper_1305_5536_amd.solver import Solver, cartesian
    dim = len(n_max)
    mhd = physics == "mhd"
    ncoef = (5 if mhd else dim + 2) * (1 + dim) + ((3 + (8 if dim == 3 else 5)) if mhd else 0)
    ncells = int(np.prod(n_max))
    assert ncells * ncoef < LIMIT, (n_max, ncoef)
    elem = 8 if precision == "fp64" else 4
    need = 6.5 * ncoef * ncells * elem
    free, _ = torch.cuda.mem_get_info()
    if free < need:
        pytest.skip(f"needs {need / 1e9:.0f} GB of free device memory, {free / 1e9:.0f} GB free")
    nx = n_max[0]
    small = (nx,) + (2,) * (dim - 1)
    lo = (0.0,) * dim
    hi_max = (1.0,) * dim
    # the same spacing along every axis as the large mesh (2/n = 2 x 1/n exactly)
    hi_small = (1.0,) + tuple(2.0 / n for n in n_max[1:])
    U_small = W.project_cartesian(_fields(mhd), small, lo, hi_small, mhd=mhd)
    rows = U_small.reshape(ncoef, -1, nx)
    assert np.array_equal(rows, np.broadcast_to(rows[:, :1], rows.shape))

    ss = Solver(cartesian(small, lo, hi_small), physics=physics, precision=precision,
                gamma=G53)
    sl = Solver(cartesian(n_max, lo, hi_max), physics=physics, precision=precision, gamma=G53)
    h = 1.0 / max(n_max)
    dt = 0.1 * h
    Us = ss.to_device(U_small)
    print(f"max-size {physics} {dim}D {n_max} {precision}: {ncells} cells x {ncoef}", flush=True)
    Ul = Us.view(ncoef, -1, nx)[:, :1, :].expand(ncoef, ncells // nx, nx).contiguous().view(-1)

    def rows_equal(big, ref):
        big = big.view(ncoef, -1, nx)
        return torch.equal(big, ref.view(ncoef, -1, nx)[:, :1, :].expand_as(big))

    assert rows_equal(Ul, Us)
    # CFL step: a minimum over identical rows
    assert sl.cfl_dt(Ul, 0.3).item() == ss.cfl_dt(Us, 0.3).item()
    # one SSP-RK2 step (the library's own path: the fused step kernel for 2D Euler)
    a_small = ss.step(Us, dt)
    out = sl.step(Ul, dt)
    sl.check()
    ss.check()
    assert rows_equal(a_small, a_small)
    assert rows_equal(out, a_small)
    # the two stage kernels
    V1 = sl.empty()
    sl.stage1(Ul, dt, V1)
    sl.stage2(Ul, V1, dt, out)
    V1s = ss.empty()
    b_small = ss.empty()
    ss.stage1(Us, dt, V1s)
    ss.stage2(Us, V1s, dt, b_small)
    sl.check()
    assert rows_equal(V1, V1s)
    assert rows_equal(out, b_small)
    # right-hand side alone
    del V1
    sl.rhs(Ul, out)
    assert rows_equal(out, ss.rhs(Us))
    sl.check()
    del out, Ul
    sl.close()
    torch.cuda.empty_cache()
    # the small mesh against the oracle, without and with the limiter
    tol = 1e-13 if precision == "fp64" else 2e-5
    om = oracle.Mesh.cartesian(small, lo, hi_small)
    sn = Solver(cartesian(small, lo, hi_small), physics=physics, precision=precision,
                gamma=G53, limiter=False)
    ref = oracle.step(om, U_small, dt, G53, False, mhd=mhd)
    err = _field_error(sn.step(Us, dt).double().cpu().numpy(), ref, ncoef, means, h)
    print(f"  small mesh {small} vs oracle, one step, no limiter: {err:.3e}", flush=True)
    assert err < tol, err
    ref = oracle.step(om, U_small, dt, G53, True, mhd=mhd)
    err = _field_error(a_small.double().cpu().numpy(), ref, ncoef, means, h)
    bound = tol
    if mhd:
        # B_x is constant here (div B = 0 with x-only variation), so its gradients
        # are rounding noise, and the field's common alpha (Sec. 2.5), which the
        # B_x noise can set, scales the B_y, B_z gradients: the limited step moves
        # by far more than one ulp under one-ulp changes of the input, in the
        # oracle as well.  The bound is ten times that self-sensitivity.
        rng = np.random.default_rng(0)
        Up = U_small * (1.0 + rng.choice([-1.0, 1.0], size=U_small.shape) * 2.0 ** -52)
        e_self = _field_error(oracle.step(om, Up, dt, G53, True, mhd=True), ref, ncoef, means, h)
        bound = max(tol, 10.0 * e_self)
        print(f"  oracle self-sensitivity to one ulp: {e_self:.3e}", flush=True)
    print(f"  small mesh {small} vs oracle, one step, limiter: {err:.3e}", flush=True)
    assert err < bound, (err, bound)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_largest_2d_euler_mesh(oracle, torch_cuda, precision):
    # 13377^2 cells x 12 coefficients = 2147329548 < 2^31 (one more column
    # would pass it); ragged in both axes (60-column strips, rows per wave)
    _run_max_case(torch_cuda, (13377, 13377), "euler", precision, oracle, [0, 3, 6, 9])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_largest_2d_mhd_mesh(oracle, torch_cuda, precision):
    # 9663 x 9662 cells x 23 coefficients = 2147369838 < 2^31
    _run_max_case(torch_cuda, (9663, 9662), "mhd", precision, oracle,
                  [0, 3, 6, 9, 12, 15, 16, 17])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_largest_3d_mhd_mesh(oracle, torch_cuda, precision):
    # 411 x 409 x 412 cells x 31 coefficients = 2146960428 < 2^31 (one more
    # column would pass it); ragged in x
    # (64-cell strips), y (groups of four rows) and z (planes per workgroup)
    _run_max_case(torch_cuda, (411, 409, 412), "mhd", precision, oracle,
                  [0, 4, 8, 12, 16, 20, 21, 22])


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_largest_batch(oracle, torch_cuda, precision):
    """A batch of three uneven 2D Euler instances whose cells total just below
    2^31 / 12 (the batch's indexing limit): per instance, every row of the CFL
    step, of one step and of the two stages equals bit for bit the single-mesh
    stage kernels on two rows of the same spacings."""
    torch = torch_cuda
    from paper_1305_5536_amd.solver import Solver, batch, cartesian
    sizes = [(8191, 9000), (5003, 12000), (6700, 6746)]
    total = sum(nx * ny for nx, ny in sizes)
    assert total * 12 < LIMIT and (total + 6746) * 12 >= LIMIT
    elem = 8 if precision == "fp64" else 4
    need = 6.5 * 12 * total * elem
    free, _ = torch.cuda.mem_get_info()
    if free < need:
        pytest.skip(f"needs {need / 1e9:.0f} GB of free device memory, {free / 1e9:.0f} GB free")
    b = Solver(batch(sizes), precision=precision, gamma=G53)
    off = [int(v) for v in b.offsets]
    U = b.empty()
    smalls = []
    for i, (nx, ny) in enumerate(sizes):
        lo, hi = (0.0, 0.0), (1.0, 2.0 / ny)
        Us_host = W.project_cartesian(_fields(False), (nx, 2), lo, hi)
        ss = Solver(cartesian((nx, 2), lo, hi), precision=precision, gamma=G53)
        Us = ss.to_device(Us_host)
        U.view(12, -1)[:, off[i]:off[i + 1]].view(12, ny, nx).copy_(
            Us.view(12, 2, nx)[:, :1, :].expand(12, ny, nx))
        smalls.append((ss, Us, Us_host, lo, hi))
    print(f"max-size batch {sizes} {precision}: {total} cells x 12", flush=True)

    def inst_rows_equal(big, i, ref):
        nx, ny = sizes[i]
        v = big.view(12, -1)[:, off[i]:off[i + 1]].view(12, ny, nx)
        return torch.equal(v, ref.view(12, 2, nx)[:, :1, :].expand(12, ny, nx))

    dtb = b.cfl_dt(U, 0.3)
    out = b.step(U, dtb)
    V1 = b.empty()
    b.stage1(U, dtb, V1)
    b.check()
    for i, (ss, Us, Us_host, lo, hi) in enumerate(smalls):
        dt = ss.cfl_dt(Us, 0.3)
        assert dt.item() == dtb[i].item(), i
        v1, ref = ss.empty(), ss.empty()
        ss.stage1(Us, dt, v1)
        ss.stage2(Us, v1, dt, ref)
        ss.check()
        assert inst_rows_equal(U, i, Us), i
        assert inst_rows_equal(V1, i, v1), i
        assert inst_rows_equal(out, i, ref), i
    b.stage2(U, V1, dtb, out)
    b.check()
    for i, (ss, Us, Us_host, lo, hi) in enumerate(smalls):
        dt = ss.cfl_dt(Us, 0.3)
        v1, ref = ss.empty(), ss.empty()
        ss.stage1(Us, dt, v1)
        ss.stage2(Us, v1, dt, ref)
        assert inst_rows_equal(out, i, ref), i
    # the smallest instance's two-row mesh against the oracle
    ss, Us, Us_host, lo, hi = smalls[2]
    om = oracle.Mesh.cartesian((sizes[2][0], 2), lo, hi)
    dt = oracle.cfl_dt(om, Us_host, G53, 0.3)
    # (FP32: the CFL step of the rounded state)
    assert abs(dt - dtb[2].item()) <= (1e-14 if precision == "fp64" else 1e-6) * dt
    v1, got = ss.empty(), ss.empty()
    dt_dev = torch.tensor([dt], dtype=torch.float64, device=ss.device)
    ss.stage1(Us, dt_dev, v1)
    ss.stage2(Us, v1, dt_dev, got)
    err = _field_error(got.double().cpu().numpy(), oracle.step(om, Us_host, dt, G53, True), 12,
                       [0, 3, 6, 9], 1.0 / sizes[2][0])
    print(f"  two-row mesh of instance 2 vs oracle, one step: {err:.3e}", flush=True)
    assert err < (1e-13 if precision == "fp64" else 2e-5), err
    del U, V1, out
    b.close()
    torch.cuda.empty_cache()


def _grid_facelist(nx, ny, h):
    """A periodic nx x ny grid of square cells of side h written as a face-list
    descriptor (cells x fastest; per cell its +x face, then its +y face).  With h
    a power of two every coordinate and offset is exact, so every cell sees the
    same geometry bit for bit."""
    nc = nx * ny
    i = np.tile(np.arange(nx), ny)
    j = np.repeat(np.arange(ny), nx)
    cen = np.stack([(i + 0.5) * h, (j + 0.5) * h], axis=1)
    fc = np.empty((2 * nc, 2), np.int32)
    fc[0::2, 0] = fc[1::2, 0] = np.arange(nc)
    fc[0::2, 1] = j * nx + (i + 1) % nx
    fc[1::2, 1] = ((j + 1) % ny) * nx + i
    nrm = np.zeros((2 * nc, 2))
    nrm[0::2, 0] = 1.0
    nrm[1::2, 1] = 1.0
    xf = np.repeat(cen, 2, axis=0)
    xf[0::2, 0] += 0.5 * h
    xf[1::2, 1] += 0.5 * h
    sh = np.zeros((2 * nc, 2), np.int8)
    sh[0::2, 0] = i + 1 == nx
    sh[1::2, 1] = j + 1 == ny
    m2 = h ** 4 / 12.0
    return {"kind": "facelist", "box": np.array([nx * h, ny * h]),
            "cell_volume": np.full(nc, h * h), "cell_centroid": cen,
            "cell_moments": np.tile([m2, 0.0, m2], (nc, 1)),
            "face_cells": fc, "face_area": np.full(2 * nc, h), "face_normal": nrm,
            "face_centroid": xf, "face_shift": sh}


@pytest.mark.timeout(300)
def test_largest_facelist_mesh(oracle, torch_cuda):
    """The face-list path (static Voronoi meshes) at its limit, 20 nfaces just below
    2^31: a 7327^2 periodic grid written as a face list (53.7M cells, 107M faces),
    FP64, with a state that varies along x only.  Cells in different positions of
    their blocks may sum their faces in a different order, so rows are compared to
    the two-row mesh's result to 1e-13 rather than bit for bit."""
    torch = torch_cuda
    from paper_1305_5536_amd.solver import Solver
    nx = ny = 7327
    h = 2.0 ** -13
    nc = nx * ny
    assert 20 * 2 * nc < LIMIT and 20 * 2 * (nc + ny) >= LIMIT
    free, _ = torch.cuda.mem_get_info()
    if free < 120e9:
        pytest.skip(f"needs 120 GB of free device memory, {free / 1e9:.0f} GB free")
    d_small = _grid_facelist(nx, 2, h)
    U_small = W.project_cartesian(_fields(False), (nx, 2), (0.0, 0.0), (nx * h, 2 * h))
    ss = Solver(d_small, gamma=G53)
    Us = ss.to_device(U_small)
    print(f"max-size face list {nx}x{ny}: {nc} cells, {2 * nc} faces; building", flush=True)
    sb = Solver(_grid_facelist(nx, ny, h), gamma=G53)
    print("  mesh built", flush=True)
    Ub = Us.view(12, 2, nx)[:, :1, :].expand(12, ny, nx).contiguous().view(-1)
    w = torch.full((12, 1, 1), h, dtype=torch.float64, device=Us.device)
    w[0::3] = 1.0
    scale = Us.view(12, -1)[0::3].abs().max().item()

    def rows_err(big, small):
        big = big.view(12, ny, nx)
        ref = small.view(12, 2, nx)[:, :1, :]
        return ((big - ref).abs() * w).max().item() / scale

    dt_b, dt_s = sb.cfl_dt(Ub, 0.3).item(), ss.cfl_dt(Us, 0.3).item()
    assert abs(dt_b - dt_s) <= 1e-14 * dt_s, (dt_b, dt_s)
    dt = 0.5 * dt_s
    a = ss.step(Us, dt)
    out = sb.step(Ub, dt)
    sb.check()
    ss.check()
    e_step = rows_err(out, a)
    V1, v1 = sb.empty(), ss.empty()
    sb.stage1(Ub, dt, V1)
    ss.stage1(Us, dt, v1)
    e_st1 = rows_err(V1, v1)
    sb.stage2(Ub, V1, dt, out)
    b = ss.empty()
    ss.stage2(Us, v1, dt, b)
    sb.check()
    e_st2 = rows_err(out, b)
    print(f"  rows vs two-row mesh: step {e_step:.2e}, stage 1 {e_st1:.2e}, stage 2 {e_st2:.2e}",
          flush=True)
    assert max(e_step, e_st1, e_st2) < 1e-13, (e_step, e_st1, e_st2)
    del Ub, V1, out
    sb.close()
    torch.cuda.empty_cache()
    om = oracle.Mesh.facelist(d_small)
    err = _field_error(a.double().cpu().numpy(), oracle.step(om, U_small, dt, G53, True), 12,
                       [0, 3, 6, 9], h)
    print(f"  two-row face list vs oracle, one step: {err:.3e}", flush=True)
    assert err < 1e-13, err
