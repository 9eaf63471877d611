"""Pins of the oracle's CFL step, signal speeds, HLLD outer wave speeds and the
common field alpha of the MHD limiter.

* The fast magnetosonic speed is the largest characteristic speed of the ideal
  MHD equations: the largest eigenvalue of the flux Jacobian dF.n/dU minus
  v.n.  The Jacobian is taken here by complex-step differentiation of a NumPy
  flux, so the pin does not restate the closed form the oracle evaluates.
* The CFL step (reading Z7, dt = cfl min_e 2 V_e / sum_f A_f (|v.n_f| +
  c(n_f))) has a closed form on a box: cfl / sum_d (|v_d| + c_d) / h_d, with the
  fast speed along each axis equal to max(a, |B|/sqrt(rho)) where B is parallel
  to it and sqrt(a^2 + B^2/rho) where it is perpendicular.
* HLLD returns the left state's physical flux exactly when its outer left speed
  S_L = min(v_nL, v_nR) - max(c_fL, c_fR) is >= 0 (reading Z4); boosting both
  states along n moves S_L through zero, and the switch must happen where the
  NumPy fast speeds put it.
* HLLD's star states divide by rho (S - v_n)(S - S_M) - B_n^2, which vanishes
  where the fast speed meets the Alfven speed: tangential field (near) zero and
  B_n^2 >= gamma p (reading Z4 takes the outer transverse v and B there).  Two
  equal states must still give the physical flux (consistency, exact in the
  limit); a missing switch divides rounding noise by rounding noise, a switch
  to zero transverse field loses S_L B_t.
* The limiter (Sec. 2.5, reading Z5) gives the three field components one alpha:
  on fields that vary along one axis that alpha has the 1D closed form
  min over components of min(1, 2 min(|D+|, |D-|) / (|g| h)) (0 at a strict
  extremum), and it scales every coefficient of the divergence-free basis.
"""
import math

import numpy as np
import pytest

import np_physics as P

G53 = 5.0 / 3.0
G14 = 1.4


def _rand_mhd(rng, vamp=0.3):
    rho = rng.uniform(0.5, 2.0)
    v = rng.uniform(-vamp, vamp, 3)
    p = rng.uniform(0.3, 2.0)
    B = rng.uniform(-1.2, 1.2, 3)
    return P.mhd_state(rho, v, p, B, G53)


def _unit(rng, d):
    x = rng.normal(size=d)
    return x / np.linalg.norm(x)


def _cf_from_jacobian(u, n, gamma, mhd):
    J = P.flux_jacobian(u, n, gamma, mhd)
    lam = np.linalg.eigvals(J).real
    dim = 3 if mhd else len(u) - 2
    vn = u[1:1 + dim] @ np.asarray(n)[:dim] / u[0]
    return lam.max() - vn


# ------------------------------------------------------------ signal speeds
def test_fast_speed_is_largest_characteristic_speed(oracle):
    rng = np.random.default_rng(71)
    for _ in range(40):
        u = _rand_mhd(rng)
        n = _unit(rng, 3)
        cf = oracle.signal_speed(u, n, G53, mhd=True)
        assert cf == pytest.approx(_cf_from_jacobian(u, n, G53, True), rel=1e-9)


def test_sound_speed_is_largest_characteristic_speed(oracle):
    rng = np.random.default_rng(72)
    for dim in (2, 3):
        for _ in range(10):
            u = P.euler_state(rng.uniform(0.5, 2), rng.uniform(-0.5, 0.5, dim),
                              rng.uniform(0.3, 2), G14)
            n = _unit(rng, dim)
            c = oracle.signal_speed(u, n, G14)
            assert c == pytest.approx(_cf_from_jacobian(u, n, G14, False), rel=1e-10)


def test_fast_speed_parallel_and_perpendicular_field(oracle):
    rho, p = 1.3, 0.7
    a = math.sqrt(G53 * p / rho)
    for Bmag in (0.2, 1.5):  # Alfven speed below and above the sound speed
        b = Bmag / math.sqrt(rho)
        n = np.array([0.0, 0.6, 0.8])
        par = P.mhd_state(rho, [0.1, -0.2, 0.3], p, Bmag * n, G53)
        perp = P.mhd_state(rho, [0.1, -0.2, 0.3], p, Bmag * np.array([1.0, 0, 0]), G53)
        assert oracle.signal_speed(par, n, G53, mhd=True) == pytest.approx(max(a, b), rel=1e-14)
        assert oracle.signal_speed(perp, n, G53, mhd=True) == pytest.approx(
            math.sqrt(a * a + b * b), rel=1e-14)
    zero = P.mhd_state(rho, [0.1, 0, 0], p, [0, 0, 0], G53)
    assert oracle.signal_speed(zero, [1, 0, 0], G53, mhd=True) == pytest.approx(a, rel=1e-14)


# ----------------------------------------------------------------- CFL step
def _uniform(ncoef, nc, mean_values, stride):
    U = np.zeros((ncoef, nc))
    for k, val in enumerate(mean_values):
        U[k * stride] = val
    return U


def test_cfl_dt_euler2d_box_closed_form(oracle):
    n, lo, hi = (7, 5), (0.0, -0.2), (1.3, 0.2)
    hx, hy = 1.3 / 7, 0.4 / 5
    rho, v, p = 1.2, np.array([0.3, -0.7]), 0.9
    u = P.euler_state(rho, v, p, G14)
    U = _uniform(12, 35, u, 3)
    m = oracle.Mesh.cartesian(n, lo, hi)
    c = math.sqrt(G14 * p / rho)
    want = 0.3 / ((abs(v[0]) + c) / hx + (abs(v[1]) + c) / hy)
    assert oracle.cfl_dt(m, U.reshape(-1), G14, 0.3) == pytest.approx(want, rel=1e-14)
    # one hot cell sets the step: the minimum over cells of the same form
    hot = P.euler_state(0.8, [-1.1, 0.4], 3.0, G14)
    U[0::3, 17] = hot
    ch = math.sqrt(G14 * 3.0 / 0.8)
    want_hot = 0.3 / ((1.1 + ch) / hx + (0.4 + ch) / hy)
    assert want_hot < want
    assert oracle.cfl_dt(m, U.reshape(-1), G14, 0.3) == pytest.approx(want_hot, rel=1e-14)


@pytest.mark.parametrize("axis", [0, 1, 2])
def test_cfl_dt_mhd3d_box_closed_form(oracle, axis):
    n, lo, hi = (3, 4, 5), (0.0, 0.0, 0.0), (0.6, 1.0, 2.0)
    h = [0.2, 0.25, 0.4]
    rho, v, p, Bmag = 1.1, np.array([0.2, -0.3, 0.5]), 0.8, 1.4
    B = np.zeros(3)
    B[axis] = Bmag
    u = P.mhd_state(rho, v, p, B, G53)
    U = np.zeros((31, 60))
    for k in range(5):
        U[4 * k] = u[k]
    U[20:23] = B[:, None]
    a = math.sqrt(G53 * p / rho)
    b = Bmag / math.sqrt(rho)
    s = sum((abs(v[d]) + (max(a, b) if d == axis else math.sqrt(a * a + b * b))) / h[d]
            for d in range(3))
    m = oracle.Mesh.cartesian(n, lo, hi)
    assert oracle.cfl_dt(m, U.reshape(-1), G53, 0.4, mhd=True) == pytest.approx(0.4 / s, rel=1e-14)


def grid_as_facelist(nx, ny, box):
    """A periodic nx x ny box grid written as a face-list descriptor."""
    hx, hy = box[0] / nx, box[1] / ny
    nc = nx * ny
    cen = np.array([[(i + 0.5) * hx, (j + 0.5) * hy] for j in range(ny) for i in range(nx)])
    V = np.full(nc, hx * hy)
    Mo = np.tile([hx * hy * hx * hx / 12, 0.0, hx * hy * hy * hy / 12], (nc, 1))
    fc, A, nrm, xf, sh = [], [], [], [], []
    for j in range(ny):
        for i in range(nx):
            e = j * nx + i
            fc.append((e, j * nx + (i + 1) % nx))
            A.append(hy)
            nrm.append((1.0, 0.0))
            xf.append(cen[e] + (0.5 * hx, 0.0))
            sh.append((1 if i + 1 == nx else 0, 0))
            fc.append((e, ((j + 1) % ny) * nx + i))
            A.append(hx)
            nrm.append((0.0, 1.0))
            xf.append(cen[e] + (0.0, 0.5 * hy))
            sh.append((0, 1 if j + 1 == ny else 0))
    return {"kind": "facelist", "box": np.array(box, float), "cell_volume": V,
            "cell_centroid": cen, "cell_moments": Mo,
            "face_cells": np.array(fc, np.int32), "face_area": np.array(A),
            "face_normal": np.array(nrm), "face_centroid": np.array(xf),
            "face_shift": np.array(sh, np.int8)}


def test_cfl_dt_facelist_closed_form(oracle):
    box = (1.5, 0.6)
    d = grid_as_facelist(6, 4, box)
    hx, hy = 0.25, 0.15
    rho, v, p = 0.9, np.array([-0.4, 0.25]), 1.7
    U = _uniform(12, 24, P.euler_state(rho, v, p, G53), 3)
    c = math.sqrt(G53 * p / rho)
    want = 0.35 / ((abs(v[0]) + c) / hx + (abs(v[1]) + c) / hy)
    m = oracle.Mesh.facelist(d)
    assert oracle.cfl_dt(m, U.reshape(-1), G53, 0.35) == pytest.approx(want, rel=1e-14)
    # a non-uniform state: the face-list path and the box path give one step
    rng = np.random.default_rng(5)
    U[0::3] *= rng.uniform(0.8, 1.2, (4, 24))
    mb = oracle.Mesh.cartesian((6, 4), (0, 0), box)
    assert oracle.cfl_dt(m, U.reshape(-1), G53, 0.35) == pytest.approx(
        oracle.cfl_dt(mb, U.reshape(-1), G53, 0.35), rel=1e-14)


# ------------------------------------------------------- HLLD outer speeds
def _boosted(rho, v, p, B, V):
    return P.mhd_state(rho, np.asarray(v) + np.array([V, 0, 0]), p, B, G53)


@pytest.mark.parametrize("side", ["left", "right"])
def test_hlld_outer_speeds_switch_where_fast_speeds_put_them(oracle, side):
    """Both states boosted by V along n = e_x: the flux is exactly the upwind
    state's physical flux once the outer wave on that side changes sign, at the
    boost fixed by S_L = min(v_n) - max(c_f) (or S_R = max(v_n) + max(c_f)).
    The states are chosen so that a Davis-type estimate min(v_nL - c_fL,
    v_nR - c_fR) would switch 0.5 away."""
    n = np.array([1.0, 0.0, 0.0])
    Bn = 0.4
    L = (1.0, [-0.2, 0.2, -0.1], 0.8, [Bn, 0.3, 0.2])      # lower v_n, lower c_f
    R = (0.5, [0.3, -0.1, 0.2], 1.6, [Bn, -0.9, 0.7])     # higher v_n, higher c_f
    cfL = _cf_from_jacobian(_boosted(*L, 0.0), n, G53, True)
    cfR = _cf_from_jacobian(_boosted(*R, 0.0), n, G53, True)
    assert cfR > cfL + 0.3
    vnL, vnR = L[1][0], R[1][0]
    if side == "left":
        V0 = max(cfL, cfR) - min(vnL, vnR)   # S_L = 0
        up = 0
        sgn = 1.0
    else:
        V0 = -(max(vnL, vnR) + max(cfL, cfR))  # S_R = 0
        up = 1
        sgn = -1.0
    for V, exact in ((V0 + sgn * 1e-9, True), (V0 - sgn * 2e-3, False), (V0 - sgn * 0.3, False)):
        uL, uR = _boosted(*L, V), _boosted(*R, V)
        F = oracle.hlld(uL, uR, n, G53)
        Fup = P.flux((uL, uR)[up], n, G53, True)
        dev = np.abs(F - Fup).max() / np.abs(Fup).max()
        if exact:
            assert dev < 1e-14, (side, V, dev)
        else:
            assert dev > 1e-7, (side, V, dev)


# --------------------------------------------------- common field alpha (MHD)
@pytest.mark.parametrize("bt", [0.0, 1e-9, 1e-7])
def test_hlld_degenerate_star_states_keep_consistency(oracle, bt):
    """Equal left and right states with B_n^2 > gamma p and a tangential field of
    magnitude bt: the fast speed equals the Alfven speed up to O(bt^2), so the
    star-state denominator is rounding noise, and the flux must still be the
    physical one (NumPy flux, not the oracle's), finite, in every HLLD region."""
    rng = np.random.default_rng(91)
    for _ in range(200):
        rho, p = rng.uniform(0.5, 2.0), rng.uniform(0.1, 1.0)
        n = _unit(rng, 3)
        bn = math.sqrt(G53 * p * rng.uniform(1.5, 6.0)) * rng.choice([-1.0, 1.0])
        t = _unit(rng, 3)
        t -= (t @ n) * n
        t /= np.linalg.norm(t)
        B = bn * n + bt * t
        ca = abs(bn) / math.sqrt(rho)
        # normal velocity inside the fan (every region of HLLD in turn), any
        # tangential velocity
        vn = rng.uniform(-0.95, 0.95) * ca
        vt = rng.normal(0.0, 0.5, 3)
        vt -= (vt @ n) * n
        u = P.mhd_state(rho, vn * n + vt, p, B, G53)
        F = oracle.hlld(u, u, n, G53)
        ref = P.flux(u, n, G53, True)
        assert np.all(np.isfinite(F))
        assert np.allclose(F, ref, rtol=1e-12, atol=1e-13), (F - ref, bt)


def _closed_form_alpha(phim, phi, phip, g, h):
    """1D limiter factor of one variable: the largest alpha in [0, 1] with both
    face extrapolations phi -+ alpha g h/2 inside [min, max] of the three
    means: min(1, 2 min(|D+|, |D-|)/(|g| h)) on monotone data, 0 at a strict
    extremum."""
    if g == 0:
        return 1.0
    dp, dm = phip - phi, phi - phim
    if dp * dm <= 0:
        return 0.0
    return min(1.0, 2.0 * min(abs(dp), abs(dm)) / (abs(g) * h))


def _field_along_x(rng, nx):
    """Means of one period of two phase-shifted sinusoids (monotone away from
    two extrema each), slopes their derivatives times random factors 0.5..3,
    so that most cells are limited and the two components' alphas differ."""
    x = (np.arange(nx) + 0.5) / nx
    ph = rng.uniform(0, 2 * math.pi, 2)
    by, bz = np.sin(2 * math.pi * x + ph[0]), 0.7 * np.sin(2 * math.pi * x + ph[1])
    gy = 2 * math.pi * np.cos(2 * math.pi * x + ph[0]) * rng.uniform(0.5, 3, nx)
    gz = 0.7 * 2 * math.pi * np.cos(2 * math.pi * x + ph[1]) * rng.uniform(0.5, 3, nx)
    return by, bz, gy, gz


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_mhd3d_common_alpha_closed_form(oracle, seed):
    rng = np.random.default_rng(seed)
    nx, ny, nz = 16, 2, 2
    h = 1.0 / nx
    by, bz, gy, gz = _field_along_x(rng, nx)
    nc = nx * ny * nz
    U = np.zeros((31, nc))
    ii = np.arange(nc) % nx
    U[0], U[16] = 1.0, 3.0                     # uniform rho, E (hydro limiter idle)
    U[20], U[21], U[22] = 0.3, by[ii], bz[ii]  # B means
    U[23 + 2] = gy[ii]                         # a6: dB_y/dx (V6 = (0, x, 0))
    U[23 + 4] = gz[ii]                         # a8: dB_z/dx (V8 = (0, 0, x))
    m = oracle.Mesh.cartesian((nx, ny, nz), (0, 0, 0), (1, 1, 1))
    Ul = oracle.limit(m, U.reshape(-1), mhd=True).reshape(31, -1)
    assert np.array_equal(Ul[:23], U[:23])
    nsplit = 0
    for e in range(nc):
        i = e % nx
        ay = _closed_form_alpha(by[i - 1], by[i], by[(i + 1) % nx], gy[i], h)
        az = _closed_form_alpha(bz[i - 1], bz[i], bz[(i + 1) % nx], gz[i], h)
        a = min(ay, az)
        nsplit += (0 < min(ay, az) < max(ay, az))
        assert Ul[25, e] == pytest.approx(a * U[25, e], rel=1e-13, abs=1e-15)
        assert Ul[27, e] == pytest.approx(a * U[27, e], rel=1e-13, abs=1e-15)
    assert nsplit > 0  # cells where the two components alone would disagree
    assert not np.any(Ul[[23, 24, 26, 28, 29, 30]])


def test_mhd2d_common_alpha_closed_form(oracle):
    """2D field basis: B_y = b_y + a2 x (V4 = (0, x)), B_z in the Taylor basis
    (its x-derivative is the fourth field coefficient); B_x constant."""
    rng = np.random.default_rng(9)
    nx, ny = 13, 2
    h = 1.0 / nx
    by, bz, gy, gz = _field_along_x(rng, nx)
    nc = nx * ny
    U = np.zeros((23, nc))
    ii = np.arange(nc) % nx
    U[0], U[12] = 1.0, 3.0
    U[15], U[16], U[17] = -0.2, by[ii], bz[ii]
    U[18 + 1] = gy[ii]
    U[18 + 3] = gz[ii]
    m = oracle.Mesh.cartesian((nx, ny), (0, 0), (1, 1))
    Ul = oracle.limit(m, U.reshape(-1), mhd=True).reshape(23, -1)
    for e in range(nc):
        i = e % nx
        a = min(_closed_form_alpha(by[i - 1], by[i], by[(i + 1) % nx], gy[i], h),
                _closed_form_alpha(bz[i - 1], bz[i], bz[(i + 1) % nx], gz[i], h))
        assert Ul[19, e] == pytest.approx(a * U[19, e], rel=1e-13, abs=1e-15)
        assert Ul[21, e] == pytest.approx(a * U[21, e], rel=1e-13, abs=1e-15)


def test_mhd3d_limited_field_bounds_and_single_alpha(oracle):
    """Random fields: every basis coefficient of a cell is scaled by the same
    alpha; each component's limited extrapolation to every face centroid lies
    within that component's bounds over the cell and its face neighbours; and
    alpha is the largest such factor (a slightly larger one breaks a bound)."""
    import workloads as W
    n = (5, 4, 3)
    U = W.random_p1_state(n, (0, 0, 0), (1, 1, 1), G53, seed=17, amp=0.2, mhd=True,
                          bamp=0.3).reshape(31, -1)
    m = oracle.Mesh.cartesian(n, (0, 0, 0), (1, 1, 1))
    Ul = oracle.limit(m, U.reshape(-1), mhd=True).reshape(31, -1)
    h = np.array([1 / 5, 1 / 4, 1 / 3])
    Jb = [np.zeros((3, 3)) for _ in range(8)]
    for j, (c, d) in enumerate([(0, 1), (0, 2), (1, 0), (1, 2), (2, 0), (2, 1)]):
        Jb[j][c, d] = 1
    Jb[6][0, 0], Jb[6][1, 1] = 1, -1
    Jb[7][0, 0], Jb[7][2, 2] = 1, -1

    def idx(i, j, k):
        return ((k % 3) * 4 + (j % 4)) * 5 + (i % 5)

    limited = 0
    for e in range(60):
        i, j, k = e % 5, (e // 5) % 4, e // 20
        a0, a1 = U[23:, e], Ul[23:, e]
        nz = np.abs(a0) > 0
        ratio = a1[nz] / a0[nz]
        assert np.ptp(ratio) < 1e-14
        alpha = ratio[0]
        assert 0.0 <= alpha <= 1.0
        nbrs = [idx(i - 1, j, k), idx(i + 1, j, k), idx(i, j - 1, k), idx(i, j + 1, k),
                idx(i, j, k - 1), idx(i, j, k + 1)]
        faces = [(-h[0] / 2, 0, 0), (h[0] / 2, 0, 0), (0, -h[1] / 2, 0), (0, h[1] / 2, 0),
                 (0, 0, -h[2] / 2), (0, 0, h[2] / 2)]

        def worst(scale):
            viol = -np.inf
            for c in range(3):
                vals = U[20 + c, [e] + nbrs]
                grad = sum(a0[q] * Jb[q][c] for q in range(8)) * scale
                for r in faces:
                    x = U[20 + c, e] + grad @ np.array(r)
                    viol = max(viol, x - vals.max(), vals.min() - x)
            return viol

        assert worst(alpha) <= 1e-14
        if alpha < 1.0:
            limited += 1
            assert worst(alpha * (1 + 1e-9) + 1e-12) > 0
    assert limited > 5
