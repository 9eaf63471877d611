"""Pins of the CPU oracle against what the paper and the mathematics fix.

None of these compares the oracle with itself: each checks a closed form, an
invariant, a textbook special case or a convergence order, chosen so that a dropped
term, a wrong sign or index, or a transposed operand fails at least one of them.
"""
import math

import numpy as np
import pytest

import workloads as W

G14 = 1.4
G53 = 5.0 / 3.0


def _order(errs, ns):
    return [math.log(errs[i] / errs[i + 1]) / math.log(ns[i + 1] / ns[i])
            for i in range(len(errs) - 1)]


# ------------------------------------------------------------------ L(U) pins
def test_free_stream_euler2d(oracle):
    """A uniform state has L(U) = 0 (checks face closure and the volume rule)."""
    m = oracle.Mesh.cartesian((7, 5), (0.0, -1.0), (1.0, 2.0))
    U = np.zeros((12, 35))
    U[0], U[3], U[6], U[9] = 1.3, 0.4, -0.2, 2.5
    L = oracle.rhs(m, U.reshape(-1), G14).reshape(12, -1)
    # L means carry 1/V and gradients 12/(V h^2): scale the roundoff bound.
    assert np.abs(L[0::3]).max() < 1e-13
    assert np.abs(L).max() < 1e-11


def test_free_stream_mhd3d(oracle):
    m = oracle.Mesh.cartesian((3, 4, 2), (0, 0, 0), (1.0, 1.0, 0.5))
    U = np.zeros((31, 24))
    U[0], U[4], U[8], U[12], U[16] = 1.1, 0.3, -0.2, 0.1, 3.0
    U[20], U[21], U[22] = 0.5, -0.4, 0.3
    L = oracle.rhs(m, U.reshape(-1), G53, mhd=True)
    assert np.abs(L).max() < 1e-11


def test_conservation_euler2d_limited(oracle):
    """Sum_e V_e u_e of every conserved variable is constant over steps
    (periodic box; face fluxes enter both neighbours with opposite signs)."""
    n = (12, 10)
    U = W.random_p1_state(n, (0, 0), (1, 1), G14, seed=3, amp=0.3)
    m = oracle.Mesh.cartesian(n, (0, 0), (1, 1))
    V = 1.0 / 120
    tot0 = U.reshape(12, -1)[0::3].sum(1) * V
    ref = np.abs(U.reshape(12, -1)[0::3]).sum(1) * V
    for _ in range(10):
        U = oracle.step(m, U, 0.004, G14, True)
    tot1 = U.reshape(12, -1)[0::3].sum(1) * V
    assert np.all(np.abs(tot1 - tot0) <= 1e-13 * ref)


def test_conservation_mhd3d(oracle):
    n = (4, 4, 4)
    U = W.random_p1_state(n, (0, 0, 0), (1, 1, 1), G53, seed=5, amp=0.2, mhd=True)
    m = oracle.Mesh.cartesian(n, (0, 0, 0), (1, 1, 1))
    U2 = U.reshape(31, -1)
    idx = [0, 4, 8, 12, 16, 20, 21, 22]
    tot0 = U2[idx].sum(1)
    ref = np.abs(U2[idx]).sum(1)
    for _ in range(4):
        U = oracle.step(m, U, 0.005, G53, True, mhd=True)
    tot1 = U.reshape(31, -1)[idx].sum(1)
    assert np.all(np.abs(tot1 - tot0) <= 1e-13 * ref)


@pytest.mark.parametrize("vel,aspect", [((1.0, 1.0), 1), ((1.0, 0.5), 2)])
def test_vortex_second_order(oracle, vel, aspect):
    """Exact advected isentropic vortex: L1 error of the density means falls at
    second order.  The second case uses non-square cells and a non-diagonal
    drift so that an x/y transposition cannot hide."""
    ns = [16, 32, 64]
    errs = []
    for n in ns:
        shape = (n, n * aspect)
        m = oracle.Mesh.cartesian(shape, (0, 0), (10, 10))
        U0 = W.project_cartesian(W.vortex_fields(0.0, G14, vel=vel), shape, (0, 0), (10, 10))
        U1, _ = oracle.run(m, U0, 0, G14, 0.3, False, t_end=1.0)
        ex = W.project_cartesian(W.vortex_fields(1.0, G14, vel=vel), shape, (0, 0), (10, 10),
                                 nq=6).reshape(12, -1)[0]
        errs.append(np.abs(U1.reshape(12, -1)[0] - ex).mean())
    orders = _order(errs, ns)
    assert min(orders) >= 1.8, (errs, orders)


@pytest.mark.parametrize("axis", [0, 1])
def test_acoustic_wave_second_order(oracle, axis):
    """The paper's 1D acoustic wave (sound speed 1, period 1): after one period
    the solution returns to its initial state; the L1 error is second order."""
    ns = [16, 32, 64]
    errs = []
    for n in ns:
        U0 = W.acoustic_state(n, axis=axis)
        shape = (n, 2) if axis == 0 else (2, n)
        m = oracle.Mesh.cartesian(shape, (0, 0), (1, 1))
        U1, _ = oracle.run(m, U0, 0, G53, 0.3, False, t_end=1.0)
        errs.append(np.abs(U1.reshape(12, -1)[0] - U0.reshape(12, -1)[0]).mean())
    orders = _order(errs, ns)
    assert min(orders) >= 1.8, (errs, orders)


def _fv_hll_means(Um, shape, h, gamma):
    """Textbook first-order Godunov update with the HLL flux (Davis speeds)."""
    nx, ny = shape
    rho, mx, my, E = [Um[k].reshape(ny, nx) for k in range(4)]

    def prim(r, a, b, e):
        u, v = a / r, b / r
        p = (gamma - 1) * (e - 0.5 * r * (u * u + v * v))
        return u, v, p, np.sqrt(gamma * p / r)

    def hll_x(L, R, normal_axis):
        (rl, al, bl, el), (rr, ar, br, er) = L, R
        ul, vl, pl, cl = prim(rl, al, bl, el)
        ur, vr, pr, cr = prim(rr, ar, br, er)
        if normal_axis == 1:  # rotate: the normal velocity is v
            ul, vl, ur, vr = vl, ul, vr, ur
        ql = [rl, al, bl, el]
        qr = [rr, ar, br, er]

        def F(q, un, p):
            r, a, b, e = q
            f = [r * un, a * un, b * un, (e + p) * un]
            f[1 + normal_axis] = f[1 + normal_axis] + p
            return f

        fl, fr = F(ql, ul, pl), F(qr, ur, pr)
        sl = np.minimum(ul - cl, ur - cr)
        sr = np.maximum(ul + cl, ur + cr)
        out = []
        for k in range(4):
            mid = (sr * fl[k] - sl * fr[k] + sl * sr * (qr[k] - ql[k])) / (sr - sl)
            out.append(np.where(sl >= 0, fl[k], np.where(sr <= 0, fr[k], mid)))
        return out

    q = [rho, mx, my, E]
    qe = [np.roll(a, -1, axis=1) for a in q]
    qn = [np.roll(a, -1, axis=0) for a in q]
    fx = hll_x(q, qe, 0)
    fy = hll_x(q, qn, 1)
    out = []
    for k in range(4):
        d = -(fx[k] - np.roll(fx[k], 1, axis=1)) / h[0] - (fy[k] - np.roll(fy[k], 1, axis=0)) / h[1]
        out.append(d.reshape(-1))
    return np.array(out)


def test_fv_reduction(oracle):
    """With zero gradients the mean equation is the finite-volume update (Sec.
    2.2: the means decouple and obey the FV equation)."""
    shape = (9, 7)
    U = W.random_p1_state(shape, (0, 0), (1, 1.4), G14, seed=11, amp=0.4).reshape(12, -1)
    U[1::3] = 0.0
    U[2::3] = 0.0
    m = oracle.Mesh.cartesian(shape, (0, 0), (1, 1.4))
    L = oracle.rhs(m, U.reshape(-1), G14).reshape(12, -1)
    ref = _fv_hll_means(U[0::3], shape, (1 / 9, 1.4 / 7), G14)
    assert np.allclose(L[0::3], ref, rtol=0, atol=1e-13 * np.abs(ref).max())


# ------------------------------------------------------------ Riemann solvers
def _euler_state(rng, dim=2):
    rho = rng.uniform(0.5, 2.0)
    v = rng.uniform(-1, 1, dim)
    p = rng.uniform(0.5, 2.0)
    return np.array([rho, *(rho * v), p / (G14 - 1) + 0.5 * rho * v @ v])


def _mhd_state(rng, bn=None, n=None):
    rho = rng.uniform(0.5, 2.0)
    v = rng.uniform(-1, 1, 3)
    p = rng.uniform(0.3, 2.0)
    B = rng.uniform(-1, 1, 3)
    if bn is not None:
        B = B - (B @ n) * n + bn * n
    return np.array([rho, *(rho * v), p / (G53 - 1) + 0.5 * rho * v @ v + 0.5 * B @ B, *B])


def _unit(rng, d):
    n = rng.normal(size=d)
    return n / np.linalg.norm(n)


def test_hll_invariants(oracle):
    rng = np.random.default_rng(7)
    for _ in range(200):
        uL, uR = _euler_state(rng), _euler_state(rng)
        n = _unit(rng, 2)
        F = oracle.hll(uL, uR, n, G14)
        # consistency
        assert np.allclose(oracle.hll(uL, uL, n, G14), oracle.flux(uL, n, G14), rtol=1e-14, atol=1e-14)
        # antisymmetry: swapping sides and flipping the normal negates the flux
        assert np.allclose(oracle.hll(uR, uL, -n, G14), -F, rtol=1e-13, atol=1e-13)
    # supersonic to the right: pure upwind
    uL = np.array([1.0, 5.0, 0.0, 0.6 / 0.4 + 12.5])
    uR = np.array([1.2, 6.0, 0.0, 0.7 / 0.4 + 15.0])
    assert np.array_equal(oracle.hll(uL, uR, [1.0, 0.0], G14), oracle.flux(uL, [1.0, 0.0], G14))
    assert np.array_equal(oracle.hll(uL, uR, [-1.0, 0.0], G14), oracle.flux(uR, [-1.0, 0.0], G14))


def _hllc_textbook(uL, uR, gamma):
    """HLLC (Toro, Riemann Solvers, ch. 10) along x for a 3D Euler state, with
    the HLLD outer speeds S_L = min(u) - max(c), S_R = max(u) + max(c)."""
    def prim(u):
        r = u[0]
        v = u[1:4] / r
        p = (gamma - 1) * (u[4] - 0.5 * r * v @ v)
        return r, v, p, math.sqrt(gamma * p / r)

    rl, vl, pl, cl = prim(uL)
    rr, vr, pr, cr = prim(uR)
    sl = min(vl[0], vr[0]) - max(cl, cr)
    sr = max(vl[0], vr[0]) + max(cl, cr)
    ss = (pr - pl + rl * vl[0] * (sl - vl[0]) - rr * vr[0] * (sr - vr[0])) / (
        rl * (sl - vl[0]) - rr * (sr - vr[0]))

    def F(u, v, p):
        return np.array([u[0] * v[0], u[1] * v[0] + p, u[2] * v[0], u[3] * v[0], (u[4] + p) * v[0]])

    def star(u, r, v, p, s):
        f = r * (s - v[0]) / (s - ss)
        return f * np.array([1, ss, v[1], v[2], u[4] / r + (ss - v[0]) * (ss + p / (r * (s - v[0])))])

    if sl >= 0:
        return F(uL, vl, pl)
    if sr <= 0:
        return F(uR, vr, pr)
    if ss >= 0:
        return F(uL, vl, pl) + sl * (star(uL, rl, vl, pl, sl) - uL)
    return F(uR, vr, pr) + sr * (star(uR, rr, vr, pr, sr) - uR)


def test_hlld_invariants(oracle):
    rng = np.random.default_rng(8)
    for _ in range(200):
        n = _unit(rng, 3)
        bn = rng.uniform(-1, 1)
        uL, uR = _mhd_state(rng, bn, n), _mhd_state(rng, bn, n)
        F = oracle.hlld(uL, uR, n, G53)
        assert np.allclose(oracle.hlld(uL, uL, n, G53), oracle.flux(uL, n, G53, mhd=True),
                           rtol=1e-13, atol=1e-13)
        assert np.allclose(oracle.hlld(uR, uL, -n, G53), -F, rtol=1e-12, atol=1e-12)
        # normal component of the induction flux vanishes
        assert abs(F[5:8] @ n) < 1e-13
        # rotation invariance: rotate states, fields and the normal together
        Q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
        if np.linalg.det(Q) < 0:
            Q[:, 0] *= -1

        def rot(u):
            return np.array([u[0], *(Q @ u[1:4]), u[4], *(Q @ u[5:8])])

        FR = oracle.hlld(rot(uL), rot(uR), Q @ n, G53)
        assert np.allclose(FR, rot(F), rtol=1e-11, atol=1e-11)


def test_hlld_reduces_to_hllc_without_field(oracle):
    rng = np.random.default_rng(9)
    for _ in range(200):
        uL = _mhd_state(rng)
        uR = _mhd_state(rng)
        for u in (uL, uR):
            B = u[5:8].copy()
            u[4] -= 0.5 * B @ B
            u[5:8] = 0.0
        F = oracle.hlld(uL, uR, [1.0, 0.0, 0.0], G53)
        ref = _hllc_textbook(uL[:5], uR[:5], G53)
        assert np.allclose(F[:5], ref, rtol=1e-12, atol=1e-12)
        assert np.all(F[5:] == 0.0)


def test_hlld_stationary_contact_and_tangential(oracle):
    """HLLD resolves an isolated stationary contact (density jump only, B_n != 0)
    and a stationary tangential discontinuity (B_n = 0, total pressure equal)
    exactly: zero mass flux."""
    n = np.array([1.0, 0.0, 0.0])
    B = np.array([0.7, 0.3, -0.2])
    p = 1.0
    uL = np.array([1.0, 0, 0, 0, p / (G53 - 1) + 0.5 * B @ B, *B])
    uR = np.array([0.3, 0, 0, 0, p / (G53 - 1) + 0.5 * B @ B, *B])
    F = oracle.hlld(uL, uR, n, G53)
    assert abs(F[0]) < 1e-15
    assert np.allclose(F, oracle.flux(uL, n, G53, mhd=True), atol=1e-14)
    # tangential discontinuity
    BL = np.array([0.0, 0.5, 0.1])
    BR = np.array([0.0, -0.2, 0.6])
    pL = 1.0
    pR = pL + 0.5 * (BL @ BL - BR @ BR)
    uL = np.array([1.0, 0, 0.3, 0, pL / (G53 - 1) + 0.5 * 0.09 + 0.5 * BL @ BL, *BL])
    uR = np.array([2.0, 0, -0.4, 0, pR / (G53 - 1) + 0.5 * 2 * 0.04 + 0.5 * BR @ BR, *BR])
    F = oracle.hlld(uL, uR, n, G53)
    assert abs(F[0]) < 1e-14
    assert abs(F[1] - (pL + 0.5 * BL @ BL)) < 1e-13


def test_hlld_isolated_rotational_discontinuity(oracle):
    """An isolated rotational (Alfven) discontinuity is resolved exactly, which pins the
    HLLD middle (Alfven) states that the contact and tangential cases leave free.  With
    normal field b, density rho and pressure continuous, the tangential field rotating
    at fixed magnitude and v_t - s B_t / sqrt(rho) continuous (s = sign(b) sign(u_n - V)),
    the jump conditions hold for the speed V = u_n - s |b| / sqrt(rho) (checked here:
    F(u_R) - F(u_L) = V (u_R - u_L)), so the exact flux on the face is F(u_L) for V > 0
    and F(u_R) for V < 0.  A two-wave HLL flux with the same outer speeds misses it."""
    rng = np.random.default_rng(21)
    n = np.array([1.0, 0.0, 0.0])
    for _ in range(200):
        rho, p = float(np.exp(rng.normal(0, 0.5))), float(np.exp(rng.normal(0, 0.5)))
        b = float(rng.uniform(0.2, 1.5)) * rng.choice([-1.0, 1.0])
        side = rng.choice([-1.0, 1.0])
        V = float(rng.uniform(-0.5, 0.5))
        un = side * abs(b) / math.sqrt(rho) + V
        mag = float(rng.uniform(0.1, 1.0))
        th = rng.uniform(0, 2 * math.pi, 2)
        Bt = [mag * np.array([math.cos(a), math.sin(a)]) for a in th]
        v0 = rng.normal(0, 0.3, 2)
        s = math.copysign(1.0, b) * side

        def state(bt):
            v = np.array([un, *(v0 + s * bt / math.sqrt(rho))])
            B = np.array([b, *bt])
            return np.array([rho, *(rho * v), p / (G53 - 1) + 0.5 * rho * v @ v + 0.5 * B @ B, *B])

        uL, uR = state(Bt[0]), state(Bt[1])
        FL = oracle.flux(uL, n, G53, mhd=True)
        FR = oracle.flux(uR, n, G53, mhd=True)
        assert np.allclose(FR - FL, V * (uR - uL), rtol=0, atol=1e-12)
        exact = FL if V > 0 else FR
        F = oracle.hlld(uL, uR, n, G53)
        assert np.allclose(F, exact, rtol=1e-13, atol=1e-13), (F, exact)
        if abs(V) < 0.1 and mag > 0.3 and abs(math.cos(th[0] - th[1])) < 0.5:
            # outer fast speeds (Davis), then the two-wave HLL average
            def cf(u):
                a2 = G53 * p / rho
                B2 = u[5:8] @ u[5:8] / rho
                return math.sqrt(0.5 * (a2 + B2 + math.sqrt((a2 + B2) ** 2 - 4 * a2 * b * b / rho)))
            SL = min(un - cf(uL), un - cf(uR))
            SR = max(un + cf(uL), un + cf(uR))
            Fh = (SR * FL - SL * FR + SL * SR * (uR - uL)) / (SR - SL)
            assert np.abs(Fh - exact).max() > 1e-3


# ------------------------------------------------------------------- limiter
def test_limiter_1d_closed_form(oracle):
    """On data varying along x only, the limited slope is
    min(g, 2 D+/h, 2 D-/h) for monotone increasing means with g > 0 (Sec. 2.5),
    and the means are untouched."""
    rng = np.random.default_rng(4)
    n = 24
    h = 1.0 / n
    means = np.cumsum(rng.uniform(0.1, 1.0, n)) * 0.01 + 1.0
    # periodic wrap breaks monotonicity at the ends: test interior cells
    g = rng.uniform(0.0, 3.0, n) * (means[1] - means[0]) / h
    U = np.zeros((12, n * 3))
    for v, base in ((0, 1.0), (1, 0.0), (2, 0.0), (3, 2.5)):
        U[3 * v] = np.tile(means if v == 0 else base + 0 * means, 3)
    U[1] = np.tile(g, 3)
    Ul = oracle.limit(oracle.Mesh.cartesian((n, 3), (0, 0), (1, 0.3)), U.reshape(-1)).reshape(12, -1)
    dp = np.roll(means, -1) - means
    dm = means - np.roll(means, 1)
    ref = np.minimum(g, np.minimum(2 * dp / h, 2 * dm / h))
    assert np.allclose(Ul[1][1:n - 1], ref[1:n - 1], rtol=1e-14, atol=0)
    assert np.array_equal(Ul[0::3], U[0::3])
    assert np.array_equal(Ul[2], U[2])


def test_limiter_bounds_and_smooth(oracle):
    n = (16, 16)
    m = oracle.Mesh.cartesian(n, (0, 0), (1, 1))
    U = W.random_p1_state(n, (0, 0), (1, 1), G14, seed=12, amp=0.3).reshape(12, -1)
    U2 = U.copy()
    U2[1::3] *= 3.0
    U2[2::3] *= -2.0
    Ul = oracle.limit(m, U2.reshape(-1)).reshape(12, -1)
    for v in range(4):
        gx, gy = U2[3 * v + 1], U2[3 * v + 2]
        lx, ly = Ul[3 * v + 1], Ul[3 * v + 2]
        with np.errstate(invalid="ignore", divide="ignore"):
            ax = np.where(gx != 0, lx / gx, 1.0)
            ay = np.where(gy != 0, ly / gy, 1.0)
        assert np.all((ax >= -1e-15) & (ax <= 1 + 1e-15))
        # one alpha per variable scales both components
        both = (gx != 0) & (gy != 0)
        assert np.allclose(ax[both], ay[both], rtol=1e-12)
        # limited extrapolation at face centroids stays within neighbour bounds
        mean = U2[3 * v].reshape(16, 16)
        nb = [np.roll(mean, s, a) for s in (1, -1) for a in (0, 1)]
        hi = np.maximum.reduce([mean] + nb).reshape(-1)
        lo = np.minimum.reduce([mean] + nb).reshape(-1)
        for sx, sy in ((0.5, 0), (-0.5, 0), (0, 0.5), (0, -0.5)):
            ext = U2[3 * v] + (lx * sx + ly * sy) / 16
            assert np.all(ext <= hi + 1e-13) and np.all(ext >= lo - 1e-13)


def test_limiter_keeps_resolved_sinusoid(oracle):
    """A well-resolved sine along x: cells whose face extrapolations stay inside
    the neighbour means keep alpha = 1 (exactly the unlimited gradient)."""
    n = 64
    x = (np.arange(n) + 0.5) / n
    U = np.zeros((12, n * 3))
    U[0] = np.tile(1.0 + 0.1 * np.sin(2 * np.pi * x), 3)
    U[1] = np.tile(0.1 * 2 * np.pi * np.cos(2 * np.pi * x), 3)
    U[9] = 2.5
    Ul = oracle.limit(oracle.Mesh.cartesian((n, 3), (0, 0), (1, 3.0 / n)), U.reshape(-1)).reshape(12, -1)
    mean = U[0][:n]
    g = U[1][:n]
    h = 1.0 / n
    inside = (mean + 0.5 * h * g <= np.maximum(np.roll(mean, -1), mean)) & \
             (mean - 0.5 * h * g >= np.minimum(np.roll(mean, 1), mean)) & \
             (mean + 0.5 * h * g >= np.minimum(np.roll(mean, -1), mean)) & \
             (mean - 0.5 * h * g <= np.maximum(np.roll(mean, 1), mean))
    assert inside.sum() > n // 2
    assert np.array_equal(Ul[1][:n][inside], g[inside])


# ----------------------------------------------------- geometry and B basis
def test_cartesian_mass_matrix_and_volume_rule(oracle):
    m = oracle.Mesh.cartesian((5, 3, 4), (0, 0, 0), (1.0, 0.6, 2.0))
    V, c, M, rq, wq = m.cell_geometry(7)
    h = np.array([0.2, 0.2, 0.5])
    assert math.isclose(V, h.prod(), rel_tol=1e-15)
    assert np.allclose(M, np.diag(V * h ** 2 / 12), rtol=1e-15, atol=0)
    # the 2-point tensor rule integrates every monomial of degree <= 3 per axis
    rng = np.random.default_rng(1)
    for _ in range(10):
        a = rng.integers(0, 4, 3)
        exact = V * np.prod([(h[d] / 2) ** a[d] / (a[d] + 1) if a[d] % 2 == 0 else 0.0
                             for d in range(3)])
        quad = float(np.sum(wq * np.prod(rq ** a, axis=1)))
        assert math.isclose(quad, exact, rel_tol=1e-13, abs_tol=1e-17)


def test_gram_matrix_closed_form(oracle):
    """The mass matrix of V4..V11 is their Gram matrix; on a box it is
    diag(m_y, m_z, m_x, m_z, m_x, m_y) (+) [[m_x+m_y, m_x], [m_x, m_x+m_z]]."""
    mx, my, mz = 0.3, 0.7, 1.1
    G = oracle.gram_B(np.diag([mx, my, mz]))
    ref = np.zeros((8, 8))
    ref[:6, :6] = np.diag([my, mz, mx, mz, mx, my])
    ref[6:, 6:] = [[mx + my, mx], [mx, mx + mz]]
    assert np.allclose(G, ref, rtol=0, atol=1e-15)
    # general moments: symmetric positive definite and equal to the Gram matrix
    # integrated by brute-force sampling of the basis at a point cloud
    rng = np.random.default_rng(2)
    P = rng.normal(size=(4000, 3)) * [1.0, 0.5, 2.0] + [0.2, -0.1, 0.3]
    P -= P.mean(0)
    M = P.T @ P / len(P)
    G = oracle.gram_B(M)
    assert np.allclose(G, G.T)
    assert np.all(np.linalg.eigvalsh(G) > 0)
    ev = np.array([[oracle.eval_B(np.zeros(3), np.eye(8)[j], p) for j in range(8)] for p in P[:500]])
    Pm = P[:500] - P[:500].mean(0)
    ev = np.array([[oracle.eval_B(np.zeros(3), np.eye(8)[j], p) for j in range(8)] for p in Pm])
    brute = np.einsum("pjc,pkc->jk", ev, ev) / len(Pm)
    assert np.allclose(oracle.gram_B(Pm.T @ Pm / len(Pm)), brute, rtol=1e-12, atol=1e-14)


def test_B_basis_divergence_free(oracle):
    """Each cell's own B polynomial has zero divergence: its outward flux
    through the cell boundary (exact face quadrature of a linear field) is zero,
    and the structural trace of the gradient vanishes."""
    rng = np.random.default_rng(3)
    h = np.array([0.3, 0.5, 0.2])
    s = 1 / math.sqrt(3)
    for _ in range(20):
        bbar = rng.normal(size=3)
        a = rng.normal(size=8)
        flux = 0.0
        for d in range(3):
            t1, t2 = [q for q in range(3) if q != d]
            A = h[t1] * h[t2]
            for side in (-1, 1):
                for s1 in (-1, 1):
                    for s2 in (-1, 1):
                        r = np.zeros(3)
                        r[d] = side * h[d] / 2
                        r[t1] = s1 * s * h[t1] / 2
                        r[t2] = s2 * s * h[t2] / 2
                        flux += side * A / 4 * oracle.eval_B(bbar, a, r)[d]
        assert abs(flux) < 1e-14
        # divergence by central differences of the linear field is exact
        div = sum((oracle.eval_B(bbar, a, np.eye(3)[d]) - oracle.eval_B(bbar, a, -np.eye(3)[d]))[d] / 2
                  for d in range(3))
        assert abs(div) < 1e-14


def test_stokes_divergence_of_projected_field(oracle):
    """A smooth divergence-free field projected on the basis: the Stokes
    estimate (face-averaged normal B, Sec. 2.6) is a small O(h^2) residual."""
    errs = []
    for n in (4, 8):
        U = W.random_p1_state((n, n, n), (0, 0, 0), (1, 1, 1), G53, seed=21, mhd=True)
        m = oracle.Mesh.cartesian((n, n, n), (0, 0, 0), (1, 1, 1))
        errs.append(np.abs(oracle.divB(m, U)).max())
    assert errs[1] < errs[0] / 3


# ------------------------------------------------------------- MHD convergence
@pytest.mark.parametrize("plane", [(0, 1), (1, 2), (0, 2)])
def test_alfven_wave_second_order(oracle, plane):
    """Circularly polarised Alfven wave (an exact nonlinear ideal-MHD solution)
    travelling obliquely in each coordinate plane: after one period the L1 error
    of B and v falls at second order.  Exercises every a_j coefficient of the
    divergence-free basis and the HLLD middle waves."""
    ns = [8, 16, 32]
    errs = []
    for n in ns:
        U0, shape, hi = W.alfven_state(n, plane)
        m = oracle.Mesh.cartesian(shape, (0, 0, 0), hi)
        T = 1.0 / math.sqrt(2.0)
        U1, _ = oracle.run(m, U0, 0, G53, 0.3, False, mhd=True, t_end=T)
        A = U1.reshape(31, -1)
        B0 = U0.reshape(31, -1)
        idx = [4, 8, 12, 20, 21, 22]  # momentum means and B means
        errs.append(np.abs(A[idx] - B0[idx]).mean())
    orders = _order(errs, ns)
    assert min(orders) >= 1.8, (errs, orders)


# ------------------------------------------------------------------- gresho
def test_gresho_ic_force_balance():
    """The printed Gresho profiles satisfy dp/dr = rho v_phi^2 / r (Sec. 3.4)."""
    r = np.linspace(0.01, 0.6, 2000)
    vphi = np.where(r < 0.2, 5 * r, np.where(r < 0.4, 2 - 5 * r, 0.0))
    p = np.where(r < 0.2, 5 + 12.5 * r * r,
                 np.where(r < 0.4, 9 + 12.5 * r * r - 20 * r + 4 * np.log(r / 0.2), 3 + 4 * math.log(2)))
    dpdr = np.gradient(p, r)
    inner = (np.abs(r - 0.2) > 0.01) & (np.abs(r - 0.4) > 0.01)
    assert np.allclose(dpdr[inner][1:-1], (vphi ** 2 / r)[inner][1:-1], atol=2e-3)
    # continuity of p at the breakpoints
    for rb in (0.2, 0.4):
        i = np.searchsorted(r, rb)
        assert abs(p[i] - p[i - 1]) < 1e-2


# ------------------------------------------------------------------- JVP
def test_step_jvp_matches_central_fd(oracle):
    """Dual-number directional derivative of one limited step against central
    finite differences of the step itself."""
    n = (8, 8)
    m = oracle.Mesh.cartesian(n, (0, 0), (1, 1))
    U = W.random_p1_state(n, (0, 0), (1, 1), G14, seed=31, amp=0.2)
    rng = np.random.default_rng(5)
    d = rng.normal(size=U.size) * 1e-2
    _, J = oracle.step_jvp(m, U, d, 0.01, G14, False)
    eps = 1e-5
    fd = (oracle.step(m, U + eps * d, 0.01, G14, False) - oracle.step(m, U - eps * d, 0.01, G14, False)) / (2 * eps)
    assert np.allclose(J, fd, rtol=1e-6, atol=1e-9 * np.abs(fd).max())
