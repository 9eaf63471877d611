"""Periodic Cartesian meshes and seeded initial states (P1 L2 projections).

Every random number comes from ``numpy.random.default_rng(seed)``; the recipes are
stated in each function.  Projections use tensor Gauss-Legendre quadrature per cell
(4 points per axis in 2D, 3 in 3D): the mean is the cell average of each conserved
field, the gradient is the first moment divided by the second moment (the P1
projection on a box), and B is projected onto the span of the divergence-free
functions V1..V11 of Sec. 2.2 by a Gram solve.
"""
from __future__ import annotations

import math

import numpy as np


def _gauss(nq: int):
    x, w = np.polynomial.legendre.leggauss(nq)
    return 0.5 * x, 0.5 * w  # nodes on [-1/2, 1/2], weights summing to 1


def cartesian_centres(n, lo, hi):
    """Cell-centre coordinates (x fastest) and spacings of a Cartesian mesh."""
    dim = len(n)
    h = [(hi[d] - lo[d]) / n[d] for d in range(dim)]
    axes = [lo[d] + (np.arange(n[d]) + 0.5) * h[d] for d in range(dim)]
    grids = np.meshgrid(*axes[::-1], indexing="ij")[::-1]  # x fastest in C order
    return [g.reshape(-1) for g in grids], h


# The divergence-free magnetic functions V4..V11 of Sec. 2.2 (offsets r from the
# centroid); used only to project initial fields.
def _vb(r):
    x, y, z = r
    zero = 0.0 * x
    return [
        (y, zero, zero), (z, zero, zero), (zero, x, zero), (zero, z, zero),
        (zero, zero, x), (zero, zero, y), (x, -y, zero), (x, zero, -z),
    ]


def project_cartesian(fields, n, lo, hi, nq=None, mhd=False):
    """P1 projection of ``fields(*X) -> list of conserved arrays`` on every cell.

    Returns the coefficient-major state as a flat float64 array.
    """
    dim = len(n)
    nq = nq or (4 if dim == 2 else 3)
    centres, h = cartesian_centres(n, lo, hi)
    nc = centres[0].size
    xs, ws = _gauss(nq)
    nh = 5 if mhd else dim + 2
    means = None
    first = None
    second = np.zeros(dim)
    bproj = np.zeros((8, nc)) if mhd else None
    gram = np.zeros((8, 8)) if mhd else None
    for idx in np.ndindex(*([nq] * dim)):
        r = [xs[idx[d]] * h[d] for d in range(dim)]
        w = float(np.prod([ws[i] for i in idx]))
        vals = fields(*[centres[d] + r[d] for d in range(dim)])
        if means is None:
            means = np.zeros((len(vals), nc))
            first = np.zeros((nh, dim, nc))
        for k, v in enumerate(vals):
            means[k] += w * v
        for v in range(nh):
            for d in range(dim):
                first[v, d] += w * vals[v] * r[d]
        for d in range(dim):
            second[d] += w * r[d] ** 2
        if mhd:
            basis = _vb(r)
            for j in range(8):
                bproj[j] += w * sum(vals[5 + c] * basis[j][c] for c in range(3))
                for i in range(8):
                    gram[i, j] += w * sum(basis[i][c] * basis[j][c] for c in range(3))
    ncoef = nh * (1 + dim) + (11 if mhd else 0)
    U = np.zeros((ncoef, nc))
    for v in range(nh):
        U[v * (1 + dim)] = means[v]
        for d in range(dim):
            U[v * (1 + dim) + 1 + d] = first[v, d] / second[d]
    if mhd:
        base = nh * (1 + dim)
        U[base:base + 3] = means[5:8]
        U[base + 3:base + 11] = np.linalg.solve(gram, bproj)
    return U.reshape(-1)


def _euler_conserved(rho, vel, p, gamma):
    ke = 0.5 * rho * sum(v * v for v in vel)
    return [rho] + [rho * v for v in vel] + [p / (gamma - 1.0) + ke]


def _mhd_conserved(rho, vel, p, B, gamma):
    ke = 0.5 * rho * sum(v * v for v in vel)
    me = 0.5 * sum(b * b for b in B)
    return [rho] + [rho * v for v in vel] + [p / (gamma - 1.0) + ke + me] + list(B)


# ----------------------------------------------------------- isentropic vortex
def vortex_fields(t=0.0, gamma=1.4, beta=5.0, x0=(5.0, 5.0), vel=(1.0, 1.0), L=10.0):
    """Shu's isentropic vortex advected by ``vel`` on the periodic box [0, L]^2.

    Background (rho, u, v, p) = (1, vel, 1).  Returns ``fields(X, Y)``.
    """

    def f(X, Y):
        xt = X - x0[0] - vel[0] * t
        yt = Y - x0[1] - vel[1] * t
        xt = (xt + 0.5 * L) % L - 0.5 * L
        yt = (yt + 0.5 * L) % L - 0.5 * L
        r2 = xt * xt + yt * yt
        e = np.exp(0.5 * (1.0 - r2))
        du = -beta / (2 * math.pi) * e * yt
        dv = beta / (2 * math.pi) * e * xt
        T = 1.0 - (gamma - 1.0) * beta ** 2 / (8 * gamma * math.pi ** 2) * e * e
        rho = T ** (1.0 / (gamma - 1.0))
        p = rho * T
        return _euler_conserved(rho, [vel[0] + du, vel[1] + dv], p, gamma)

    return f


def vortex_cell_means(n, t, gamma=1.4, vel=(1.0, 1.0), L=10.0, nq=6):
    """Exact cell averages of the conserved vortex fields at time t."""
    U = project_cartesian(vortex_fields(t, gamma, vel=vel, L=L), n, (0.0, 0.0), (L, L), nq=nq)
    return U.reshape(12, -1)[0::3]


def c1_state(n=64, seed=1001, noise=1e-6):
    """Isentropic vortex on [0,10]^2, gamma 1.4, plus uniform density noise of
    amplitude ``noise`` on the cell means (seeded)."""
    U = project_cartesian(vortex_fields(0.0, 1.4), (n, n), (0.0, 0.0), (10.0, 10.0))
    if noise:
        rng = np.random.default_rng(seed)
        U = U.reshape(12, -1)
        U[0] += noise * rng.uniform(-1.0, 1.0, U.shape[1])
        U = U.reshape(-1)
    return U


# ------------------------------------------------------------------ shear layer
def c2_state(n=2048, seed=1002, gamma=5.0 / 3.0):
    """Shear layer on [0,1]^2: rho=2, vx=0.5 for |y-1/2|<1/4, else rho=1, vx=-0.5;
    p=2.5; vy = 0.01 sum_{k=1..8} sin(2 pi k x + phi_k), phi_k ~ U[0, 2pi);
    then U(-1e-3, 1e-3) added to each cell-mean vy (momentum and energy adjusted
    so the mean pressure is unchanged)."""
    rng = np.random.default_rng(seed)
    phases = rng.uniform(0.0, 2 * math.pi, 8)

    def f(X, Y):
        inside = np.abs(Y - 0.5) < 0.25
        rho = np.where(inside, 2.0, 1.0)
        vx = np.where(inside, 0.5, -0.5)
        vy = 0.01 * sum(np.sin(2 * math.pi * k * X + phases[k - 1]) for k in range(1, 9))
        return _euler_conserved(rho, [vx, vy], 2.5 + 0.0 * X, gamma)

    U = project_cartesian(f, (n, n), (0.0, 0.0), (1.0, 1.0)).reshape(12, -1)
    dv = rng.uniform(-1e-3, 1e-3, U.shape[1])
    rho = U[0]
    my = U[6].copy()
    U[6] = my + rho * dv
    U[9] += my * dv + 0.5 * rho * dv * dv
    return U.reshape(-1)


# ---------------------------------------------------------------- random modes
def _modes(rng, nmodes, kmax, dim, norm="inf"):
    ks = []
    while len(ks) < nmodes:
        k = rng.integers(-kmax, kmax + 1, dim)
        if not np.any(k):
            continue
        if norm == "l2" and np.linalg.norm(k) > kmax:
            continue
        ks.append(k)
    return np.array(ks)


def random_p1_state(n, lo, hi, gamma, seed, amp=0.1, nmodes=4, kmax=3, mhd=False, bamp=0.3):
    """Smooth random state: rho = 1 + amp * sum of random modes, v likewise, p = 1
    (+ amp modes); MHD adds B = B0 + curl of a random vector potential."""
    rng = np.random.default_rng(seed)
    dim = len(n)
    L = np.array([hi[d] - lo[d] for d in range(dim)])

    def series(nm):
        k = _modes(rng, nm, kmax, dim)
        a = rng.uniform(0.5, 1.0, nm)
        ph = rng.uniform(0, 2 * math.pi, nm)
        return k, a, ph

    sr, sp = series(nmodes), series(nmodes)
    sv = [series(nmodes) for _ in range(3 if mhd else dim)]
    sa = [series(nmodes) for _ in range(3)] if mhd else None
    b0 = rng.uniform(-0.5, 0.5, 3) * bamp if mhd else None

    def ev(X, s):
        k, a, ph = s
        out = 0.0 * X[0]
        for m in range(len(a)):
            th = sum(2 * math.pi * k[m][d] * (X[d] - lo[d]) / L[d] for d in range(dim)) + ph[m]
            out = out + a[m] * np.sin(th)
        return out / len(a)

    def f(*X):
        rho = 1.0 + amp * ev(X, sr)
        p = 1.0 + amp * ev(X, sp)
        vel = [amp * ev(X, s) for s in sv]
        if not mhd:
            return _euler_conserved(rho, vel, p, gamma)
        # B = b0 + curl A, A_c = sum a sin(theta): curl computed analytically.
        B = [b0[c] + 0.0 * X[0] for c in range(3)]
        for c in range(3):
            k, a, ph = sa[c]
            for m in range(len(a)):
                th = sum(2 * math.pi * k[m][d] * (X[d] - lo[d]) / L[d] for d in range(3)) + ph[m]
                g = [2 * math.pi * k[m][d] / L[d] * a[m] * np.cos(th) / len(a) * bamp
                     for d in range(3)]
                # (curl A)_i = eps_ijk d_j A_k with A = e_c * sin(...)
                B[(c + 1) % 3] = B[(c + 1) % 3] + g[(c + 2) % 3]
                B[(c + 2) % 3] = B[(c + 2) % 3] - g[(c + 1) % 3]
        return _mhd_conserved(rho, vel, p, B, gamma)

    return project_cartesian(f, n, lo, hi, mhd=mhd)


# ---------------------------------------------------------------- MHD turbulence
def c3_state(n=256, seed=1003, gamma=5.0 / 3.0, nq=3):
    """3D MHD on [0,1]^3: rho = 1, p = 1; v = sum_{m=1..16} a_m sin(2 pi k_m.x +
    phi_m) with integer k_m, 1 <= |k_m| <= 4, a_m ~ N(0, I3), rescaled to an rms
    |v| of 0.5; A from 16 modes drawn the same way, B = curl A, rescaled to an
    rms |B| of 0.3 (rms over cell centres)."""
    rng = np.random.default_rng(seed)
    kv = _modes(rng, 16, 4, 3, norm="l2")
    av = rng.normal(size=(16, 3))
    pv = rng.uniform(0, 2 * math.pi, 16)
    kA = _modes(rng, 16, 4, 3, norm="l2")
    aA = rng.normal(size=(16, 3))
    pA = rng.uniform(0, 2 * math.pi, 16)
    two_pi = 2 * math.pi

    def vfield(X):
        out = [0.0 * X[0] for _ in range(3)]
        for m in range(16):
            s = np.sin(two_pi * (kv[m][0] * X[0] + kv[m][1] * X[1] + kv[m][2] * X[2]) + pv[m])
            for c in range(3):
                out[c] = out[c] + av[m][c] * s
        return out

    def bfield(X):
        out = [0.0 * X[0] for _ in range(3)]
        for m in range(16):
            cth = np.cos(two_pi * (kA[m][0] * X[0] + kA[m][1] * X[1] + kA[m][2] * X[2]) + pA[m])
            q = np.cross(two_pi * kA[m], aA[m])
            for c in range(3):
                out[c] = out[c] + q[c] * cth
        return out

    # rms rescaling from a coarse sample of cell centres (distinct integer modes
    # are orthogonal on the grid, so any grid of >= 9 points per axis is exact).
    ns = 16
    g = (np.arange(ns) + 0.5) / ns
    S = np.meshgrid(g, g, g, indexing="ij")
    S = [s.reshape(-1) for s in S]
    vs = vfield(S)
    bs = bfield(S)
    sv = 0.5 / math.sqrt(np.mean(sum(v * v for v in vs)))
    sb = 0.3 / math.sqrt(np.mean(sum(b * b for b in bs)))

    def f(X, Y, Z):
        Xs = (X, Y, Z)
        vel = [sv * v for v in vfield(Xs)]
        B = [sb * b for b in bfield(Xs)]
        one = 1.0 + 0.0 * X
        return _mhd_conserved(one, vel, one, B, gamma)

    return project_cartesian(f, (n, n, n), (0.0,) * 3, (1.0,) * 3, nq=nq, mhd=True)


# -------------------------------------------------------------- paper's tests
def acoustic_state(n, t=0.0, ny=2, axis=0, amp=1e-6):
    """The 1D acoustic wave of Sec. 3.1: rho = 1, p = 3/5, gamma = 5/3 (sound speed
    1), unit wavelength in a unit periodic box, amplitude 1e-6, right-moving;
    laid along ``axis`` of a 2D mesh with ``ny`` cells across."""
    gamma = 5.0 / 3.0

    def f(X, Y):
        s = X if axis == 0 else Y
        d = amp * np.sin(2 * math.pi * (s - t))
        rho = 1.0 + d
        u = d  # c * drho / rho0 with c = 1, rho0 = 1
        p = 0.6 + d  # c^2 drho
        vel = [u, 0.0 * X] if axis == 0 else [0.0 * X, u]
        return _euler_conserved(rho, vel, p, gamma)

    shape = (n, ny) if axis == 0 else (ny, n)
    return project_cartesian(f, shape, (0.0, 0.0), (1.0, 1.0))


def gresho_state(n, gamma=5.0 / 3.0):
    """Gresho vortex of Sec. 3.4 on [0,1]^2 centred at (1/2, 1/2): rho = 1 and the
    printed piecewise v_phi(r), p(r)."""

    def f(X, Y):
        dx, dy = X - 0.5, Y - 0.5
        r = np.sqrt(dx * dx + dy * dy)
        vphi = np.where(r < 0.2, 5 * r, np.where(r < 0.4, 2 - 5 * r, 0.0))
        rs = np.maximum(r, 1e-300)
        p = np.where(r < 0.2, 5 + 12.5 * r * r,
                     np.where(r < 0.4, 9 + 12.5 * r * r - 20 * r + 4 * np.log(rs / 0.2),
                              3 + 4 * math.log(2.0)))
        vx = -vphi * dy / rs
        vy = vphi * dx / rs
        return _euler_conserved(1.0 + 0.0 * X, [vx, vy], p, gamma)

    return project_cartesian(f, (n, n), (0.0, 0.0), (1.0, 1.0))


def alfven_state(n, plane=(0, 1), t=0.0, amp=0.1, p0=0.1, gamma=5.0 / 3.0):
    """Travelling circularly polarised Alfven wave, an exact nonlinear solution of
    ideal MHD: rho = 1, p = p0, B_par = 1, B_perp of magnitude ``amp`` rotating
    with phase 2 pi (k.x - t |k|) and v_perp = -B_perp.  The wave vector is
    (1, 1) in the given coordinate plane of the unit cube (wavelength 1/sqrt 2,
    Alfven speed 1, period 1/sqrt 2).  Mesh n x n cells in that plane and one cell
    across it."""
    a, b = plane
    third = 3 - a - b
    kvec = np.zeros(3)
    kvec[a] = kvec[b] = 1.0
    khat = kvec / np.linalg.norm(kvec)
    e1 = np.zeros(3)
    e1[a], e1[b] = -1.0 / math.sqrt(2), 1.0 / math.sqrt(2)
    e2 = np.zeros(3)
    e2[third] = 1.0
    kn = np.linalg.norm(kvec)

    def f(X, Y, Z):
        Xs = (X, Y, Z)
        ph = 2 * math.pi * (sum(kvec[d] * Xs[d] for d in range(3)) - kn * t)
        b1 = amp * np.sin(ph)
        b2 = amp * np.cos(ph)
        B = [khat[c] + b1 * e1[c] + b2 * e2[c] for c in range(3)]
        vel = [-(b1 * e1[c] + b2 * e2[c]) for c in range(3)]
        return _mhd_conserved(1.0 + 0.0 * X, vel, p0 + 0.0 * X, B, gamma)

    shape = [1, 1, 1]
    shape[a] = shape[b] = n
    hi = [1.0, 1.0, 1.0]
    hi[third] = 1.0 / n
    return project_cartesian(f, tuple(shape), (0.0, 0.0, 0.0), tuple(hi), mhd=True), tuple(shape), tuple(hi)


# ------------------------------------------------------------------ batched C5
def batched_instances(ninst=256, seed_sizes=1005, seed0=2005, gamma=5.0 / 3.0):
    """Sizes N_i = 64 + 32 * rng.integers(0, 15) (N in {64, ..., 512}) and the
    per-instance random-mode state on [0,1]^2: rho = 1 + 0.1 * (sum of 4 modes)/4
    with |k|_inf <= 3 and a ~ U[0.5, 1], v likewise, p = 1 (seed 2005 + i)."""
    rng = np.random.default_rng(seed_sizes)
    sizes = 64 + 32 * rng.integers(0, 15, ninst)
    return [int(s) for s in sizes]


def batched_state(N, seed, gamma=5.0 / 3.0):
    rng = np.random.default_rng(seed)

    def series():
        k = _modes(rng, 4, 3, 2)
        a = rng.uniform(0.5, 1.0, 4)
        ph = rng.uniform(0, 2 * math.pi, 4)
        return k, a, ph

    s_rho, s_u, s_v = series(), series(), series()

    def ev(X, Y, s):
        k, a, ph = s
        return sum(a[m] * np.sin(2 * math.pi * (k[m][0] * X + k[m][1] * Y) + ph[m])
                   for m in range(4)) / 4.0

    def f(X, Y):
        rho = 1.0 + 0.1 * ev(X, Y, s_rho)
        vel = [0.1 * ev(X, Y, s_u), 0.1 * ev(X, Y, s_v)]
        return _euler_conserved(rho, vel, 1.0 + 0.0 * X, gamma)

    return project_cartesian(f, (N, N), (0.0, 0.0), (1.0, 1.0))
