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


# The 2D magnetic functions of Sec. 2.2 (V3, V4, V5 for (B_x, B_y)) and the
# Taylor functions x, y of B_z; used only to project initial fields.
def _vb2(r):
    x, y = r
    zero = 0.0 * x
    return [(y, zero, zero), (zero, x, zero), (x, -y, zero), (zero, zero, x), (zero, zero, y)]


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
    nb = 8 if dim == 3 else 5
    bfun = _vb if dim == 3 else _vb2
    bproj = np.zeros((nb, nc)) if mhd else None
    gram = np.zeros((nb, nb)) if mhd else None
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
            basis = bfun(r)
            for j in range(nb):
                bproj[j] += w * sum(vals[5 + c] * basis[j][c] for c in range(3))
                for i in range(nb):
                    gram[i, j] += w * sum(basis[i][c] * basis[j][c] for c in range(3))
    ncoef = nh * (1 + dim) + ((3 + nb) if mhd else 0)
    U = np.zeros((ncoef, nc))
    for v in range(nh):
        U[v * (1 + dim)] = means[v]
        for d in range(dim):
            U[v * (1 + dim) + 1 + d] = first[v, d] / second[d]
    if mhd:
        base = nh * (1 + dim)
        U[base:base + 3] = means[5:8]
        U[base + 3:base + 3 + nb] = np.linalg.solve(gram, bproj)
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


def random_p1_state(n, lo, hi, gamma, seed, amp=0.1, nmodes=4, kmax=3, mhd=False, bamp=0.03):
    """Smooth random state: rho = 1 + amp * sum of random modes, v likewise, p = 1
    (+ amp modes); MHD adds B = B0 + curl of a random vector potential of
    amplitude ``bamp`` (|B| stays O(2 pi kmax bamp)), B0 ~ U(-0.5, 0.5)*10 bamp."""
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
    b0 = rng.uniform(-0.5, 0.5, 3) * 10 * bamp if mhd else None

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
                th = sum(2 * math.pi * k[m][d] * (X[d] - lo[d]) / L[d] for d in range(dim)) + ph[m]
                g = [2 * math.pi * k[m][d] / L[d] * a[m] * np.cos(th) / len(a) * bamp
                     for d in range(dim)] + [0.0 * X[0]] * (3 - dim)
                # (curl A)_i = eps_ijk d_j A_k with A = e_c * sin(...)
                B[(c + 1) % 3] = B[(c + 1) % 3] + g[(c + 2) % 3]
                B[(c + 2) % 3] = B[(c + 2) % 3] - g[(c + 1) % 3]
        return _mhd_conserved(rho, vel, p, B, gamma)

    return project_cartesian(f, n, lo, hi, mhd=mhd)


# ---------------------------------------------------------------- MHD turbulence
def _c3_modes(seed):
    rng = np.random.default_rng(seed)
    kv = _modes(rng, 16, 4, 3, norm="l2")
    av = rng.normal(size=(16, 3))
    pv = rng.uniform(0, 2 * math.pi, 16)
    kA = _modes(rng, 16, 4, 3, norm="l2")
    aA = rng.normal(size=(16, 3))
    pA = rng.uniform(0, 2 * math.pi, 16)
    # B = curl A: mode m contributes 2 pi cos(theta) (k_m x a_m)
    qB = np.array([np.cross(2 * math.pi * kA[m], aA[m]) for m in range(16)])
    # rms rescaling from cell centres of a 16^3 grid (distinct integer modes
    # with |k| <= 4 are orthogonal on it)
    g = (np.arange(16) + 0.5) / 16
    S = np.stack(np.meshgrid(g, g, g, indexing="ij")).reshape(3, -1)
    vs = (av.T @ np.sin(2 * math.pi * kv @ S + pv[:, None]))
    bs = (qB.T @ np.cos(2 * math.pi * kA @ S + pA[:, None]))
    sv = 0.5 / math.sqrt(np.mean(np.sum(vs * vs, axis=0)))
    sb = 0.3 / math.sqrt(np.mean(np.sum(bs * bs, axis=0)))
    return kv, av * sv, pv, kA, qB * sb, pA


def c3_state(n=256, seed=1003, gamma=5.0 / 3.0, nq=None):
    """3D MHD on [0,1]^3: rho = 1, p = 1; v = sum_{m=1..16} a_m sin(2 pi k_m.x +
    phi_m) with integer k_m, 1 <= |k_m| <= 4, a_m ~ N(0, I3), rescaled to an rms
    |v| of 0.5; A from 16 modes drawn the same way, B = curl A, rescaled to an
    rms |B| of 0.3 (rms over cell centres).  P1 projection with an nq^3 Gauss
    rule per cell (nq = 3, or 2 from 128^3 up); each mode's phase at the cell
    centre is computed once and shifted to the quadrature points with the sum
    formulas (torch CPU tensors, float64)."""
    import torch
    nq = nq or (3 if n < 128 else 2)
    kv, av, pv, kA, qB, pA = _c3_modes(seed)
    h = 1.0 / n
    xs, ws = _gauss(nq)
    c = (torch.arange(n, dtype=torch.float64) + 0.5) * h
    nc = n ** 3
    # cell centres, x fastest
    Z, Y, X = torch.meshgrid(c, c, c, indexing="ij")
    X, Y, Z = X.reshape(-1), Y.reshape(-1), Z.reshape(-1)
    tp = 2 * math.pi

    def phases(k, ph):
        out = []
        for m in range(16):
            th = tp * (float(k[m][0]) * X + float(k[m][1]) * Y + float(k[m][2]) * Z) + float(ph[m])
            out.append((torch.sin(th), torch.cos(th)))
        return out

    Pv = phases(kv, pv)
    PA = phases(kA, pA)
    del X, Y, Z
    U = torch.zeros((31, nc), dtype=torch.float64)
    second = 0.0
    gram = np.zeros((8, 8))
    gv = [[1, 2, 3], [5, 6, 7], [9, 10, 11], [13, 14, 15], [17, 18, 19]]
    for idx in np.ndindex(nq, nq, nq):
        r = [xs[idx[d]] * h for d in range(3)]
        w = float(ws[idx[0]] * ws[idx[1]] * ws[idx[2]])
        vel = [torch.zeros(nc, dtype=torch.float64) for _ in range(3)]
        B = [torch.zeros(nc, dtype=torch.float64) for _ in range(3)]
        for m in range(16):
            dv = tp * float(kv[m] @ r)
            s_ = Pv[m][0] * math.cos(dv) + Pv[m][1] * math.sin(dv)
            for cc in range(3):
                vel[cc].add_(s_, alpha=float(av[m][cc]))
            dA = tp * float(kA[m] @ r)
            c_ = PA[m][1] * math.cos(dA) - PA[m][0] * math.sin(dA)
            for cc in range(3):
                B[cc].add_(c_, alpha=float(qB[m][cc]))
        rho = 1.0
        E = 1.0 / (gamma - 1.0) + 0.5 * (vel[0] ** 2 + vel[1] ** 2 + vel[2] ** 2) + \
            0.5 * (B[0] ** 2 + B[1] ** 2 + B[2] ** 2)
        cons = [None, vel[0], vel[1], vel[2], E]
        U[0] += w * rho
        for v in range(1, 5):
            U[4 * v].add_(cons[v], alpha=w)
            for d in range(3):
                U[gv[v][d]].add_(cons[v], alpha=w * r[d])
        for cc in range(3):
            U[20 + cc].add_(B[cc], alpha=w)
        basis = _vb([np.array(r[0]), np.array(r[1]), np.array(r[2])])
        for j in range(8):
            for cc in range(3):
                coef = float(basis[j][cc])
                if coef != 0.0:
                    U[23 + j].add_(B[cc], alpha=w * coef)
            for i in range(8):
                gram[i, j] += w * sum(float(basis[i][cc]) * float(basis[j][cc]) for cc in range(3))
        second += w * r[0] ** 2
    # gradients: first moments over second moments (same on every axis here);
    # rho is uniform so its gradient stays zero
    for v in range(1, 5):
        for d in range(3):
            U[gv[v][d]] /= second
    ginv = torch.as_tensor(np.linalg.inv(gram))
    U[23:31] = ginv @ U[23:31]
    return U.reshape(-1).numpy()


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


# ------------------------------------------------------------------- 2D MHD
def alfven2d_state(n, t=0.0, amp=0.1, p0=0.1, gamma=5.0 / 3.0):
    """Travelling circularly polarised Alfven wave on the unit square, an exact
    nonlinear solution of ideal MHD: rho = 1, p = p0, B_par = 1 along k = (1, 1),
    B_perp of magnitude ``amp`` rotating between the in-plane normal and z,
    v_perp = -B_perp (wavelength 1/sqrt 2, Alfven speed 1)."""
    kvec = np.array([1.0, 1.0])
    kn = np.linalg.norm(kvec)
    khat = np.array([1.0, 1.0, 0.0]) / kn
    e1 = np.array([-1.0, 1.0, 0.0]) / math.sqrt(2)
    e2 = np.array([0.0, 0.0, 1.0])

    def f(X, Y):
        ph = 2 * math.pi * (kvec[0] * X + kvec[1] * Y - kn * t)
        b1 = amp * np.sin(ph)
        b2 = amp * np.cos(ph)
        B = [khat[c] + b1 * e1[c] + b2 * e2[c] for c in range(3)]
        vel = [-(b1 * e1[c] + b2 * e2[c]) for c in range(3)]
        return _mhd_conserved(1.0 + 0.0 * X, vel, p0 + 0.0 * X, B, gamma)

    return project_cartesian(f, (n, n), (0.0, 0.0), (1.0, 1.0), mhd=True)


def orszag_tang_state(n, gamma=5.0 / 3.0, nq=None):
    """The paper's Orszag-Tang setup (Sec. 3.9) on the unit square: rho =
    gamma^2/(4 pi), p = gamma/(4 pi), v = (-sin 2 pi y, sin 2 pi x), and B =
    (-sin 2 pi y, sin 4 pi x) in the units of the cited setup, i.e. divided by
    sqrt(4 pi) in the units used here (magnetic pressure B^2/2).  ``n`` is the
    cell count per side or a pair (nx, ny)."""
    s4 = math.sqrt(4 * math.pi)
    shape = (n, n) if np.isscalar(n) else tuple(n)

    def f(X, Y):
        rho = gamma ** 2 / (4 * math.pi) + 0.0 * X
        p = gamma / (4 * math.pi) + 0.0 * X
        vel = [-np.sin(2 * math.pi * Y), np.sin(2 * math.pi * X), 0.0 * X]
        B = [-np.sin(2 * math.pi * Y) / s4, np.sin(4 * math.pi * X) / s4, 0.0 * X]
        return _mhd_conserved(rho, vel, p, B, gamma)

    return project_cartesian(f, shape, (0.0, 0.0), (1.0, 1.0), nq=nq, mhd=True)


def rotor_state(n, gamma=5.0 / 3.0, nq=None):
    """The paper's magnetic rotor (Sec. 3.8) on the unit square: a dense
    rotating disc (rho = 10 for r <= 0.1, tapered to 1 at r = 0.115), p = 0.5,
    B_x = 2.5/sqrt(4 pi), B_y = 0, the ambient fluid at rest."""
    r0, r1 = 0.1, 0.115

    def f(X, Y):
        dx, dy = X - 0.5, Y - 0.5
        r = np.sqrt(dx * dx + dy * dy)
        fr = (r1 - r) / (r1 - r0)
        inner, taper = r <= r0, (r > r0) & (r <= r1)
        rho = np.where(inner, 10.0, np.where(taper, 1.0 + 9.0 * fr, 1.0))
        rs = np.where(r > 0, r, 1.0)
        vx = np.where(inner, -dy / r0, np.where(taper, -fr * dy / rs, 0.0))
        vy = np.where(inner, dx / r0, np.where(taper, fr * dx / rs, 0.0))
        B = [2.5 / math.sqrt(4 * math.pi) + 0.0 * X, 0.0 * X, 0.0 * X]
        return _mhd_conserved(rho, [vx, vy, 0.0 * X], 0.5 + 0.0 * X, B, gamma)

    return project_cartesian(f, (n, n), (0.0, 0.0), (1.0, 1.0), nq=nq, mhd=True)


# ------------------------------------------------------------------ batched C5
def batched_instances(ninst=256, seed_sizes=1005, seed0=2005, gamma=5.0 / 3.0):
    """Sizes N_i = 64 + 32 * rng.integers(0, 15) (N in {64, ..., 512}) and the
    per-instance random-mode state on [0,1]^2: rho = 1 + 0.1 * (sum of 4 modes)/4
    with |k|_inf <= 3 and a ~ U[0.5, 1], v likewise, p = 1 (seed 2005 + i)."""
    rng = np.random.default_rng(seed_sizes)
    sizes = 64 + 32 * rng.integers(0, 15, ninst)
    return [int(s) for s in sizes]


def batched_state(N, seed, gamma=5.0 / 3.0):
    """P1 projection (4x4 Gauss points per cell) of instance ``seed``'s fields on
    an N x N periodic mesh of [0,1]^2.  Each mode sin(2 pi k.x + phi) is
    evaluated as a sum of products of per-axis sines and cosines, so the cost
    is O(N^2) multiply-adds per mode and quadrature point."""
    rng = np.random.default_rng(seed)

    def series():
        k = _modes(rng, 4, 3, 2)
        a = rng.uniform(0.5, 1.0, 4)
        ph = rng.uniform(0, 2 * math.pi, 4)
        return k, a, ph

    s_rho, s_u, s_v = series(), series(), series()
    h = 1.0 / N
    xc = (np.arange(N) + 0.5) * h

    xs, ws = _gauss(4)
    means = np.zeros((4, N, N))
    first = np.zeros((4, 2, N, N))
    second = 0.0
    for iy in range(4):
        for ix in range(4):
            rx, ry, w = xs[ix] * h, xs[iy] * h, ws[ix] * ws[iy]
            def at(s):  # (N, N) [y, x] values of a series at the shifted points
                k, a, ph = s
                out = np.zeros((N, N))
                for m in range(4):
                    A = 2 * math.pi * k[m][0] * (xc + rx) + ph[m]
                    B = 2 * math.pi * k[m][1] * (xc + ry)
                    out += a[m] * (np.cos(B)[:, None] * np.sin(A)[None, :] +
                                   np.sin(B)[:, None] * np.cos(A)[None, :])
                return out / 4.0

            rho = 1.0 + 0.1 * at(s_rho)
            vel = [0.1 * at(s_u), 0.1 * at(s_v)]
            vals = _euler_conserved(rho, vel, 1.0, gamma)
            for v in range(4):
                means[v] += w * vals[v]
                first[v, 0] += w * vals[v] * rx
                first[v, 1] += w * vals[v] * ry
            second += w * rx * rx
    U = np.zeros((12, N * N))
    for v in range(4):
        U[3 * v] = means[v].reshape(-1)
        U[3 * v + 1] = (first[v, 0] / second).reshape(-1)
        U[3 * v + 2] = (first[v, 1] / second).reshape(-1)
    return U.reshape(-1)
