"""Brute-force face-by-face pin of the oracle's L(U) on tiny periodic meshes.

The oracle computes L(U) cell by cell with the paper's folded per-cell algebra.
Here the same discrete operator is assembled the other way round, from the
weak form alone (Sec. 2.2, eqn:fv and eqn:dgderiv; the divergence-free B basis
of Sec. 2.2): for every cell and every test function phi of its space,

    d/dt int_K U phi = - sum_faces sum_g w_g phi(x_g) Fhat(x_g) . n
                       + sum_q w_q F(U(x_q)) : grad phi(x_q),

looping over FACES (each face's Gauss-point fluxes scattered to both cells with
opposite signs), then solving with a mass matrix computed here by quadrature
(Cartesian) or taken from the mesh descriptor's moments (polygons).  The
quadrature rules are the method's own (two Gauss points per 2D face, 2x2 per 3D
face, 2x2(x2) tensor Gauss in boxes, the 4-point principal-axis rule on
polygons), so the two sides compute the same operator and must agree to
rounding.  Physical fluxes and the HLL solver are written here in NumPy; the
HLLD solver is the oracle's (a library primitive with its own pins).
"""
import math

import numpy as np
import pytest

import workloads as W
from np_physics import flux as _flux, hll as _hll
from workloads import voronoi as WV

G53 = 5.0 / 3.0
G14 = 1.4
SQ3 = 1.0 / math.sqrt(3.0)


# --------------------------------------------------------------- the bases
def _b_basis(dim):
    """Vector test functions of B as 3x3 matrices J (psi(r) = J r), after the
    three constant unit vectors: 3D V4..V11, 2D V3..V5 plus the Taylor
    functions x, y of B_z (Sec. 2.2)."""
    def m(*entries):
        J = np.zeros((3, 3))
        for c, d, s in entries:
            J[c, d] = s
        return J
    if dim == 3:
        return [m((0, 1, 1)), m((0, 2, 1)), m((1, 0, 1)), m((1, 2, 1)), m((2, 0, 1)),
                m((2, 1, 1)), m((0, 0, 1), (1, 1, -1)), m((0, 0, 1), (2, 2, -1))]
    return [m((0, 1, 1)), m((1, 0, 1)), m((0, 0, 1), (1, 1, -1)), m((2, 0, 1)), m((2, 1, 1))]


class Layout:
    """Coefficient-major layout: hydro variable v has (mean, d/dx_1..d/dx_dim)
    at arrays v(1+dim)..; MHD then B means and the B basis coefficients."""

    def __init__(self, dim, mhd):
        self.dim, self.mhd = dim, mhd
        self.nh = 5 if mhd else dim + 2
        self.Jb = _b_basis(dim) if mhd else []
        self.ncoef = self.nh * (1 + dim) + (3 + len(self.Jb) if mhd else 0)

    def unpack(self, U, e):
        """(hydro coefficients [nh, 1+dim], B coefficients [3 + nfun])."""
        d1 = 1 + self.dim
        h = np.array([[U[v * d1 + c, e] for c in range(d1)] for v in range(self.nh)])
        b = U[self.nh * d1:, e] if self.mhd else None
        return h, b

    def evaluate(self, h, b, r):
        r3 = np.zeros(3)
        r3[:self.dim] = r[:self.dim]
        u = h[:, 0] + h[:, 1:] @ r3[:self.dim]
        if not self.mhd:
            return u
        B = b[:3].copy()
        for j, J in enumerate(self.Jb):
            B += b[3 + j] * (J @ r3)
        return np.concatenate([u, B])


# --------------------------------------------------------------- geometry
def _cartesian_geometry(n, lo, hi):
    """Cells (V, centroid) and faces (L, R, n, weights, Gauss points from L's
    centroid, R's centroid offset) of a periodic box mesh."""
    dim = len(n)
    h = np.array([(hi[d] - lo[d]) / n[d] for d in range(dim)])
    V = float(np.prod(h))
    ncell = int(np.prod(n))

    def idx(a):
        e = 0
        for d in reversed(range(dim)):
            e = e * n[d] + (a[d] % n[d])
        return e

    faces = []
    for e in range(ncell):
        a = []
        t = e
        for d in range(dim):
            a.append(t % n[d])
            t //= n[d]
        for d in range(dim):
            b = list(a)
            b[d] += 1
            nrm = np.zeros(3)
            nrm[d] = 1.0
            dLR = np.zeros(3)
            dLR[d] = h[d]
            tang = [q for q in range(dim) if q != d]
            A = float(np.prod([h[q] for q in tang]))
            pts = []
            for signs in np.ndindex(*([2] * len(tang))):
                r = np.zeros(3)
                r[d] = 0.5 * h[d]
                for q, s in zip(tang, signs):
                    r[q] = (2 * s - 1) * 0.5 * h[q] * SQ3
                pts.append(r)
            w = A / len(pts)
            faces.append((e, idx(b), nrm, [w] * len(pts), pts, dLR))
    # volume rule: tensor 2-point Gauss; mass-matrix rule: tensor 3-point Gauss
    vq = [np.array([(2 * s - 1) * 0.5 * h[d] * SQ3 for d, s in enumerate(sg)] + [0.0] * (3 - dim))
          for sg in np.ndindex(*([2] * dim))]
    vw = [V / len(vq)] * len(vq)
    g3, w3 = np.polynomial.legendre.leggauss(3)
    mq, mw = [], []
    for ii in np.ndindex(*([3] * dim)):
        mq.append(np.array([0.5 * h[d] * g3[i] for d, i in enumerate(ii)] + [0.0] * (3 - dim)))
        mw.append(V * np.prod([0.5 * w3[i] for i in ii]))
    cells = [dict(V=V, vq=vq, vw=vw, mq=mq, mw=mw) for _ in range(ncell)]
    return cells, faces


def _facelist_geometry(d):
    """Cells and faces of a 2D face-list mesh descriptor (the generator's
    geometry is the input both sides share)."""
    V, c, Mo = d["cell_volume"], d["cell_centroid"], d["cell_moments"]
    box = np.asarray(d["box"])
    cells = []
    for e in range(len(V)):
        M = np.array([[Mo[e, 0], Mo[e, 1]], [Mo[e, 1], Mo[e, 2]]])
        lam, ev = np.linalg.eigh(M)
        vq, vw = [], []
        for k in range(2):
            r = math.sqrt(2.0 * lam[k] / V[e])
            for s in (-1.0, 1.0):
                vq.append(np.array([s * r * ev[0, k], s * r * ev[1, k], 0.0]))
                vw.append(V[e] / 4.0)
        cells.append(dict(V=V[e], M=M, vq=vq, vw=vw))
    faces = []
    for f in range(len(d["face_area"])):
        L, R = int(d["face_cells"][f, 0]), int(d["face_cells"][f, 1])
        nrm = np.array([d["face_normal"][f, 0], d["face_normal"][f, 1], 0.0])
        A = d["face_area"][f]
        xf = d["face_centroid"][f] - c[L]
        t = np.array([-nrm[1], nrm[0]])
        o = A / (2.0 * math.sqrt(3.0))
        pts = [np.array([*(xf - o * t), 0.0]), np.array([*(xf + o * t), 0.0])]
        dLR = np.array([*(c[R] + d["face_shift"][f] * box - c[L]), 0.0])
        faces.append((L, R, nrm, [0.5 * A, 0.5 * A], pts, dLR))
    return cells, faces


# ------------------------------------------------------- the brute force
def brute_rhs(cells, faces, U, gamma, dim, mhd):
    lay = Layout(dim, mhd)
    nc = len(cells)
    U = np.asarray(U, dtype=np.float64).reshape(lay.ncoef, nc)
    nb = 1 + dim  # scalar test functions 1, r_1..r_dim
    Rh = np.zeros((nc, lay.nh, nb))
    Rb = np.zeros((nc, 3 + len(lay.Jb)))

    def phi(r):
        return np.concatenate([[1.0], r[:dim]])

    def psi(r):  # vector test functions as rows
        rows = [np.eye(3)[c] for c in range(3)] + [J @ r for J in lay.Jb]
        return np.array(rows)

    for (L, R, nrm, ws, pts, dLR) in faces:
        hL, bL = lay.unpack(U, L)
        hR, bR = lay.unpack(U, R)
        for w, rL in zip(ws, pts):
            rR = rL - dLR
            uL, uR = lay.evaluate(hL, bL, rL), lay.evaluate(hR, bR, rR)
            if mhd:
                import oracle
                bn = 0.5 * (uL[5:8] @ nrm + uR[5:8] @ nrm)
                uL[5:8] += (bn - uL[5:8] @ nrm) * nrm
                uR[5:8] += (bn - uR[5:8] @ nrm) * nrm
                F = oracle.hlld(uL, uR, nrm, gamma)
            else:
                F = _hll(uL, uR, nrm, gamma)
            Rh[L] -= w * np.outer(F[:lay.nh], phi(rL))
            Rh[R] += w * np.outer(F[:lay.nh], phi(rR))
            if mhd:
                Rb[L] -= w * psi(rL) @ F[5:8]
                Rb[R] += w * psi(rR) @ F[5:8]
    for e, cg in enumerate(cells):
        h, b = lay.unpack(U, e)
        for w, r in zip(cg["vw"], cg["vq"]):
            u = lay.evaluate(h, b, r)
            Fd = [_flux(u, np.eye(3)[d], gamma, mhd) for d in range(dim)]
            # grad phi: 0 for the constant, e_d for r_d
            for d in range(dim):
                Rh[e][:, 1 + d] += w * Fd[d][:lay.nh]
            if mhd:
                for j, J in enumerate(lay.Jb):
                    Rb[e][3 + j] += w * sum(J[c, d] * Fd[d][5 + c]
                                            for c in range(3) for d in range(dim))
    out = np.zeros((lay.ncoef, nc))
    for e, cg in enumerate(cells):
        if "M" in cg:  # polygon: int phi phi^T = diag(V, M) about the centroid
            Mh = np.zeros((nb, nb))
            Mh[0, 0] = cg["V"]
            Mh[1:, 1:] = cg["M"]
        else:
            Mh = sum(w * np.outer(phi(r), phi(r)) for w, r in zip(cg["mw"], cg["mq"]))
        sol = np.linalg.solve(Mh, Rh[e].T).T  # [nh, nb]
        for v in range(lay.nh):
            out[v * nb:(v + 1) * nb, e] = sol[v]
        if mhd:
            Mb = sum(w * psi(r) @ psi(r).T for w, r in zip(cg["mw"], cg["mq"]))
            out[lay.nh * nb:, e] = np.linalg.solve(Mb, Rb[e])
    return out


def _random_coeffs(lay, nc, seed, amp=0.15):
    """Independent random coefficients around a uniform physical state (no
    smoothness), so every term of the operator is active in every cell."""
    rng = np.random.default_rng(seed)
    U = amp * rng.uniform(-1, 1, (lay.ncoef, nc))
    nb = 1 + lay.dim
    U[0] += 1.0                                  # rho
    U[(lay.nh - 1) * nb] += 2.5                  # E
    if lay.mhd:
        U[lay.nh * nb: lay.nh * nb + 3] += np.array([0.3, -0.2, 0.25])[:, None]
        U[lay.nh * nb + 3:] *= 0.5
    return U


def _compare(oracle_out, brute, tol):
    scale = np.abs(oracle_out).max(axis=1, keepdims=True)
    err = np.abs(oracle_out - brute) / scale
    assert err.max() < tol, f"max relative deviation {err.max():.3e} (array {err.max(1).argmax()})"


@pytest.mark.parametrize("n", [(3, 3), (4, 4), (5, 3)])
def test_face_loop_euler2d_cartesian(oracle, n):
    lo, hi = (0.0, -0.5), (1.0, 0.7)
    lay = Layout(2, False)
    U = _random_coeffs(lay, n[0] * n[1], seed=11 + n[0])
    cells, faces = _cartesian_geometry(n, lo, hi)
    m = oracle.Mesh.cartesian(n, lo, hi)
    ref = oracle.rhs(m, U.reshape(-1), G53).reshape(lay.ncoef, -1)
    _compare(ref, brute_rhs(cells, faces, U, G53, 2, False), 1e-14)


@pytest.mark.parametrize("n", [(2, 2, 2), (3, 2, 2)])
def test_face_loop_mhd3d_cartesian(oracle, n):
    lo, hi = (0.0, 0.0, 0.0), (1.0, 0.8, 1.3)
    lay = Layout(3, True)
    U = _random_coeffs(lay, int(np.prod(n)), seed=21 + n[0])
    cells, faces = _cartesian_geometry(n, lo, hi)
    m = oracle.Mesh.cartesian(n, lo, hi)
    ref = oracle.rhs(m, U.reshape(-1), G53, mhd=True).reshape(lay.ncoef, -1)
    _compare(ref, brute_rhs(cells, faces, U, G53, 3, True), 1e-13)


def test_face_loop_mhd2d_cartesian(oracle):
    n, lo, hi = (3, 4), (0.0, 0.0), (1.0, 1.2)
    lay = Layout(2, True)
    U = _random_coeffs(lay, 12, seed=31)
    cells, faces = _cartesian_geometry(n, lo, hi)
    m = oracle.Mesh.cartesian(n, lo, hi)
    ref = oracle.rhs(m, U.reshape(-1), G53, mhd=True).reshape(lay.ncoef, -1)
    _compare(ref, brute_rhs(cells, faces, U, G53, 2, True), 1e-13)


@pytest.mark.parametrize("ncell,lloyd", [(20, 1), (23, 0)])
def test_face_loop_euler2d_voronoi(oracle, ncell, lloyd):
    d = WV.periodic_voronoi(ncell, seed=41 + ncell, lloyd=lloyd)
    lay = Layout(2, False)
    U = _random_coeffs(lay, ncell, seed=51)
    cells, faces = _facelist_geometry(d)
    m = oracle.Mesh.facelist(d)
    ref = oracle.rhs(m, U.reshape(-1), G53).reshape(lay.ncoef, -1)
    _compare(ref, brute_rhs(cells, faces, U, G53, 2, False), 1e-13)


def test_face_loop_detects_smooth_state_operator(oracle):
    """On a smooth projected state (the operator of the parity runs), the two
    assemblies also agree."""
    n, lo, hi = (4, 4), (0.0, 0.0), (1.0, 1.0)
    U = W.random_p1_state(n, lo, hi, G14, seed=5, amp=0.2).reshape(12, -1)
    cells, faces = _cartesian_geometry(n, lo, hi)
    m = oracle.Mesh.cartesian(n, lo, hi)
    ref = oracle.rhs(m, U.reshape(-1), G14).reshape(12, -1)
    _compare(ref, brute_rhs(cells, faces, U, G14, 2, False), 1e-13)
