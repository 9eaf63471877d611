// Plain FP64 CPU oracle for the second-order centroidal-Taylor discontinuous
// Galerkin scheme (Mocz et al. 2013, "A discontinuous Galerkin method for
// solving the fluid and MHD equations in astrophysical simulations").
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
// call this file; only the tests, the smoke check and the CPU-baseline leg of
// the benchmark do.  It shares no code, header, table or constant with the
// GPU library: everything here is written out from the paper's equations.
//
// What it computes (each function cites the passage it follows):
//   * the semi-discrete DG right-hand side L(U) of the weak form, Sec. 2.2
//     eqn:dg, eqn:fv, eqn:dgderiv, eqn:fv3d, eqn:dgderiv3d, eqn:GalerkUpdate,
//     with the locally divergence-free 3D magnetic basis V1..V11 of Sec. 2.2;
//   * the Arepo slope limiter of Sec. 2.5 (alpha = min(1, min_j psi_ij));
//   * the HLL flux (Euler) and the HLLD flux (MHD, Miyoshi & Kusano 2005, the
//     solver named in Sec. 2.3), normal B averaged at the face (Sec. 2.6);
//   * one SSP-RK2 step with the limiter applied at the start of each stage;
//   * the CFL time step; the Stokes divergence estimator of Sec. 2.6.
//
// Readings taken where the paper is silent (listed in full in the design
// notes): two Gauss points per 2D face / 2x2 per 3D face; 2-point tensor Gauss
// volume rules on Cartesian cells and the 4-point principal-axis rule on
// polygonal cells; the limiter works on conserved coefficients and uses one
// common alpha for the three B components; the mass matrix of the B basis is
// the Gram matrix of V4..V11 (the printed 8x8 matrix has typos).
//
// Everything is templated on the scalar so that a dual-number type gives exact
// directional derivatives (J v) of the step for adjoint checks.
//
// Parity pins live in tests/ (convergence on exact solutions, conservation,
// free-stream preservation, FV reduction, Riemann-solver invariants, limiter
// closed forms, Gram/mass-matrix closed forms, divergence-free basis; a
// face-by-face NumPy assembly of the weak form on tiny meshes; the CFL step's
// closed forms on boxes; the signal speed as the largest eigenvalue of the flux
// Jacobian; where HLLD's outer speeds switch to the upwind flux; the common
// field alpha's 1D closed form).  One reading stays shared rather than pinned:
// the switch of HLLD's star states to the outer values when its denominator is
// degenerate (a tolerance of 1e-12 relative).

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

// ---------------------------------------------------------------- scalars --
struct Dual {
  double v, d;
  Dual() : v(0), d(0) {}
  Dual(double a) : v(a), d(0) {}
  Dual(double a, double b) : v(a), d(b) {}
};
inline Dual operator+(Dual a, Dual b) { return {a.v + b.v, a.d + b.d}; }
inline Dual operator-(Dual a, Dual b) { return {a.v - b.v, a.d - b.d}; }
inline Dual operator-(Dual a) { return {-a.v, -a.d}; }
inline Dual operator*(Dual a, Dual b) { return {a.v * b.v, a.d * b.v + a.v * b.d}; }
inline Dual operator/(Dual a, Dual b) {
  double q = a.v / b.v;
  return {q, (a.d - q * b.d) / b.v};
}
inline Dual& operator+=(Dual& a, Dual b) { a = a + b; return a; }
inline Dual& operator-=(Dual& a, Dual b) { a = a - b; return a; }
inline Dual& operator*=(Dual& a, Dual b) { a = a * b; return a; }
inline bool operator<(Dual a, Dual b) { return a.v < b.v; }
inline bool operator>(Dual a, Dual b) { return a.v > b.v; }
inline bool operator<=(Dual a, Dual b) { return a.v <= b.v; }
inline bool operator>=(Dual a, Dual b) { return a.v >= b.v; }
inline bool operator==(Dual a, Dual b) { return a.v == b.v; }

inline double val(double a) { return a; }
inline double val(const Dual& a) { return a.v; }
inline double dsqrt(double a) { return std::sqrt(a); }
inline Dual dsqrt(Dual a) {
  double s = std::sqrt(a.v);
  return {s, a.d / (2.0 * s)};
}
inline double dabs(double a) { return std::fabs(a); }
inline Dual dabs(Dual a) { return a.v < 0 ? -a : a; }
// min/max return the first argument on ties (the branch an adjoint follows).
template <class T> inline T dmin(T a, T b) { return (b < a) ? b : a; }
template <class T> inline T dmax(T a, T b) { return (b > a) ? b : a; }
template <class T> inline bool finite(T a) { return std::isfinite(val(a)); }
inline double dpow(double a, double e) { return std::pow(a, e); }
inline Dual dpow(Dual a, double e) {
  double p = std::pow(a.v, e);
  return {p, e * p / a.v * a.d};
}

// ------------------------------------------------------------------- mesh --
// A face f joins cells L and R; its unit normal n points from L to R.
// Positions are offsets in the local frame of L's centroid (Sec. 2.2 writes the
// expansion in coordinates with origin at the centroid): rc is the face
// centroid, rg the Gauss points, and dLR the centroid of R's periodic image
// next to L.  Offsets from R's centroid are these minus dLR.
struct FaceGeo {
  int64_t L, R;
  double n[3];
  double A;
  double rc[3];
  double dLR[3];
  int ng;
  double rg[4][3];
  double wg[4];
};

// Volume geometry of one cell: volume, centroid, inverse second-moment
// matrix, and the volume quadrature (offsets from the centroid, weights).
struct CellGeo {
  double V;
  double c[3];
  double M[3][3];
  int nq;
  double rq[8][3];
  double wq[8];
};

struct Mesh {
  int dim = 2;
  int kind = 0;  // 0 periodic Cartesian, 1 face list (2D)
  int64_t nc = 0, nf = 0;
  // Cartesian
  int64_t N[3] = {1, 1, 1};
  double lo[3] = {0, 0, 0}, h[3] = {1, 1, 1};
  // face list
  double box[3] = {1, 1, 1};
  std::vector<double> cV, cc, cM;            // per cell
  std::vector<int64_t> fL, fR;               // per face
  std::vector<double> fn, fA, fx, fsh;       // per face
  std::vector<int64_t> cptr, cf;             // CSR cell -> (face, side)
  std::vector<int8_t> cside;

  int64_t cidx(int64_t i, int64_t j, int64_t k) const {
    i = ((i % N[0]) + N[0]) % N[0];
    j = ((j % N[1]) + N[1]) % N[1];
    k = ((k % N[2]) + N[2]) % N[2];
    return (k * N[1] + j) * N[0] + i;
  }
  void cijk(int64_t e, int64_t& i, int64_t& j, int64_t& k) const {
    i = e % N[0];
    j = (e / N[0]) % N[1];
    k = e / (N[0] * N[1]);
  }

  // Faces of cell e as (face id, side) pairs; side 0 means e is the L cell.
  // Cartesian order: -x, +x, -y, +y, -z, +z.
  int cell_faces(int64_t e, int64_t* f, int* side) const {
    if (kind == 0) {
      int64_t i, j, k;
      cijk(e, i, j, k);
      int m = 0;
      for (int d = 0; d < dim; ++d) {
        int64_t a[3] = {i, j, k};
        a[d] -= 1;
        f[m] = d * nc + cidx(a[0], a[1], a[2]);
        side[m] = 1;
        ++m;
        f[m] = d * nc + e;
        side[m] = 0;
        ++m;
      }
      return m;
    }
    int m = 0;
    for (int64_t p = cptr[e]; p < cptr[e + 1]; ++p) {
      f[m] = cf[p];
      side[m] = cside[p];
      ++m;
    }
    return m;
  }

  void face(int64_t f, FaceGeo& g) const {
    if (kind == 0) {
      // Face on the +d side of cell e.  2-point Gauss-Legendre per axis of
      // the face (tensor product in 3D).
      int d = (int)(f / nc);
      int64_t e = f % nc;
      int64_t i, j, k;
      cijk(e, i, j, k);
      int64_t a[3] = {i, j, k};
      a[d] += 1;
      g.L = e;
      g.R = cidx(a[0], a[1], a[2]);
      double A = 1.0;
      for (int q = 0; q < dim; ++q)
        if (q != d) A *= h[q];
      g.A = A;
      // The face sits half a cell from L's centroid along d; R's centroid (or
      // its periodic image) one cell away.
      for (int q = 0; q < 3; ++q) {
        g.n[q] = (q == d) ? 1.0 : 0.0;
        g.rc[q] = (q == d) ? 0.5 * h[q] : 0.0;
        g.dLR[q] = (q == d) ? h[q] : 0.0;
      }
      const double s = 1.0 / std::sqrt(3.0);
      if (dim == 2) {
        int t = 1 - d;  // the tangential axis
        g.ng = 2;
        for (int p = 0; p < 2; ++p) {
          for (int q = 0; q < 3; ++q) g.rg[p][q] = g.rc[q];
          g.rg[p][t] += (p == 0 ? -1.0 : 1.0) * 0.5 * h[t] * s;
          g.wg[p] = 0.5 * A;
        }
      } else {
        int t1 = (d + 1) % 3, t2 = (d + 2) % 3;
        if (t1 > t2) std::swap(t1, t2);
        g.ng = 4;
        int p = 0;
        for (int s1 = -1; s1 <= 1; s1 += 2)
          for (int s2 = -1; s2 <= 1; s2 += 2) {
            for (int q = 0; q < 3; ++q) g.rg[p][q] = g.rc[q];
            g.rg[p][t1] += s1 * 0.5 * h[t1] * s;
            g.rg[p][t2] += s2 * 0.5 * h[t2] * s;
            g.wg[p] = 0.25 * A;
            ++p;
          }
      }
      return;
    }
    // Face list (2D): a straight segment with centroid xc and length A;
    // Gauss points at xc -+ A/(2 sqrt 3) t with t = (-n_y, n_x).
    g.L = fL[f];
    g.R = fR[f];
    g.A = fA[f];
    for (int q = 0; q < 3; ++q) {
      g.n[q] = q < 2 ? fn[2 * f + q] : 0.0;
      g.rc[q] = q < 2 ? fx[2 * f + q] - cc[2 * g.L + q] : 0.0;
      g.dLR[q] = q < 2 ? cc[2 * g.R + q] + fsh[2 * f + q] - cc[2 * g.L + q] : 0.0;
    }
    double t[2] = {-g.n[1], g.n[0]};
    double o = g.A / (2.0 * std::sqrt(3.0));
    g.ng = 2;
    for (int p = 0; p < 2; ++p) {
      double sg = p == 0 ? -1.0 : 1.0;
      g.rg[p][0] = g.rc[0] + sg * o * t[0];
      g.rg[p][1] = g.rc[1] + sg * o * t[1];
      g.rg[p][2] = 0.0;
      g.wg[p] = 0.5 * g.A;
    }
  }

  void cell(int64_t e, CellGeo& g) const {
    std::memset(&g, 0, sizeof(g));
    if (kind == 0) {
      int64_t i, j, k;
      cijk(e, i, j, k);
      int64_t a[3] = {i, j, k};
      g.V = 1.0;
      for (int d = 0; d < dim; ++d) {
        g.V *= h[d];
        g.c[d] = lo[d] + (a[d] + 0.5) * h[d];
      }
      // Second moments of a box about its centroid: V h_d^2 / 12 on the
      // diagonal (the mass matrix of Sec. 2.2).
      for (int d = 0; d < dim; ++d) g.M[d][d] = g.V * h[d] * h[d] / 12.0;
      // Tensor 2-point Gauss rule, points at -+ h/(2 sqrt 3) on each axis.
      const double s = 1.0 / std::sqrt(3.0);
      int nq = 1 << dim;
      g.nq = nq;
      for (int q = 0; q < nq; ++q) {
        for (int d = 0; d < dim; ++d) {
          int bit = (q >> (dim - 1 - d)) & 1;
          g.rq[q][d] = (bit ? 1.0 : -1.0) * 0.5 * h[d] * s;
        }
        g.wq[q] = g.V / nq;
      }
      return;
    }
    g.V = cV[e];
    g.c[0] = cc[2 * e];
    g.c[1] = cc[2 * e + 1];
    g.M[0][0] = cM[3 * e];
    g.M[0][1] = g.M[1][0] = cM[3 * e + 1];
    g.M[1][1] = cM[3 * e + 2];
    // Principal-axis rule: M = sum_k lam_k e_k e_k^T, points c -+
    // sqrt(2 lam_k / V) e_k, weights V/4.  It reproduces the volume, the zero
    // first moments and M, so it integrates every quadratic exactly.
    double a = g.M[0][0], b = g.M[0][1], d = g.M[1][1];
    double tr = 0.5 * (a + d);
    double disc = std::sqrt(0.25 * (a - d) * (a - d) + b * b);
    double lam[2] = {tr + disc, tr - disc};
    double ev[2][2];
    if (b == 0.0) {
      if (a >= d) {
        ev[0][0] = 1; ev[0][1] = 0; ev[1][0] = 0; ev[1][1] = 1;
      } else {
        ev[0][0] = 0; ev[0][1] = 1; ev[1][0] = 1; ev[1][1] = 0;
      }
    } else {
      for (int k = 0; k < 2; ++k) {
        double vx = b, vy = lam[k] - a;
        double nn = std::sqrt(vx * vx + vy * vy);
        ev[k][0] = vx / nn;
        ev[k][1] = vy / nn;
      }
    }
    g.nq = 4;
    int q = 0;
    for (int k = 0; k < 2; ++k) {
      double r = std::sqrt(2.0 * lam[k] / g.V);
      for (int s = -1; s <= 1; s += 2) {
        g.rq[q][0] = s * r * ev[k][0];
        g.rq[q][1] = s * r * ev[k][1];
        g.rq[q][2] = 0.0;
        g.wq[q] = 0.25 * g.V;
        ++q;
      }
    }
  }
};

// --------------------------------------------------------------- physics --
// Conserved variables (Sec. 2.1): rho, rho v (dim components for Euler, 3 for
// MHD), total energy rho e, and for MHD B (3 components).  Units with mu0 = 1:
// p_total = p_gas + B^2/2, E = p_gas/(gamma-1) + rho v^2/2 + B^2/2.
struct Phys {
  int dim;      // spatial dimension of the mesh
  int mhd;      // 0 Euler, 1 ideal MHD (2D or 3D; velocity and B have 3 components)
  double gamma;
  int riemann = 0;  // Euler face flux: 0 HLL (Davis speeds), 1 exact Riemann solver
  int nv() const { return mhd ? 8 : dim + 2; }
  int nvel() const { return mhd ? 3 : dim; }
  int nhyd() const { return mhd ? 5 : dim + 2; }  // Taylor-basis variables
  // non-constant B basis functions: V4..V11 in 3D; in 2D V3..V5 for (B_x, B_y)
  // plus the two Taylor functions x, y of B_z
  int nfun() const { return dim == 3 ? 8 : 5; }
  int ncoef() const { return mhd ? 5 * (1 + dim) + 3 + nfun() : (dim + 2) * (1 + dim); }
};

// The locally divergence-free magnetic basis of Sec. 2.2 (3D), functions
// V4..V11 written as linear maps: V_j,c(r) = sum_d LB[j][c][d] r_d.
//   V4=(y,0,0) V5=(z,0,0) V6=(0,x,0) V7=(0,z,0) V8=(0,0,x) V9=(0,0,y)
//   V10=(x,-y,0) V11=(x,0,-z)
double LB[8][3][3];
struct LBInit {
  LBInit() {
    std::memset(LB, 0, sizeof(LB));
    LB[0][0][1] = 1;                    // V4
    LB[1][0][2] = 1;                    // V5
    LB[2][1][0] = 1;                    // V6
    LB[3][1][2] = 1;                    // V7
    LB[4][2][0] = 1;                    // V8
    LB[5][2][1] = 1;                    // V9
    LB[6][0][0] = 1; LB[6][1][1] = -1;  // V10
    LB[7][0][0] = 1; LB[7][2][2] = -1;  // V11
  }
} lbinit;

// The 2D magnetic basis (Sec. 2.2): V3 = (y, 0), V4 = (0, x), V5 = (x, -y) for
// (B_x, B_y), with coefficients alpha_1 = dB_x/dy, alpha_2 = dB_y/dx,
// alpha_3 = dB_x/dx = -dB_y/dy, and B_z in the Taylor basis (x, y).
double LB2[8][3][3];
struct LB2Init {
  LB2Init() {
    std::memset(LB2, 0, sizeof(LB2));
    LB2[0][0][1] = 1;                     // V3: B_x = y
    LB2[1][1][0] = 1;                     // V4: B_y = x
    LB2[2][0][0] = 1; LB2[2][1][1] = -1;  // V5: B_x = x, B_y = -y
    LB2[3][2][0] = 1;                     // B_z = x
    LB2[4][2][1] = 1;                     // B_z = y
  }
} lb2init;

// The B basis table of the mesh dimension.
inline const double (*basis(const Phys& P))[3][3] { return P.dim == 3 ? LB : LB2; }

template <class T> struct State {
  T u[8];
};

// Gas pressure of a conserved state.
template <class T> T pressure(const Phys& P, const T* u) {
  int nvel = P.nvel();
  T rho = u[0];
  T ke = T(0);
  for (int d = 0; d < nvel; ++d) ke += u[1 + d] * u[1 + d];
  ke = T(0.5) * ke / rho;
  T E = u[1 + nvel];
  T pm = T(0);
  if (P.mhd)
    for (int c = 0; c < 3; ++c) pm += u[5 + c] * u[5 + c];
  return T(P.gamma - 1.0) * (E - ke - T(0.5) * pm);
}

// Physical flux F(U) . n (Sec. 2.1, eqn:cons).  n is a unit vector.
template <class T> void flux_n(const Phys& P, const T* u, const double* n, T* F) {
  int nvel = P.nvel();
  T rho = u[0];
  T v[3] = {T(0), T(0), T(0)};
  for (int d = 0; d < nvel; ++d) v[d] = u[1 + d] / rho;
  T p = pressure(P, u);
  T E = u[1 + nvel];
  T vn = T(0);
  for (int d = 0; d < nvel; ++d) vn += v[d] * T(n[d]);
  if (!P.mhd) {
    F[0] = rho * vn;
    for (int d = 0; d < nvel; ++d) F[1 + d] = rho * v[d] * vn + p * T(n[d]);
    F[1 + nvel] = (E + p) * vn;
    return;
  }
  const T* B = u + 5;
  T Bn = B[0] * T(n[0]) + B[1] * T(n[1]) + B[2] * T(n[2]);
  T B2 = B[0] * B[0] + B[1] * B[1] + B[2] * B[2];
  T pT = p + T(0.5) * B2;
  T vB = v[0] * B[0] + v[1] * B[1] + v[2] * B[2];
  F[0] = rho * vn;
  for (int d = 0; d < 3; ++d) F[1 + d] = rho * v[d] * vn + pT * T(n[d]) - B[d] * Bn;
  F[4] = (E + pT) * vn - Bn * vB;
  for (int d = 0; d < 3; ++d) F[5 + d] = B[d] * vn - v[d] * Bn;
}

// Sound speed (Euler) or fast magnetosonic speed along n (MHD).
template <class T> T signal_speed(const Phys& P, const T* u, const double* n) {
  T rho = u[0];
  T p = pressure(P, u);
  T a2 = T(P.gamma) * p / rho;
  if (!P.mhd) return dsqrt(a2);
  const T* B = u + 5;
  T Bn = B[0] * T(n[0]) + B[1] * T(n[1]) + B[2] * T(n[2]);
  T B2 = B[0] * B[0] + B[1] * B[1] + B[2] * B[2];
  T s = a2 + B2 / rho;
  T disc = s * s - T(4.0) * a2 * Bn * Bn / rho;
  if (disc < T(0)) disc = T(0);
  return dsqrt(T(0.5) * (s + dsqrt(disc)));
}

// HLL flux with Davis wave-speed estimates (the build's Euler Riemann solver;
// the Riemann problem is posed along the face normal, Sec. 2.3).
// code (optional): the branch taken, for finite-difference checks: 0 left of
// the fan (F_L), 2 right of it (F_R); inside, 1 | 4 (S_L from the right
// state) | 8 (S_R from the right state).
template <class T>
void hll(const Phys& P, const T* uL, const T* uR, const double* n, T* F, int* code = nullptr) {
  int nv = P.nv(), nvel = P.nvel();
  T FL[8], FR[8];
  flux_n(P, uL, n, FL);
  flux_n(P, uR, n, FR);
  T vnL = T(0), vnR = T(0);
  for (int d = 0; d < nvel; ++d) {
    vnL += uL[1 + d] / uL[0] * T(n[d]);
    vnR += uR[1 + d] / uR[0] * T(n[d]);
  }
  T cL = signal_speed(P, uL, n), cR = signal_speed(P, uR, n);
  T SL = dmin(vnL - cL, vnR - cR);
  T SR = dmax(vnL + cL, vnR + cR);
  if (code)
    *code = SL >= T(0) ? 0 : SR <= T(0) ? 2
          : 1 | ((vnR - cR) < (vnL - cL) ? 4 : 0) | ((vnR + cR) > (vnL + cL) ? 8 : 0);
  if (SL >= T(0)) {
    for (int k = 0; k < nv; ++k) F[k] = FL[k];
  } else if (SR <= T(0)) {
    for (int k = 0; k < nv; ++k) F[k] = FR[k];
  } else {
    for (int k = 0; k < nv; ++k)
      F[k] = (SR * FL[k] - SL * FR[k] + SL * SR * (uR[k] - uL[k])) / (SR - SL);
  }
}

// HLLD flux of Miyoshi & Kusano (2005) for ideal MHD, the solver the paper
// names (Sec. 2.3).  Written in vector form: normal components along n,
// transverse components as 3-vectors orthogonal to n.  Both input states must
// already carry the same normal field Bn (the face average of Sec. 2.6).
template <class T>
void hlld(const Phys& P, const T* uL, const T* uR, const double* n, T* F) {
  struct Side {
    T rho, vn, vt[3], Bt[3], p, pT, E, vB, u[8], F[8], cf;
  } s[2];
  T Bn = uL[5] * T(n[0]) + uL[6] * T(n[1]) + uL[7] * T(n[2]);
  for (int a = 0; a < 2; ++a) {
    const T* u = a == 0 ? uL : uR;
    Side& S = s[a];
    for (int k = 0; k < 8; ++k) S.u[k] = u[k];
    S.rho = u[0];
    T v[3] = {u[1] / u[0], u[2] / u[0], u[3] / u[0]};
    S.vn = v[0] * T(n[0]) + v[1] * T(n[1]) + v[2] * T(n[2]);
    T bn = u[5] * T(n[0]) + u[6] * T(n[1]) + u[7] * T(n[2]);
    for (int d = 0; d < 3; ++d) {
      S.vt[d] = v[d] - S.vn * T(n[d]);
      S.Bt[d] = u[5 + d] - bn * T(n[d]);
    }
    S.p = pressure(P, u);
    T B2 = u[5] * u[5] + u[6] * u[6] + u[7] * u[7];
    S.pT = S.p + T(0.5) * B2;
    S.E = u[4];
    S.vB = v[0] * u[5] + v[1] * u[6] + v[2] * u[7];
    flux_n(P, u, n, S.F);
    S.cf = signal_speed(P, u, n);
  }
  Side& L = s[0];
  Side& R = s[1];
  // Outer wave speeds.
  T cmax = dmax(L.cf, R.cf);
  T SL = dmin(L.vn, R.vn) - cmax;
  T SR = dmax(L.vn, R.vn) + cmax;
  if (SL >= T(0)) {
    for (int k = 0; k < 8; ++k) F[k] = L.F[k];
    return;
  }
  if (SR <= T(0)) {
    for (int k = 0; k < 8; ++k) F[k] = R.F[k];
    return;
  }
  // Contact speed and star total pressure.
  T dL = (SL - L.vn) * L.rho, dR = (SR - R.vn) * R.rho;
  T SM = (dR * R.vn - dL * L.vn - R.pT + L.pT) / (dR - dL);
  T pTs = (dR * L.pT - dL * R.pT + dL * dR * (R.vn - L.vn)) / (dR - dL);
  // Single-star states.
  struct Star {
    T rho, vt[3], Bt[3], E, u[8], F[8], sq;
  } st[2];
  T Sa[2] = {SL, SR};
  for (int a = 0; a < 2; ++a) {
    Side& S = s[a];
    Star& Z = st[a];
    T Sm = Sa[a] - S.vn;
    Z.rho = S.rho * Sm / (Sa[a] - SM);
    T den = S.rho * Sm * (Sa[a] - SM) - Bn * Bn;
    T scale = S.rho * Sm * Sm + Bn * Bn;
    bool degenerate = dabs(den) <= T(1e-12) * scale;
    for (int d = 0; d < 3; ++d) {
      if (degenerate) {
        Z.vt[d] = S.vt[d];
        Z.Bt[d] = S.Bt[d];
      } else {
        Z.vt[d] = S.vt[d] - Bn * S.Bt[d] * (SM - S.vn) / den;
        Z.Bt[d] = S.Bt[d] * (S.rho * Sm * Sm - Bn * Bn) / den;
      }
    }
    T vBs = SM * Bn;
    for (int d = 0; d < 3; ++d) vBs += Z.vt[d] * Z.Bt[d];
    Z.E = (Sm * S.E - S.pT * S.vn + pTs * SM + Bn * (S.vB - vBs)) / (Sa[a] - SM);
    Z.u[0] = Z.rho;
    for (int d = 0; d < 3; ++d) {
      Z.u[1 + d] = Z.rho * (SM * T(n[d]) + Z.vt[d]);
      Z.u[5 + d] = Bn * T(n[d]) + Z.Bt[d];
    }
    Z.u[4] = Z.E;
    for (int k = 0; k < 8; ++k) Z.F[k] = S.F[k] + Sa[a] * (Z.u[k] - S.u[k]);
    Z.sq = dsqrt(Z.rho);
  }
  T absBn = dabs(Bn);
  T SsL = SM - absBn / st[0].sq;
  T SsR = SM + absBn / st[1].sq;
  if (SsL >= T(0)) {
    for (int k = 0; k < 8; ++k) F[k] = st[0].F[k];
    return;
  }
  if (SsR <= T(0)) {
    for (int k = 0; k < 8; ++k) F[k] = st[1].F[k];
    return;
  }
  // Double-star states (rotational discontinuities).
  T sgn = Bn < T(0) ? T(-1) : T(1);
  T sL = st[0].sq, sR = st[1].sq;
  T inv = T(1) / (sL + sR);
  T vss[3], Bss[3];
  for (int d = 0; d < 3; ++d) {
    vss[d] = (sL * st[0].vt[d] + sR * st[1].vt[d] + (st[1].Bt[d] - st[0].Bt[d]) * sgn) * inv;
    Bss[d] = (sL * st[1].Bt[d] + sR * st[0].Bt[d] + sL * sR * (st[1].vt[d] - st[0].vt[d]) * sgn) * inv;
  }
  T vBss = SM * Bn;
  for (int d = 0; d < 3; ++d) vBss += vss[d] * Bss[d];
  int a = (SM >= T(0)) ? 0 : 1;
  Star& Z = st[a];
  T vBs = SM * Bn;
  for (int d = 0; d < 3; ++d) vBs += Z.vt[d] * Z.Bt[d];
  T Ess = a == 0 ? Z.E - sL * (vBs - vBss) * sgn : Z.E + sR * (vBs - vBss) * sgn;
  T uss[8];
  uss[0] = Z.rho;
  for (int d = 0; d < 3; ++d) {
    uss[1 + d] = Z.rho * (SM * T(n[d]) + vss[d]);
    uss[5 + d] = Bn * T(n[d]) + Bss[d];
  }
  uss[4] = Ess;
  T Ss = a == 0 ? SsL : SsR;
  for (int k = 0; k < 8; ++k) F[k] = Z.F[k] + Ss * (uss[k] - Z.u[k]);
}

// Exact Riemann solver for the Euler equations, the Euler flux the paper uses
// (Sec. 2.3), posed along the face normal n.  In the face frame the two outer
// waves are each a shock or a rarefaction; across a wave on side K the
// velocity changes by f_K(p), with f_K from the Rankine-Hugoniot conditions
// when p > p_K and from the isentropic relation with the Riemann invariant
// u +- 2c/(gamma-1) when p <= p_K.  The star pressure p* solves
// f_L(p) + f_R(p) + u_R - u_L = 0 (Newton's method started from the value
// that is exact when both waves are rarefactions); u* = (u_L + u_R)/2 +
// (f_R(p*) - f_L(p*))/2.  The state on the face (x/t = 0) follows from the
// position of the waves, and the tangential velocity is the one upwind of the
// contact.  F is the physical flux of that state.  Returns false on vacuum
// generation (u_R - u_L >= 2 (c_L + c_R)/(gamma - 1)).
template <class T> void wave_relation(T p, T rK, T pK, T cK, double g, T& f, T& df) {
  if (p > pK) {
    T A = T(2.0 / (g + 1.0)) / rK;
    T B = T((g - 1.0) / (g + 1.0)) * pK;
    T s = dsqrt(A / (p + B));
    f = (p - pK) * s;
    df = s * (T(1) - (p - pK) / (T(2) * (p + B)));
  } else {
    T r = dpow(p / pK, (g - 1.0) / (2.0 * g));
    f = T(2.0 / (g - 1.0)) * cK * (r - T(1));
    df = r * pK / (p * rK * cK);
  }
}

template <class T>
bool exact_riemann(const Phys& P, const T* uL, const T* uR, const double* n, T* F,
                   T* star = nullptr, T* face_state = nullptr) {
  const int nvel = P.nvel();
  const double g = P.gamma;
  T r[2], un[2], vt[2][3], p[2], c[2];
  for (int a = 0; a < 2; ++a) {
    const T* u = a == 0 ? uL : uR;
    r[a] = u[0];
    un[a] = T(0);
    for (int d = 0; d < nvel; ++d) un[a] += u[1 + d] / u[0] * T(n[d]);
    for (int d = 0; d < 3; ++d) vt[a][d] = d < nvel ? u[1 + d] / u[0] - un[a] * T(n[d]) : T(0);
    p[a] = pressure(P, u);
    c[a] = dsqrt(T(g) * p[a] / r[a]);
  }
  const T du = un[1] - un[0];
  if (!(T(2.0 / (g - 1.0)) * (c[0] + c[1]) > du)) return false;
  const double z = (g - 1.0) / (2.0 * g);
  T ps = dpow((c[0] + c[1] - T(0.5 * (g - 1.0)) * du) /
                  (c[0] / dpow(p[0], z) + c[1] / dpow(p[1], z)),
              1.0 / z);
  T fL, dfL, fR, dfR;
  for (int it = 0; it < 100; ++it) {
    wave_relation(ps, r[0], p[0], c[0], g, fL, dfL);
    wave_relation(ps, r[1], p[1], c[1], g, fR, dfR);
    T pn = ps - (fL + fR + du) / (dfL + dfR);
    if (!(pn > T(0))) pn = T(0.5) * ps;
    const bool done = dabs(pn - ps) <= T(1e-15) * (pn + ps);
    ps = pn;
    if (done) break;
  }
  wave_relation(ps, r[0], p[0], c[0], g, fL, dfL);
  wave_relation(ps, r[1], p[1], c[1], g, fR, dfR);
  const T us = T(0.5) * (un[0] + un[1]) + T(0.5) * (fR - fL);
  if (star) {
    star[0] = ps;
    star[1] = us;
  }
  // sample the self-similar solution on the face, x/t = 0
  const double G1 = (g + 1.0) / (2.0 * g), G2 = (g - 1.0) / (2.0 * g), G6 = (g - 1.0) / (g + 1.0);
  const int a = us >= T(0) ? 0 : 1;    // side of the contact the face is on
  const T sg = a == 0 ? T(1) : T(-1);  // mirror the right side onto the left
  const T ua = sg * un[a], ra = r[a], pa = p[a], ca = c[a], usa = sg * us;
  T rho, u, pr;
  if (ps > pa) {
    const T S = ua - ca * dsqrt(T(G1) * ps / pa + T(G2));  // shock speed
    if (S >= T(0)) {
      rho = ra; u = ua; pr = pa;
    } else {
      rho = ra * (ps / pa + T(G6)) / (T(G6) * ps / pa + T(1)); u = usa; pr = ps;
    }
  } else {
    const T head = ua - ca;
    const T tail = usa - ca * dpow(ps / pa, z);
    if (head >= T(0)) {
      rho = ra; u = ua; pr = pa;
    } else if (tail < T(0)) {
      rho = ra * dpow(ps / pa, 1.0 / g); u = usa; pr = ps;
    } else {  // inside the rarefaction fan: u = c there
      const T cf = T(2.0 / (g + 1.0)) * (ca + T(0.5 * (g - 1.0)) * ua);
      u = cf;
      rho = ra * dpow(cf / ca, 2.0 / (g - 1.0));
      pr = pa * dpow(cf / ca, 2.0 * g / (g - 1.0));
    }
  }
  u = sg * u;
  if (face_state) {
    face_state[0] = rho;
    face_state[1] = u;
    face_state[2] = pr;
  }
  T v[3], v2 = u * u;
  for (int d = 0; d < 3; ++d) {
    v[d] = u * T(n[d]) + vt[a][d];
    v2 += vt[a][d] * vt[a][d];
  }
  const T E = pr / T(g - 1.0) + T(0.5) * rho * v2;
  F[0] = rho * u;
  for (int d = 0; d < nvel; ++d) F[1 + d] = rho * v[d] * u + pr * T(n[d]);
  F[1 + nvel] = (E + pr) * u;
  return true;
}

// ------------------------------------------------------ cell polynomials --
// Coefficient-major layout of the state: U[k * ncells + cell].
// Hydro variable v has coefficients k = v*(1+dim) + c, c = 0 the mean and
// c = 1..dim the gradient along x, y, z.  MHD appends the B means (3 arrays)
// and the coefficients a4..a11 of V4..V11 (8 arrays).
template <class T> struct Poly {
  T m[8];        // means (all conserved variables, B included)
  T g[5][3];     // gradients of the Taylor-basis variables
  T a[8];        // a4..a11 (MHD)
};

template <class T>
void load_poly(const Phys& P, const T* U, int64_t nc, int64_t e, Poly<T>& q) {
  int dim = P.dim, nh = P.nhyd();
  for (int v = 0; v < nh; ++v) {
    q.m[v] = U[(int64_t)(v * (1 + dim)) * nc + e];
    for (int d = 0; d < 3; ++d)
      q.g[v][d] = d < dim ? U[(int64_t)(v * (1 + dim) + 1 + d) * nc + e] : T(0);
  }
  if (P.mhd) {
    int base = nh * (1 + dim);
    for (int c = 0; c < 3; ++c) q.m[5 + c] = U[(int64_t)(base + c) * nc + e];
    for (int j = 0; j < P.nfun(); ++j) q.a[j] = U[(int64_t)(base + 3 + j) * nc + e];
  }
}

template <class T>
void store_poly(const Phys& P, T* U, int64_t nc, int64_t e, const Poly<T>& q) {
  int dim = P.dim, nh = P.nhyd();
  for (int v = 0; v < nh; ++v) {
    U[(int64_t)(v * (1 + dim)) * nc + e] = q.m[v];
    for (int d = 0; d < dim; ++d) U[(int64_t)(v * (1 + dim) + 1 + d) * nc + e] = q.g[v][d];
  }
  if (P.mhd) {
    int base = nh * (1 + dim);
    for (int c = 0; c < 3; ++c) U[(int64_t)(base + c) * nc + e] = q.m[5 + c];
    for (int j = 0; j < P.nfun(); ++j) U[(int64_t)(base + 3 + j) * nc + e] = q.a[j];
  }
}

// Gradient of B component c (from the divergence-free coefficients).
template <class T> void grad_B(const Phys& P, const Poly<T>& q, int c, T* gB) {
  const auto LBp = basis(P);
  for (int d = 0; d < 3; ++d) {
    T s = T(0);
    for (int j = 0; j < P.nfun(); ++j)
      if (LBp[j][c][d] != 0.0) s += T(LBp[j][c][d]) * q.a[j];
    gB[d] = s;
  }
}

// Evaluate the cell polynomial at offset r from the centroid (Sec. 2.2: the
// Taylor expansion about the centroid; B from the divergence-free basis).
template <class T> void eval_poly(const Phys& P, const Poly<T>& q, const double* r, T* u) {
  int dim = P.dim, nh = P.nhyd();
  for (int v = 0; v < nh; ++v) {
    T s = q.m[v];
    for (int d = 0; d < dim; ++d) s += q.g[v][d] * T(r[d]);
    u[v] = s;
  }
  if (P.mhd) {
    const auto LBp = basis(P);
    for (int c = 0; c < 3; ++c) {
      T s = q.m[5 + c];
      for (int j = 0; j < P.nfun(); ++j)
        for (int d = 0; d < 3; ++d)
          if (LBp[j][c][d] != 0.0) s += q.a[j] * T(LBp[j][c][d] * r[d]);
      u[5 + c] = s;
    }
  }
}

template <class T> bool physical(const Phys& P, const T* u) {
  for (int k = 0; k < P.nv(); ++k)
    if (!finite(u[k])) return false;
  if (!(u[0] > T(0))) return false;
  T p = pressure(P, u);
  return finite(p) && p > T(0);
}

// ------------------------------------------------ MUSCL-Hancock prediction --
// Sec. 2.4: the cell's conserved mean and gradients are turned into primitive
// values (rho, v, p) and primitive gradients at the centroid (chain rule, as
// in the paper's example for d(v_x)/dy); the primitive state is advanced half
// a step with its time derivative from the quasi-linear Euler equations,
//   rho_t = -(v . grad rho + rho div v)
//   v_t   = -(v . grad) v - grad p / rho
//   p_t   = -(gamma p div v + v . grad p),
// evaluated with the centroid values and gradients, and extrapolated
// linearly to the point r (a face Gauss point or a volume point), then turned
// back into conserved variables for the Riemann solver and the volume flux.
// Euler only.
template <class T> struct Prim {
  T w[5];        // rho, v (dim components), p at the centroid, advanced by half_dt
  T gw[5][3];    // primitive gradients
};

template <class T> void predict_prim(const Phys& P, const Poly<T>& q, double half_dt, Prim<T>& out) {
  const int dim = P.dim;
  const T rho = q.m[0];
  T v[3] = {T(0), T(0), T(0)};
  for (int d = 0; d < dim; ++d) v[d] = q.m[1 + d] / rho;
  T v2 = T(0);
  for (int d = 0; d < dim; ++d) v2 += v[d] * v[d];
  const T E = q.m[1 + dim];
  const T gm1 = T(P.gamma - 1.0);
  const T p = gm1 * (E - T(0.5) * rho * v2);
  // primitive gradients at the centroid
  T grho[3], gv[3][3], gp[3];
  for (int d = 0; d < dim; ++d) {
    grho[d] = q.g[0][d];
    for (int i = 0; i < dim; ++i) gv[i][d] = (q.g[1 + i][d] - v[i] * grho[d]) / rho;
    // E = p/(gamma-1) + rho |v|^2 / 2
    T s = q.g[1 + dim][d] - T(0.5) * v2 * grho[d];
    for (int i = 0; i < dim; ++i) s -= rho * v[i] * gv[i][d];
    gp[d] = gm1 * s;
  }
  T div = T(0);
  for (int d = 0; d < dim; ++d) div += gv[d][d];
  T vgrho = T(0), vgp = T(0);
  for (int d = 0; d < dim; ++d) {
    vgrho += v[d] * grho[d];
    vgp += v[d] * gp[d];
  }
  const T rho_t = -(vgrho + rho * div);
  const T p_t = -(T(P.gamma) * p * div + vgp);
  const T h = T(half_dt);
  out.w[0] = rho + h * rho_t;
  for (int i = 0; i < dim; ++i) {
    T adv = T(0);
    for (int d = 0; d < dim; ++d) adv += v[d] * gv[i][d];
    const T vt = -(adv + gp[i] / rho);
    out.w[1 + i] = v[i] + h * vt;
  }
  out.w[1 + dim] = p + h * p_t;
  for (int d = 0; d < dim; ++d) {
    out.gw[0][d] = grho[d];
    for (int i = 0; i < dim; ++i) out.gw[1 + i][d] = gv[i][d];
    out.gw[1 + dim][d] = gp[d];
  }
}

// Conserved state of the predicted primitive polynomial at offset r.
template <class T> void eval_prim(const Phys& P, const Prim<T>& pr, const double* r, T* u) {
  const int dim = P.dim;
  T w[5];
  for (int k = 0; k < dim + 2; ++k) {
    T s = pr.w[k];
    for (int d = 0; d < dim; ++d) s += pr.gw[k][d] * T(r[d]);
    w[k] = s;
  }
  T v2 = T(0);
  u[0] = w[0];
  for (int d = 0; d < dim; ++d) {
    u[1 + d] = w[0] * w[1 + d];
    v2 += w[1 + d] * w[1 + d];
  }
  u[1 + dim] = w[1 + dim] / T(P.gamma - 1.0) + T(0.5) * w[0] * v2;
}

// Solve the small symmetric system A x = b (Gaussian elimination with
// partial pivoting), n <= 8.
template <class T> void solve_small(int n, const double* Ain, const T* b, T* x) {
  double A[8][8];
  T y[8];
  int perm[8];
  for (int i = 0; i < n; ++i) {
    perm[i] = i;
    for (int j = 0; j < n; ++j) A[i][j] = Ain[i * n + j];
    y[i] = b[i];
  }
  for (int k = 0; k < n; ++k) {
    int piv = k;
    for (int i = k + 1; i < n; ++i)
      if (std::fabs(A[i][k]) > std::fabs(A[piv][k])) piv = i;
    if (piv != k) {
      for (int j = 0; j < n; ++j) std::swap(A[k][j], A[piv][j]);
      std::swap(y[k], y[piv]);
    }
    for (int i = k + 1; i < n; ++i) {
      double f = A[i][k] / A[k][k];
      for (int j = k; j < n; ++j) A[i][j] -= f * A[k][j];
      y[i] = y[i] - T(f) * y[k];
    }
  }
  for (int i = n - 1; i >= 0; --i) {
    T s = y[i];
    for (int j = i + 1; j < n; ++j) s = s - T(A[i][j]) * x[j];
    x[i] = s / T(A[i][i]);
  }
  (void)perm;
}

// Gram matrix of the B basis, G_ij = int V_i . V_j dOmega, from the cell's
// second-moment matrix M (Sec. 2.2: the mass matrix M_B, 8x8 in 3D; in 2D the
// printed 3x3 matrix of alpha_1..alpha_3 plus the B_z block M).
void gram_B(const Phys& P, const double M[3][3], double* G) {
  const auto LBp = basis(P);
  const int nf = P.nfun();
  for (int i = 0; i < nf; ++i)
    for (int j = 0; j < nf; ++j) {
      double s = 0;
      for (int c = 0; c < 3; ++c)
        for (int d = 0; d < 3; ++d)
          for (int e = 0; e < 3; ++e) s += LBp[i][c][d] * LBp[j][c][e] * M[d][e];
      G[i * nf + j] = s;
    }
}

// ------------------------------------------------------------- operators --
struct Ctx {
  const Mesh* mesh;
  Phys P;
  int limiter;
  // Optional record of the branches a step takes (2D Euler on boxes, for
  // finite-difference checks): per stage, per cell kBranchCodes ints: the
  // limiter of the 4 variables, then HLL at the 2 Gauss points of the 4 faces.
  int* br = nullptr;
  int br_stage = 0;
};
constexpr int kBranchCodes = 12;

// Semi-discrete right-hand side L(U) for one cell (Sec. 2.2): surface terms
// over the cell's faces (Gauss points in order), then the volume term, then
// the inverse mass matrices.  Returns false on a non-physical state.
// half_dt < 0: the semi-discrete operator L(U) of the cell polynomials.
// half_dt >= 0: the MUSCL-Hancock operator, the same surface and volume terms
// with every state taken from the half-step primitive prediction (Sec. 2.4).
template <class T>
bool rhs_cell(const Ctx& C, const T* U, T* dUdt, int64_t e, double half_dt = -1.0) {
  const Mesh& M = *C.mesh;
  const Phys& P = C.P;
  const int dim = P.dim, nv = P.nv(), nh = P.nhyd();
  const int64_t nc = M.nc;
  CellGeo cg;
  M.cell(e, cg);
  Poly<T> qe;
  load_poly(P, U, nc, e, qe);

  T rmean[8], rgrad[5][3], ra[8];
  for (int k = 0; k < 8; ++k) rmean[k] = T(0), ra[k] = T(0);
  for (int v = 0; v < 5; ++v)
    for (int d = 0; d < 3; ++d) rgrad[v][d] = T(0);
  bool ok = true;

  int64_t fids[64];
  int sides[64];
  int nfc = M.cell_faces(e, fids, sides);
  for (int m = 0; m < nfc; ++m) {
    FaceGeo fg;
    M.face(fids[m], fg);
    Poly<T> qL, qR;
    load_poly(P, U, nc, fg.L, qL);
    load_poly(P, U, nc, fg.R, qR);
    Prim<T> pL, pR;
    if (half_dt >= 0) {
      predict_prim(P, qL, half_dt, pL);
      predict_prim(P, qR, half_dt, pR);
    }
    for (int p = 0; p < fg.ng; ++p) {
      double rL[3], rR[3];
      for (int d = 0; d < 3; ++d) {
        rL[d] = fg.rg[p][d];
        rR[d] = fg.rg[p][d] - fg.dLR[d];
        if (d >= dim) rL[d] = rR[d] = 0.0;
      }
      T uL[8], uR[8], F[8];
      if (half_dt >= 0) {
        eval_prim(P, pL, rL, uL);
        eval_prim(P, pR, rR, uR);
      } else {
        eval_poly(P, qL, rL, uL);
        eval_poly(P, qR, rR, uR);
      }
      if (P.mhd) {
        // One normal field for the Riemann problem: the average of the two
        // extrapolated normal components (Sec. 2.6).
        T bnL = uL[5] * T(fg.n[0]) + uL[6] * T(fg.n[1]) + uL[7] * T(fg.n[2]);
        T bnR = uR[5] * T(fg.n[0]) + uR[6] * T(fg.n[1]) + uR[7] * T(fg.n[2]);
        T bn = T(0.5) * (bnL + bnR);
        for (int d = 0; d < 3; ++d) {
          uL[5 + d] += (bn - bnL) * T(fg.n[d]);
          uR[5 + d] += (bn - bnR) * T(fg.n[d]);
        }
      }
      if (!physical(P, uL) || !physical(P, uR)) ok = false;
      if (P.mhd)
        hlld(P, uL, uR, fg.n, F);
      else if (P.riemann == 1) {
        if (!exact_riemann(P, uL, uR, fg.n, F)) ok = false;
      } else {
        int* code = nullptr;
        if (C.br && m * fg.ng + p < kBranchCodes - 4)
          code = C.br + ((int64_t)C.br_stage * nc + e) * kBranchCodes + 4 + m * fg.ng + p;
        hll(P, uL, uR, fg.n, F, code);
      }
      const double* r = sides[m] == 0 ? rL : rR;
      T sg = sides[m] == 0 ? T(-fg.wg[p]) : T(fg.wg[p]);
      for (int k = 0; k < nv; ++k) rmean[k] += sg * F[k];
      for (int v = 0; v < nh; ++v)
        for (int d = 0; d < dim; ++d) rgrad[v][d] += sg * F[v] * T(r[d]);
      if (P.mhd) {
        const auto LBp = basis(P);
        for (int j = 0; j < P.nfun(); ++j) {
          T s = T(0);
          for (int c = 0; c < 3; ++c) {
            double vj = 0;
            for (int d = 0; d < 3; ++d) vj += LBp[j][c][d] * r[d];
            if (vj != 0.0) s += F[5 + c] * T(vj);
          }
          ra[j] += sg * s;
        }
      }
    }
  }
  // Volume term: int F . grad(test) dOmega, with grad(x_d) = e_d for the
  // Taylor basis and the constant derivatives of V4..V11 for B.
  Prim<T> pe;
  if (half_dt >= 0) predict_prim(P, qe, half_dt, pe);
  for (int q = 0; q < cg.nq; ++q) {
    T u[8];
    if (half_dt >= 0)
      eval_prim(P, pe, cg.rq[q], u);
    else
      eval_poly(P, qe, cg.rq[q], u);
    if (!physical(P, u)) ok = false;
    T Fd[3][8];
    for (int d = 0; d < dim; ++d) {
      double nd[3] = {0, 0, 0};
      nd[d] = 1.0;
      flux_n(P, u, nd, Fd[d]);
    }
    T w = T(cg.wq[q]);
    for (int v = 0; v < nh; ++v)
      for (int d = 0; d < dim; ++d) rgrad[v][d] += w * Fd[d][v];
    if (P.mhd) {
      const auto LBp = basis(P);
      for (int j = 0; j < P.nfun(); ++j) {
        T s = T(0);
        for (int c = 0; c < 3; ++c)
          for (int d = 0; d < dim; ++d)
            if (LBp[j][c][d] != 0.0) s += T(LBp[j][c][d]) * Fd[d][5 + c];
        ra[j] += w * s;
      }
    }
  }
  // Inverse mass matrices: means divide by V; gradients solve M g = res
  // (Sec. 2.2, "Derivative information is obtained by matrix inversion").
  Poly<T> out;
  for (int k = 0; k < 8; ++k) out.m[k] = rmean[k] / T(cg.V);
  double Mflat[9];
  for (int i = 0; i < dim; ++i)
    for (int j = 0; j < dim; ++j) Mflat[i * dim + j] = cg.M[i][j];
  for (int v = 0; v < nh; ++v) {
    T x[3];
    solve_small(dim, Mflat, rgrad[v], x);
    for (int d = 0; d < 3; ++d) out.g[v][d] = d < dim ? x[d] : T(0);
  }
  if (P.mhd) {
    double G[64];
    gram_B(P, cg.M, G);
    solve_small(P.nfun(), G, ra, out.a);
  }
  store_poly(P, dUdt, nc, e, out);
  return ok;
}

// Arepo slope limiter on one cell (Sec. 2.5): alpha = min(1, min_j psi_ij)
// with psi from the max/min of the means over the cell and its face
// neighbours and the linear extrapolation to each face centroid.  Applied to
// the conserved Taylor variables; the three B components share one alpha.
template <class T>
void limit_cell(const Ctx& C, const T* U, T* Ul, int64_t e) {
  const Mesh& M = *C.mesh;
  const Phys& P = C.P;
  const int dim = P.dim, nh = P.nhyd();
  const int64_t nc = M.nc;
  Poly<T> q;
  load_poly(P, U, nc, e, q);
  CellGeo cg;
  M.cell(e, cg);
  int64_t fids[64];
  int sides[64];
  int nfc = M.cell_faces(e, fids, sides);
  // Neighbour means and face-centroid offsets from this cell's centroid.
  int nvar = P.mhd ? 8 : nh;
  T phimax[8], phimin[8];
  int amax[8] = {0}, amin[8] = {0};  // arg-extremal: 0 the cell, m + 1 face m's neighbour
  for (int k = 0; k < nvar; ++k) phimax[k] = phimin[k] = q.m[k];
  double rf[64][3];
  for (int m = 0; m < nfc; ++m) {
    FaceGeo fg;
    M.face(fids[m], fg);
    int64_t nb = sides[m] == 0 ? fg.R : fg.L;
    Poly<T> qn;
    load_poly(P, U, nc, nb, qn);
    for (int k = 0; k < nvar; ++k) {
      if (qn.m[k] > phimax[k]) amax[k] = m + 1;
      if (qn.m[k] < phimin[k]) amin[k] = m + 1;
      phimax[k] = dmax(phimax[k], qn.m[k]);
      phimin[k] = dmin(phimin[k], qn.m[k]);
    }
    for (int d = 0; d < 3; ++d) {
      double off = sides[m] == 0 ? 0.0 : fg.dLR[d];
      rf[m][d] = d < dim ? fg.rc[d] - off : 0.0;
    }
  }
  // code (recorded on request): 0 for alpha = 1, else the face that sets alpha
  // (m + 1), the bound's arg-extremal neighbour << 4 and its side (max) << 8
  auto alpha_of = [&](int k, const T* grad, int* code = nullptr) {
    T alpha = T(1);
    int c = 0;
    for (int m = 0; m < nfc; ++m) {
      T dphi = T(0);
      for (int d = 0; d < dim; ++d) dphi += grad[d] * T(rf[m][d]);
      T psi;
      if (dphi > T(0))
        psi = (phimax[k] - q.m[k]) / dphi;
      else if (dphi < T(0))
        psi = (phimin[k] - q.m[k]) / dphi;
      else
        psi = T(1);
      if (psi < alpha)
        c = (m + 1) | ((dphi > T(0) ? amax[k] : amin[k]) << 4) | (dphi > T(0) ? 256 : 0);
      alpha = dmin(alpha, psi);
    }
    if (code) *code = c;
    return alpha;
  };
  for (int v = 0; v < nh; ++v) {
    int* code = nullptr;
    if (C.br && v < 4) code = C.br + ((int64_t)C.br_stage * nc + e) * kBranchCodes + v;
    T alpha = alpha_of(v, q.g[v], code);
    for (int d = 0; d < dim; ++d) q.g[v][d] = alpha * q.g[v][d];
  }
  if (P.mhd) {
    T aB = T(1);
    for (int c = 0; c < 3; ++c) {
      T gB[3];
      grad_B(P, q, c, gB);
      aB = dmin(aB, alpha_of(5 + c, gB));
    }
    for (int j = 0; j < P.nfun(); ++j) q.a[j] = aB * q.a[j];
  }
  store_poly(P, Ul, nc, e, q);
}

// The WENO-type limiter of Sec. 2.5 on one cell (Euler).  For each primitive
// variable phi (rho, v, p) there are two candidate gradients: the stencil
// gradient, a least-squares fit to the face neighbours' primitive means (the
// FV method's slope), limited as in the Arepo limiter; and the cell's own
// unlimited DG gradient, the primitive gradient at the centroid from the
// conserved mean and gradients by the chain rule.  Each candidate k gets the
// oscillation factor
//   o_k = sum over faces j of |dphi_kj| + |phi_j - (phi_i + dphi_kj)|,
// with dphi_kj = grad_k . (face centroid - cell centroid) and phi_j the
// neighbour's primitive mean; the new gradient is the average of the
// candidates weighted by (eps + o_k)^(-1/2), eps the FP64 machine epsilon.
// The conserved gradients are then recomputed from the primitive ones at the
// centroid (chain rule); the means are unchanged.
template <class T> void limit_cell_weno(const Ctx& C, const T* U, T* Ul, int64_t e) {
  const Mesh& M = *C.mesh;
  const Phys& P = C.P;
  const int dim = P.dim, nh = P.nhyd();
  const int64_t nc = M.nc;
  Poly<T> q;
  load_poly(P, U, nc, e, q);
  Prim<T> pr;
  predict_prim(P, q, 0.0, pr);  // centroid values and DG primitive gradients
  int64_t fids[64];
  int sides[64];
  const int nfc = M.cell_faces(e, fids, sides);
  T wn[64][5];
  double rf[64][3], dn[64][3];
  for (int m = 0; m < nfc; ++m) {
    FaceGeo fg;
    M.face(fids[m], fg);
    const int64_t nb = sides[m] == 0 ? fg.R : fg.L;
    Poly<T> qn;
    load_poly(P, U, nc, nb, qn);
    Prim<T> pn;
    predict_prim(P, qn, 0.0, pn);
    for (int k = 0; k < nh; ++k) wn[m][k] = pn.w[k];
    for (int d = 0; d < 3; ++d) {
      const double off = sides[m] == 0 ? 0.0 : fg.dLR[d];
      rf[m][d] = d < dim ? fg.rc[d] - off : 0.0;
      // neighbour centroid relative to this cell's centroid
      dn[m][d] = d < dim ? (sides[m] == 0 ? fg.dLR[d] : -fg.dLR[d]) : 0.0;
    }
  }
  // least-squares normal matrix of the stencil
  double A[9] = {0};
  for (int m = 0; m < nfc; ++m)
    for (int i = 0; i < dim; ++i)
      for (int j = 0; j < dim; ++j) A[i * dim + j] += dn[m][i] * dn[m][j];
  const double eps = 2.220446049250313e-16;
  T gnew[5][3];
  for (int k = 0; k < nh; ++k) {
    // stencil candidate
    T b[3] = {T(0), T(0), T(0)}, gs[3] = {T(0), T(0), T(0)};
    for (int m = 0; m < nfc; ++m)
      for (int i = 0; i < dim; ++i) b[i] += T(dn[m][i]) * (wn[m][k] - pr.w[k]);
    solve_small(dim, A, b, gs);
    T hi = pr.w[k], lo = pr.w[k];
    for (int m = 0; m < nfc; ++m) {
      hi = dmax(hi, wn[m][k]);
      lo = dmin(lo, wn[m][k]);
    }
    T alpha = T(1);
    for (int m = 0; m < nfc; ++m) {
      T dphi = T(0);
      for (int d = 0; d < dim; ++d) dphi += gs[d] * T(rf[m][d]);
      T psi = T(1);
      if (dphi > T(0))
        psi = (hi - pr.w[k]) / dphi;
      else if (dphi < T(0))
        psi = (lo - pr.w[k]) / dphi;
      alpha = dmin(alpha, psi);
    }
    for (int d = 0; d < dim; ++d) gs[d] = alpha * gs[d];
    // oscillation factors and weights
    const T* cand[2] = {gs, pr.gw[k]};
    T wsum = T(0), acc[3] = {T(0), T(0), T(0)};
    for (int c = 0; c < 2; ++c) {
      T o = T(0);
      for (int m = 0; m < nfc; ++m) {
        T dphi = T(0);
        for (int d = 0; d < dim; ++d) dphi += cand[c][d] * T(rf[m][d]);
        o += dabs(dphi) + dabs(wn[m][k] - (pr.w[k] + dphi));
      }
      const T w = T(1) / dsqrt(T(eps) + o);
      wsum += w;
      for (int d = 0; d < dim; ++d) acc[d] += w * cand[c][d];
    }
    for (int d = 0; d < dim; ++d) gnew[k][d] = acc[d] / wsum;
  }
  // conserved gradients from the primitive ones at the centroid
  const T rho = pr.w[0];
  T v2 = T(0);
  for (int i = 0; i < dim; ++i) v2 += pr.w[1 + i] * pr.w[1 + i];
  for (int d = 0; d < dim; ++d) {
    q.g[0][d] = gnew[0][d];
    T vgv = T(0);
    for (int i = 0; i < dim; ++i) {
      q.g[1 + i][d] = pr.w[1 + i] * gnew[0][d] + rho * gnew[1 + i][d];
      vgv += pr.w[1 + i] * gnew[1 + i][d];
    }
    q.g[1 + dim][d] = gnew[1 + dim][d] / T(P.gamma - 1.0) + T(0.5) * v2 * gnew[0][d] + rho * vgv;
  }
  store_poly(P, Ul, nc, e, q);
}

template <class T> int rhs_all(const Ctx& C, const T* U, T* dUdt, double half_dt = -1.0) {
  int64_t nc = C.mesh->nc;
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (int64_t e = 0; e < nc; ++e)
    if (!rhs_cell(C, U, dUdt, e, half_dt)) bad |= 1;
  return bad;
}

template <class T> void limit_all(const Ctx& C, const T* U, T* Ul) {
  int64_t nc = C.mesh->nc;
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < nc; ++e) {
    if (C.limiter == 2)
      limit_cell_weno(C, U, Ul, e);
    else
      limit_cell(C, U, Ul, e);
  }
}

// One SSP-RK2 step with the limiter at the start of each stage:
//   Ua = Pi(U);  V1 = Ua + dt L(Ua);  Ub = Pi(V1);
//   U_next = Ua/2 + (Ub + dt L(Ub))/2.
template <class T> int step_all(const Ctx& C0, const T* U, double dt, T* Un) {
  Ctx C = C0, C2 = C0;  // the branch record's stage index
  C.br_stage = 0;
  C2.br_stage = 1;
  int64_t len = (int64_t)C.P.ncoef() * C.mesh->nc;
  std::vector<T> Ua(len), V1(len), L(len);
  if (C.limiter)
    limit_all(C, U, Ua.data());
  else
    std::copy(U, U + len, Ua.begin());
  int bad = rhs_all(C, Ua.data(), L.data());
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < len; ++i) V1[i] = Ua[i] + T(dt) * L[i];
  std::vector<T>& Ub = L;  // reuse storage
  if (C2.limiter)
    limit_all(C2, V1.data(), Ub.data());
  else
    std::copy(V1.begin(), V1.end(), Ub.begin());
  std::vector<T>& L2 = V1;
  bad |= rhs_all(C2, Ub.data(), L2.data());
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < len; ++i) Un[i] = T(0.5) * Ua[i] + T(0.5) * (Ub[i] + T(dt) * L2[i]);
  return bad;
}

// One MUSCL-Hancock step (Sec. 2.4), the limiter at the start of the step:
//   Ua = Pi(U);  U_next = Ua + dt L_MH(Ua; dt/2),
// L_MH the surface and volume terms of the half-step primitive prediction.
template <class T> int step_mh_all(const Ctx& C, const T* U, double dt, T* Un) {
  int64_t len = (int64_t)C.P.ncoef() * C.mesh->nc;
  std::vector<T> Ua(len), L(len);
  if (C.limiter)
    limit_all(C, U, Ua.data());
  else
    std::copy(U, U + len, Ua.begin());
  int bad = rhs_all(C, Ua.data(), L.data(), 0.5 * dt);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < len; ++i) Un[i] = Ua[i] + T(dt) * L[i];
  return bad;
}

// CFL time step from the cell means: dt = cfl * min_e 2 V_e /
// sum_f A_f (|v_e . n_f| + c_e(n_f)).
double cfl_dt(const Ctx& C, const double* U, double cfl) {
  const Mesh& M = *C.mesh;
  const Phys& P = C.P;
  int64_t nc = M.nc;
  double best = INFINITY;
#pragma omp parallel for schedule(static) reduction(min : best)
  for (int64_t e = 0; e < nc; ++e) {
    Poly<double> q;
    load_poly(P, U, nc, e, q);
    CellGeo cg;
    M.cell(e, cg);
    int64_t fids[64];
    int sides[64];
    int nfc = M.cell_faces(e, fids, sides);
    double s = 0;
    for (int m = 0; m < nfc; ++m) {
      FaceGeo fg;
      M.face(fids[m], fg);
      double vn = 0;
      for (int d = 0; d < P.nvel(); ++d) vn += q.m[1 + d] / q.m[0] * fg.n[d];
      s += fg.A * (std::fabs(vn) + signal_speed(P, q.m, fg.n));
    }
    best = std::min(best, 2.0 * cg.V / s);
  }
  return cfl * best;
}

Mesh* as_mesh(void* h) { return static_cast<Mesh*>(h); }

// ------------------------------------------------- moving mesh (Sec. 2.3) --
// On a moving mesh the flux through a face moving with velocity w (and the
// flux inside a cell moving with w) is the static flux minus the advection by
// the motion, F_m = F(U) - U w^T; the Riemann problem is solved in the rest
// frame of the face and the result carried back to the lab frame.
//
// Galilean boost of a conserved Euler state into the frame moving with w:
// the density is unchanged, m' = m - rho w, E' = E - m . w + rho |w|^2 / 2.
template <class T> void boost_state(int dim, const T* u, const double* w, T* ub) {
  T mw = T(0);
  double ww = 0.0;
  ub[0] = u[0];
  for (int d = 0; d < dim; ++d) {
    ub[1 + d] = u[1 + d] - u[0] * T(w[d]);
    mw += u[1 + d] * T(w[d]);
    ww += w[d] * w[d];
  }
  ub[1 + dim] = u[1 + dim] - mw + T(0.5 * ww) * u[0];
}

// Lab-frame flux through a surface moving with w, F(U) - U w^T, from the flux
// Fb of the same state in the surface's rest frame: the mass flux is the
// same, the momentum flux gains w times the mass flux, the energy flux gains
// w . (momentum flux) + |w|^2/2 (mass flux).
template <class T> void unboost_flux(int dim, const T* Fb, const double* w, T* F) {
  T wF = T(0);
  double ww = 0.0;
  F[0] = Fb[0];
  for (int d = 0; d < dim; ++d) {
    F[1 + d] = Fb[1 + d] + Fb[0] * T(w[d]);
    wF += Fb[1 + d] * T(w[d]);
    ww += w[d] * w[d];
  }
  F[1 + dim] = Fb[1 + dim] + wF + T(0.5 * ww) * Fb[0];
}

// Velocity of the Voronoi face between generators rL and rR (R's periodic
// image next to L) that move with wL and wR, at the point f of the face: the
// mean of the two velocities plus the normal motion of the bisector at f,
//   w = (wL + wR)/2 + [(wL - wR) . (f - (rL + rR)/2)] (rR - rL) / |rR - rL|^2.
// The normal part varies linearly along the face (the bisector turns when the
// generators move relative to each other), so it is taken at each Gauss point.
void face_velocity(const double* rL, const double* rR, const double* wL, const double* wR,
                   const double* f, double* w) {
  double d[2], dd = 0.0, s = 0.0;
  for (int k = 0; k < 2; ++k) {
    d[k] = rR[k] - rL[k];
    dd += d[k] * d[k];
    s += (wL[k] - wR[k]) * (f[k] - 0.5 * (rL[k] + rR[k]));
  }
  for (int k = 0; k < 2; ++k) w[k] = 0.5 * (wL[k] + wR[k]) + s / dd * d[k];
}

// Periodic minimum image of a coordinate difference.
inline double min_image(double d, double L) { return d - L * std::nearbyint(d / L); }

// One cell of the moving-mesh MUSCL-Hancock update (Sec. 2.3, Sec. 2.4), 2D
// Euler.  The generators move with constant velocities wg over the step; the
// fluxes are taken on the mesh H of the generators at the half step
// t^{n+1/2} (the midpoint rule in time for the moving faces and cells), and N0
// is the mesh at t^n on which the state Ua (already limited) lives.
// Every state is the half-step primitive prediction of its cell (Sec. 2.4),
// centred at the t^n centroid and evaluated at the half-step position of the
// point.  At a face Gauss point the two states are boosted into the frame of
// the face at that point (the bisector's velocity there), the Riemann flux is
// taken in that frame and carried back to the lab frame (F_m = F - U w^T).
// The volume flux is F - U w_e^T on the half-step cell's quadrature points.
// Out, in the state layout: the conserved totals Q0 = V^n ubar + dt (surface
// terms) at k = 3v, and at 3v+1, 3v+2 the first moments about the cell's
// origin carried along with w_e (c^n + (t - t^n) w_e),
//   Q1 = M^n g + dt (surface + volume terms).
template <class T>
bool moving_cell(const Ctx& C, const Mesh& N0, const T* Ua, double dt, const double* gen,
                 const double* wg, T* Q, int64_t e) {
  const Mesh& H = *C.mesh;
  const Phys& P = C.P;
  const int dim = 2, nh = 4;
  const int64_t nc = H.nc;
  const double half = 0.5 * dt;
  CellGeo c0, ch;
  N0.cell(e, c0);
  H.cell(e, ch);
  Poly<T> qe;
  load_poly(P, Ua, nc, e, qe);
  const double* we = &wg[2 * e];
  T S0[4], S1[4][2];
  for (int v = 0; v < nh; ++v) S0[v] = S1[v][0] = S1[v][1] = T(0);
  bool ok = true;
  int64_t fids[64];
  int sides[64];
  const int nfc = H.cell_faces(e, fids, sides);
  for (int m = 0; m < nfc; ++m) {
    const int64_t f = fids[m];
    FaceGeo fg;
    H.face(f, fg);
    Poly<T> qL, qR;
    load_poly(P, Ua, nc, fg.L, qL);
    load_poly(P, Ua, nc, fg.R, qR);
    Prim<T> pL, pR;
    predict_prim(P, qL, half, pL);
    predict_prim(P, qR, half, pR);
    CellGeo cL, cR;
    N0.cell(fg.L, cL);
    N0.cell(fg.R, cR);
    double rL[2], rR[2];
    for (int d = 0; d < 2; ++d) {
      rL[d] = gen[2 * fg.L + d];
      rR[d] = gen[2 * fg.R + d] + H.fsh[2 * f + d];  // fsh holds shift * box
    }
    for (int p = 0; p < fg.ng; ++p) {
      // the Gauss point (in L's periodic frame at the half step), the face
      // velocity there, and its offsets from the t^n centroids
      double xg[2], wf[2], xL[3] = {0, 0, 0}, xR[3] = {0, 0, 0}, r[2];
      for (int d = 0; d < 2; ++d) xg[d] = H.cc[2 * fg.L + d] + fg.rg[p][d];
      face_velocity(rL, rR, &wg[2 * fg.L], &wg[2 * fg.R], xg, wf);
      for (int d = 0; d < 2; ++d) {
        xL[d] = min_image(xg[d] - cL.c[d], H.box[d]);
        xR[d] = min_image(xg[d] - cR.c[d], H.box[d]);
        // relative to this cell's carried origin c^n + (dt/2) w_e
        r[d] = (sides[m] == 0 ? xL[d] : xR[d]) - half * we[d];
      }
      T uL[4], uR[4], bL[4], bR[4], Fb[4], F[4];
      eval_prim(P, pL, xL, uL);
      eval_prim(P, pR, xR, uR);
      if (!physical(P, uL) || !physical(P, uR)) ok = false;
      boost_state(dim, uL, wf, bL);
      boost_state(dim, uR, wf, bR);
      if (P.riemann == 1) {
        if (!exact_riemann(P, bL, bR, fg.n, Fb)) ok = false;
      } else {
        hll(P, bL, bR, fg.n, Fb);
      }
      unboost_flux(dim, Fb, wf, F);
      const T sg = sides[m] == 0 ? T(-fg.wg[p]) : T(fg.wg[p]);
      for (int v = 0; v < nh; ++v) {
        S0[v] += sg * F[v];
        for (int d = 0; d < 2; ++d) S1[v][d] += sg * F[v] * T(r[d]);
      }
    }
  }
  Prim<T> pe;
  predict_prim(P, qe, half, pe);
  for (int q = 0; q < ch.nq; ++q) {
    double x[3] = {0, 0, 0};
    for (int d = 0; d < 2; ++d) x[d] = min_image(ch.c[d] + ch.rq[q][d] - c0.c[d], H.box[d]);
    T u[4], b[4];
    eval_prim(P, pe, x, u);
    if (!physical(P, u)) ok = false;
    boost_state(dim, u, we, b);
    const T w = T(ch.wq[q]);
    for (int d = 0; d < 2; ++d) {
      double nd[3] = {0, 0, 0};
      nd[d] = 1.0;
      T Fb[4], F[4];
      flux_n(P, b, nd, Fb);
      unboost_flux(dim, Fb, we, F);
      for (int v = 0; v < nh; ++v) S1[v][d] += w * F[v];
    }
  }
  for (int v = 0; v < nh; ++v) {
    Q[(int64_t)(3 * v) * nc + e] = T(c0.V) * qe.m[v] + T(dt) * S0[v];
    for (int d = 0; d < 2; ++d) {
      T mg = T(c0.M[d][0]) * qe.g[v][0] + T(c0.M[d][1]) * qe.g[v][1];
      Q[(int64_t)(3 * v + 1 + d) * nc + e] = mg + T(dt) * S1[v][d];
    }
  }
  return ok;
}

// CFL step on a moving mesh: dt = cfl * min_e 2 V_e / sum_f A_f (|(v_e - w_e)
// . n_f| + c_e), the signal speed relative to the cell's own motion.
double cfl_dt_moving(const Ctx& C, const double* U, const double* wg, double cfl) {
  const Mesh& M = *C.mesh;
  const Phys& P = C.P;
  const int64_t nc = M.nc;
  double best = INFINITY;
#pragma omp parallel for schedule(static) reduction(min : best)
  for (int64_t e = 0; e < nc; ++e) {
    Poly<double> q;
    load_poly(P, U, nc, e, q);
    CellGeo cg;
    M.cell(e, cg);
    int64_t fids[64];
    int sides[64];
    const int nfc = M.cell_faces(e, fids, sides);
    double s = 0;
    for (int m = 0; m < nfc; ++m) {
      FaceGeo fg;
      M.face(fids[m], fg);
      double vn = 0;
      for (int d = 0; d < 2; ++d) vn += (q.m[1 + d] / q.m[0] - wg[2 * e + d]) * fg.n[d];
      s += fg.A * (std::fabs(vn) + signal_speed(P, q.m, fg.n));
    }
    best = std::min(best, 2.0 * cg.V / s);
  }
  return cfl * best;
}

}  // namespace

// ----------------------------------------------------------------- C ABI --
extern "C" {

int or_num_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

void or_set_num_threads(int n) {
#ifdef _OPENMP
  if (n > 0) omp_set_num_threads(n);
#else
  (void)n;
#endif
}

// Periodic Cartesian mesh of n[0] x n[1] (x n[2]) cells on [lo, hi].
void* or_mesh_cartesian(int dim, const int64_t* n, const double* lo, const double* hi) {
  Mesh* m = new Mesh();
  m->dim = dim;
  m->kind = 0;
  m->nc = 1;
  for (int d = 0; d < 3; ++d) {
    m->N[d] = d < dim ? n[d] : 1;
    m->lo[d] = d < dim ? lo[d] : 0.0;
    m->h[d] = d < dim ? (hi[d] - lo[d]) / n[d] : 1.0;
    m->nc *= m->N[d];
  }
  m->nf = dim * m->nc;
  return m;
}

// Periodic 2D face-list mesh.  face_shift holds integers in {-1,0,1}: the
// image of R next to L is c_R + shift * box.
void* or_mesh_facelist2d(int64_t ncells, int64_t nfaces, const double* box,
                         const double* cell_volume, const double* cell_centroid,
                         const double* cell_moments, const int32_t* face_cells,
                         const double* face_area, const double* face_normal,
                         const double* face_centroid, const int8_t* face_shift) {
  Mesh* m = new Mesh();
  m->dim = 2;
  m->kind = 1;
  m->nc = ncells;
  m->nf = nfaces;
  m->box[0] = box[0];
  m->box[1] = box[1];
  m->cV.assign(cell_volume, cell_volume + ncells);
  m->cc.assign(cell_centroid, cell_centroid + 2 * ncells);
  m->cM.assign(cell_moments, cell_moments + 3 * ncells);
  m->fL.resize(nfaces);
  m->fR.resize(nfaces);
  m->fA.assign(face_area, face_area + nfaces);
  m->fn.assign(face_normal, face_normal + 2 * nfaces);
  m->fx.assign(face_centroid, face_centroid + 2 * nfaces);
  m->fsh.resize(2 * nfaces);
  std::vector<int64_t> cnt(ncells + 1, 0);
  for (int64_t f = 0; f < nfaces; ++f) {
    m->fL[f] = face_cells[2 * f];
    m->fR[f] = face_cells[2 * f + 1];
    for (int d = 0; d < 2; ++d) m->fsh[2 * f + d] = face_shift[2 * f + d] * box[d];
    cnt[m->fL[f] + 1]++;
    cnt[m->fR[f] + 1]++;
  }
  for (int64_t e = 0; e < ncells; ++e) cnt[e + 1] += cnt[e];
  m->cptr = cnt;
  m->cf.resize(cnt[ncells]);
  m->cside.resize(cnt[ncells]);
  std::vector<int64_t> fill(cnt.begin(), cnt.end() - 1);
  for (int64_t f = 0; f < nfaces; ++f) {
    int64_t L = m->fL[f], R = m->fR[f];
    m->cf[fill[L]] = f;
    m->cside[fill[L]++] = 0;
    m->cf[fill[R]] = f;
    m->cside[fill[R]++] = 1;
  }
  return m;
}

void or_mesh_free(void* h) { delete as_mesh(h); }
int64_t or_mesh_ncells(void* h) { return as_mesh(h)->nc; }

int or_ncoef(int dim, int mhd) {
  Phys P{dim, mhd, 1.4};
  return P.ncoef();
}

// L(U).  Returns 0, or 5 when a non-physical state was met.
int or_rhs(void* h, int mhd, int riemann, double gamma, const double* U, double* dUdt) {
  Ctx C{as_mesh(h), Phys{as_mesh(h)->dim, mhd, gamma, riemann}, 0};
  return rhs_all(C, U, dUdt) ? 5 : 0;
}

// kind: 1 the Arepo limiter, 2 the WENO-type limiter (Euler; gamma is used
// for the primitive variables).
void or_limit(void* h, int mhd, int kind, double gamma, const double* U, double* Ul) {
  Ctx C{as_mesh(h), Phys{as_mesh(h)->dim, mhd, gamma}, kind};
  limit_all(C, U, Ul);
}

int or_step(void* h, int mhd, int riemann, int limiter, double gamma, const double* U, double dt,
            double* Un) {
  Ctx C{as_mesh(h), Phys{as_mesh(h)->dim, mhd, gamma, riemann}, limiter};
  return step_all(C, U, dt, Un) ? 5 : 0;
}

// MUSCL-Hancock step and operator (Euler only; 5 = non-physical, 4 = MHD).
// One SSP-RK2 step (2D Euler on a box, HLL) that also records the branches it
// takes: codes[2][ncells][12] (per stage and cell: the limiter of the four
// variables, then HLL at the two Gauss points of the four faces, in the
// cell's face order -x, +x, -y, +y).  Returns 1 on a non-physical state, 2 if
// the mesh or physics is not a 2D box with Euler.
int or_step_branches(void* h, int limiter, double gamma, const double* U, double dt, double* Un,
                     int* codes) {
  Mesh* M = as_mesh(h);
  if (M->kind != 0 || M->dim != 2) return 2;
  Ctx C{M, Phys{2, 0, gamma}, limiter};
  C.br = codes;
  std::fill(codes, codes + 2 * M->nc * kBranchCodes, 0);
  return step_all(C, U, dt, Un);
}

int or_step_mh(void* h, int riemann, int limiter, double gamma, const double* U, double dt,
               double* Un) {
  Ctx C{as_mesh(h), Phys{as_mesh(h)->dim, 0, gamma, riemann}, limiter};
  return step_mh_all(C, U, dt, Un) ? 5 : 0;
}

int or_rhs_mh(void* h, int riemann, double gamma, const double* U, double half_dt, double* L) {
  Ctx C{as_mesh(h), Phys{as_mesh(h)->dim, 0, gamma, riemann}, 0};
  if (!(half_dt >= 0)) return 1;
  return rhs_all(C, U, L, half_dt) ? 5 : 0;
}

// The predicted primitive polynomial of one cell state (for unit pins):
// prim[0..dim+1] the centroid values advanced by half_dt, gprim[k*3+d] the
// primitive gradients.
void or_predict_prim(int dim, double gamma, const double* mean, const double* grad,
                     double half_dt, double* prim, double* gprim) {
  Phys P{dim, 0, gamma};
  Poly<double> q;
  for (int v = 0; v < dim + 2; ++v) {
    q.m[v] = mean[v];
    for (int d = 0; d < 3; ++d) q.g[v][d] = d < dim ? grad[v * dim + d] : 0.0;
  }
  Prim<double> pr;
  predict_prim(P, q, half_dt, pr);
  for (int k = 0; k < dim + 2; ++k) {
    prim[k] = pr.w[k];
    for (int d = 0; d < 3; ++d) gprim[k * 3 + d] = d < dim ? pr.gw[k][d] : 0.0;
  }
}

// Directional derivative of one step: Un = S(U), dUn = (dS/dU) dU.
int or_step_jvp(void* h, int mhd, int limiter, double gamma, const double* U, const double* dU,
                double dt, double* Un, double* dUn) {
  Ctx C{as_mesh(h), Phys{as_mesh(h)->dim, mhd, gamma}, limiter};
  int64_t len = (int64_t)C.P.ncoef() * C.mesh->nc;
  std::vector<Dual> x(len), y(len);
  for (int64_t i = 0; i < len; ++i) x[i] = Dual(U[i], dU[i]);
  int bad = step_all(C, x.data(), dt, y.data());
  for (int64_t i = 0; i < len; ++i) {
    Un[i] = y[i].v;
    dUn[i] = y[i].d;
  }
  return bad ? 5 : 0;
}

int or_rhs_jvp(void* h, int mhd, double gamma, const double* U, const double* dU, double* L,
               double* dL) {
  Ctx C{as_mesh(h), Phys{as_mesh(h)->dim, mhd, gamma}, 0};
  int64_t len = (int64_t)C.P.ncoef() * C.mesh->nc;
  std::vector<Dual> x(len), y(len);
  for (int64_t i = 0; i < len; ++i) x[i] = Dual(U[i], dU[i]);
  int bad = rhs_all(C, x.data(), y.data());
  for (int64_t i = 0; i < len; ++i) {
    L[i] = y[i].v;
    dL[i] = y[i].d;
  }
  return bad ? 5 : 0;
}

double or_cfl_dt(void* h, int mhd, double gamma, const double* U, double cfl) {
  Ctx C{as_mesh(h), Phys{as_mesh(h)->dim, mhd, gamma}, 0};
  return cfl_dt(C, U, cfl);
}

// Riemann solvers and the physical flux on single states (for unit pins).
void or_flux(int dim, int mhd, double gamma, const double* u, const double* n, double* F) {
  Phys P{dim, mhd, gamma};
  flux_n(P, u, n, F);
}
void or_hll(int dim, int mhd, double gamma, const double* uL, const double* uR, const double* n,
            double* F) {
  Phys P{dim, mhd, gamma};
  hll(P, uL, uR, n, F);
}
void or_hlld(double gamma, const double* uL, const double* uR, const double* n, double* F) {
  Phys P{3, 1, gamma};
  hlld(P, uL, uR, n, F);
}
// Signal speed of one state along the unit normal n: the sound speed
// (Euler) or the fast magnetosonic speed (MHD), the speed the CFL bound and
// the outer HLL/HLLD wave estimates use.
double or_signal_speed(int dim, int mhd, double gamma, const double* u, const double* n) {
  Phys P{dim, mhd, gamma};
  return signal_speed(P, u, n);
}
// Exact Euler Riemann solver on single states: flux F, star = (p*, u*) and
// the primitive state (rho, u_n, p) on the face.  Returns 0, or 1 on vacuum
// generation.
int or_exact_riemann(int dim, double gamma, const double* uL, const double* uR, const double* n,
                     double* F, double* star, double* face_state) {
  Phys P{dim, 0, gamma, 1};
  return exact_riemann(P, uL, uR, n, F, star, face_state) ? 0 : 1;
}

// Mesh geometry as the oracle sees it (for pins): volume, centroid, second
// moments, quadrature points and weights of one cell.
void or_cell_geometry(void* h, int64_t e, double* V, double* c, double* M, int* nq, double* rq,
                      double* wq) {
  CellGeo g;
  as_mesh(h)->cell(e, g);
  *V = g.V;
  for (int d = 0; d < 3; ++d) c[d] = g.c[d];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) M[3 * i + j] = g.M[i][j];
  *nq = g.nq;
  for (int q = 0; q < g.nq; ++q) {
    for (int d = 0; d < 3; ++d) rq[3 * q + d] = g.rq[q][d];
    wq[q] = g.wq[q];
  }
}

// Gram matrix of V4..V11 for a second-moment matrix M (row-major 3x3).
void or_gram_B(const double* M, double* G) {
  double m[3][3];
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) m[i][j] = M[3 * i + j];
  gram_B(Phys{3, 1, 1.4}, m, G);
}

// Gram matrix of the 2D B basis (V3, V4, V5, then the B_z Taylor functions)
// from the 2x2 second-moment matrix M (row-major); G is 5x5.
void or_gram_B2(const double* M, double* G) {
  double m[3][3] = {{M[0], M[1], 0.0}, {M[2], M[3], 0.0}, {0.0, 0.0, 0.0}};
  gram_B(Phys{2, 1, 1.4}, m, G);
}

// Evaluate the B polynomial (Bbar, a4..a11) at offset r.
void or_eval_B(const double* bbar, const double* a, const double* r, double* B) {
  Phys P{3, 1, 1.4};
  Poly<double> q;
  std::memset(&q, 0, sizeof(q));
  for (int c = 0; c < 3; ++c) q.m[5 + c] = bbar[c];
  for (int j = 0; j < 8; ++j) q.a[j] = a[j];
  double u[8];
  eval_poly(P, q, r, u);
  for (int c = 0; c < 3; ++c) B[c] = u[5 + c];
}

// Stokes estimate of div B per cell (Sec. 2.6): (1/V) sum_faces B_n A, with
// B_n the face average of the two extrapolated normal fields at the face
// Gauss points.
void or_divB(void* h, const double* U, double* divB) {
  const Mesh& M = *as_mesh(h);
  Phys P{M.dim, 1, 1.4};
  int64_t nc = M.nc;
#pragma omp parallel for schedule(static)
  for (int64_t e = 0; e < nc; ++e) {
    CellGeo cg;
    M.cell(e, cg);
    int64_t fids[64];
    int sides[64];
    int nfc = M.cell_faces(e, fids, sides);
    double s = 0;
    for (int m = 0; m < nfc; ++m) {
      FaceGeo fg;
      M.face(fids[m], fg);
      Poly<double> qL, qR;
      load_poly(P, U, nc, fg.L, qL);
      load_poly(P, U, nc, fg.R, qR);
      for (int p = 0; p < fg.ng; ++p) {
        double rL[3], rR[3], uL[8], uR[8];
        for (int d = 0; d < 3; ++d) {
          rL[d] = fg.rg[p][d];
          rR[d] = fg.rg[p][d] - fg.dLR[d];
        }
        eval_poly(P, qL, rL, uL);
        eval_poly(P, qR, rR, uR);
        double bn = 0;
        for (int d = 0; d < 3; ++d) bn += 0.5 * (uL[5 + d] + uR[5 + d]) * fg.n[d];
        s += (sides[m] == 0 ? 1.0 : -1.0) * fg.wg[p] * bn;
      }
    }
    divB[e] = s / cg.V;
  }
}

// Moving-mesh MUSCL-Hancock update (2D Euler): h0 the face-list mesh at t^n
// (the state's mesh), hh the mesh of the generators at the half step,
// gen_half[ncells][2] those generator positions, wg[ncells][2] the generator
// velocities.  The limiter (0 none, 1 Arepo, 2 WENO-type) acts on h0 at the
// start of the step; Q receives the totals and moments of moving_cell.
// Returns 0, or 5 on a non-physical state.
int or_moving_update(void* h0, void* hh, int riemann, int limiter, double gamma, const double* U,
                     double dt, const double* gen_half, const double* wg, double* Q) {
  Ctx C0{as_mesh(h0), Phys{2, 0, gamma, riemann}, limiter};
  Ctx C{as_mesh(hh), Phys{2, 0, gamma, riemann}, limiter};
  const int64_t nc = C0.mesh->nc, len = 12 * nc;
  if (C.mesh->nc != nc) return 1;
  std::vector<double> Ua(len);
  if (limiter)
    limit_all(C0, U, Ua.data());
  else
    std::copy(U, U + len, Ua.begin());
  int bad = 0;
#pragma omp parallel for schedule(static) reduction(| : bad)
  for (int64_t e = 0; e < nc; ++e)
    if (!moving_cell(C, *C0.mesh, Ua.data(), dt, gen_half, wg, Q, e)) bad |= 1;
  return bad ? 5 : 0;
}

double or_cfl_dt_moving(void* h, double gamma, const double* U, const double* wg, double cfl) {
  Ctx C{as_mesh(h), Phys{2, 0, gamma}, 0};
  return cfl_dt_moving(C, U, wg, cfl);
}

}  // extern "C"
