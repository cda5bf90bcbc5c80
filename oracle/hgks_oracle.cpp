// CPU FP64 oracle of the implicit high-order gas-kinetic scheme on tetrahedra.
//
// TEST INFRASTRUCTURE ONLY: plain, slow and written to be checked against the
// paper by eye.  Only the tests, the smoke check and the CPU baseline leg of
// the benchmark use it; the product library never links or calls it and the
// two share no code.
//
// Readings of points the paper leaves open are fixed once and listed in the
// design notes; the comments below name the reading where one is used
// (A1 ... A27 refer to that list of readings).
#include "hgks_oracle.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>
#include <map>
#include <string>
#include <unordered_map>
#include <vector>
#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

using V3 = std::array<double, 3>;
using V5 = std::array<double, 5>;
using M33 = std::array<std::array<double, 3>, 3>;

thread_local std::string g_err;

V3 sub(const V3& a, const V3& b) { return {a[0] - b[0], a[1] - b[1], a[2] - b[2]}; }
V3 add(const V3& a, const V3& b) { return {a[0] + b[0], a[1] + b[1], a[2] + b[2]}; }
V3 scl(double s, const V3& a) { return {s * a[0], s * a[1], s * a[2]}; }
double dot(const V3& a, const V3& b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }
V3 cross(const V3& a, const V3& b) {
  return {a[1] * b[2] - a[2] * b[1], a[2] * b[0] - a[0] * b[2], a[0] * b[1] - a[1] * b[0]};
}
double norm(const V3& a) { return std::sqrt(dot(a, a)); }

// ---------------------------------------------------------------------------
// small dense linear algebra (plain textbook routines)
// ---------------------------------------------------------------------------

// Solve A x = b (n x n, row-major, copied) by Gaussian elimination with partial
// pivoting.  Returns false if singular.
bool gauss_solve(std::vector<double> A, std::vector<double> b, int n, int nrhs,
                 std::vector<double>& x) {
  for (int k = 0; k < n; ++k) {
    int piv = k;
    for (int r = k + 1; r < n; ++r)
      if (std::fabs(A[r * n + k]) > std::fabs(A[piv * n + k])) piv = r;
    if (A[piv * n + k] == 0.0) return false;
    if (piv != k) {
      for (int c = 0; c < n; ++c) std::swap(A[k * n + c], A[piv * n + c]);
      for (int c = 0; c < nrhs; ++c) std::swap(b[k * nrhs + c], b[piv * nrhs + c]);
    }
    for (int r = k + 1; r < n; ++r) {
      double f = A[r * n + k] / A[k * n + k];
      if (f == 0.0) continue;
      for (int c = k; c < n; ++c) A[r * n + c] -= f * A[k * n + c];
      for (int c = 0; c < nrhs; ++c) b[r * nrhs + c] -= f * b[k * nrhs + c];
    }
  }
  x.assign(n * nrhs, 0.0);
  for (int c = 0; c < nrhs; ++c)
    for (int k = n - 1; k >= 0; --k) {
      double s = b[k * nrhs + c];
      for (int j = k + 1; j < n; ++j) s -= A[k * n + j] * x[j * nrhs + c];
      x[k * nrhs + c] = s / A[k * n + k];
    }
  return true;
}

// Least squares min ||A x - B|| by Householder QR (A is m x n, m >= n,
// row-major; B is m x nrhs).  X is n x nrhs.
void householder_lsq(std::vector<double> A, std::vector<double> B, int m, int n, int nrhs,
                     std::vector<double>& X) {
  for (int k = 0; k < n; ++k) {
    double s = 0.0;
    for (int r = k; r < m; ++r) s += A[r * n + k] * A[r * n + k];
    double alpha = std::sqrt(s);
    if (alpha == 0.0) continue;
    if (A[k * n + k] > 0) alpha = -alpha;
    std::vector<double> v(m, 0.0);
    for (int r = k; r < m; ++r) v[r] = A[r * n + k];
    v[k] -= alpha;
    double vv = 0.0;
    for (int r = k; r < m; ++r) vv += v[r] * v[r];
    if (vv == 0.0) continue;
    for (int c = k; c < n; ++c) {
      double d = 0.0;
      for (int r = k; r < m; ++r) d += v[r] * A[r * n + c];
      d = 2.0 * d / vv;
      for (int r = k; r < m; ++r) A[r * n + c] -= d * v[r];
    }
    for (int c = 0; c < nrhs; ++c) {
      double d = 0.0;
      for (int r = k; r < m; ++r) d += v[r] * B[r * nrhs + c];
      d = 2.0 * d / vv;
      for (int r = k; r < m; ++r) B[r * nrhs + c] -= d * v[r];
    }
  }
  X.assign(n * nrhs, 0.0);
  for (int c = 0; c < nrhs; ++c)
    for (int k = n - 1; k >= 0; --k) {
      double s = B[k * nrhs + c];
      for (int j = k + 1; j < n; ++j) s -= A[k * n + j] * X[j * nrhs + c];
      X[k * nrhs + c] = s / A[k * n + k];
    }
}

// Eigenvalues of a symmetric n x n matrix by cyclic Jacobi rotations.
std::vector<double> sym_eigenvalues(std::vector<double> A, int n) {
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += A[p * n + q] * A[p * n + q];
    if (off < 1e-300) break;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) {
        double apq = A[p * n + q];
        if (apq == 0.0) continue;
        double theta = (A[q * n + q] - A[p * n + p]) / (2.0 * apq);
        double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < n; ++k) {
          double akp = A[k * n + p], akq = A[k * n + q];
          A[k * n + p] = c * akp - s * akq;
          A[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          double apk = A[p * n + k], aqk = A[q * n + k];
          A[p * n + k] = c * apk - s * aqk;
          A[q * n + k] = s * apk + c * aqk;
        }
      }
  }
  std::vector<double> e(n);
  for (int i = 0; i < n; ++i) e[i] = A[i * n + i];
  return e;
}

// Rank test of reading A17: the LS matrix (in scaled coordinates) is taken as
// rank deficient when sigma_min / sigma_max < 1e-10.
bool full_rank(const std::vector<double>& A, int m, int n) {
  if (m < n) return false;
  std::vector<double> G(n * n, 0.0);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j)
      for (int r = 0; r < m; ++r) G[i * n + j] += A[r * n + i] * A[r * n + j];
  std::vector<double> e = sym_eigenvalues(G, n);
  double mx = *std::max_element(e.begin(), e.end());
  double mn = *std::min_element(e.begin(), e.end());
  return mx > 0 && mn > 1e-20 * mx;
}

// ---------------------------------------------------------------------------
// Maxwellian velocity moments (Sec. 2): g = rho (lam/pi)^((K+3)/2)
// exp(-lam((u-U)^2+(v-V)^2+(w-W)^2+xi^2)), moments normalised by rho.
// ---------------------------------------------------------------------------
struct Moments {
  double mu[9], mv[9], mw[9], mxi[3];

  // half = +1: integral over u > 0, -1: over u < 0, 0: full space
  void init(double U, double V, double W, double lam, double K, int half) {
    if (half == 0) {
      mu[0] = 1.0;
      mu[1] = U;
    } else {
      double e = std::exp(-lam * U * U) / std::sqrt(M_PI * lam);
      if (half > 0) {
        mu[0] = 0.5 * std::erfc(-std::sqrt(lam) * U);
        mu[1] = U * mu[0] + 0.5 * e;
      } else {
        mu[0] = 0.5 * std::erfc(std::sqrt(lam) * U);
        mu[1] = U * mu[0] - 0.5 * e;
      }
    }
    mv[0] = 1.0; mv[1] = V;
    mw[0] = 1.0; mw[1] = W;
    for (int k = 2; k < 9; ++k) {
      mu[k] = U * mu[k - 1] + (k - 1) / (2.0 * lam) * mu[k - 2];
      mv[k] = V * mv[k - 1] + (k - 1) / (2.0 * lam) * mv[k - 2];
      mw[k] = W * mw[k - 1] + (k - 1) / (2.0 * lam) * mw[k - 2];
    }
    mxi[0] = 1.0;
    mxi[1] = K / (2.0 * lam);
    mxi[2] = K * (K + 2.0) / (4.0 * lam * lam);
  }
  double m(int a, int b, int c, int d) const { return mu[a] * mv[b] * mw[c] * mxi[d]; }
  // <u^a v^b w^c xi^(2d) psi>, psi = (1, u, v, w, (u^2+v^2+w^2+xi^2)/2)
  V5 psi(int a, int b, int c, int d) const {
    return {m(a, b, c, d), m(a + 1, b, c, d), m(a, b + 1, c, d), m(a, b, c + 1, d),
            0.5 * (m(a + 2, b, c, d) + m(a, b + 2, c, d) + m(a, b, c + 2, d) + m(a, b, c, d + 1))};
  }
  // <(co . psi) u^a v^b w^c psi>
  V5 apsi(const V5& co, int a, int b, int c) const {
    V5 r{0, 0, 0, 0, 0};
    auto acc = [&](double s, const V5& t) {
      for (int k = 0; k < 5; ++k) r[k] += s * t[k];
    };
    acc(co[0], psi(a, b, c, 0));
    acc(co[1], psi(a + 1, b, c, 0));
    acc(co[2], psi(a, b + 1, c, 0));
    acc(co[3], psi(a, b, c + 1, 0));
    acc(0.5 * co[4], psi(a + 2, b, c, 0));
    acc(0.5 * co[4], psi(a, b + 2, c, 0));
    acc(0.5 * co[4], psi(a, b, c + 2, 0));
    acc(0.5 * co[4], psi(a, b, c, 1));
    return r;
  }
};

// Solve <a psi> = rhs for the expansion coefficients a of Sec. 2 (the 5x5
// moment system with the full-space Maxwellian), by plain elimination.
V5 slope_solve(const Moments& M, const V5& rhs) {
  std::vector<double> A(25), b(rhs.begin(), rhs.end()), x;
  for (int j = 0; j < 5; ++j) {
    V5 e{0, 0, 0, 0, 0};
    e[j] = 1.0;
    V5 col = M.apsi(e, 0, 0, 0);
    for (int k = 0; k < 5; ++k) A[k * 5 + j] = col[k];
  }
  gauss_solve(A, b, 5, 1, x);
  return {x[0], x[1], x[2], x[3], x[4]};
}

struct Prim {
  double rho, U, V, W, p, lam;
};
Prim to_prim(const V5& q, double gamma) {
  Prim s;
  s.rho = q[0];
  s.U = q[1] / q[0];
  s.V = q[2] / q[0];
  s.W = q[3] / q[0];
  s.p = (gamma - 1.0) * (q[4] - 0.5 * s.rho * (s.U * s.U + s.V * s.V + s.W * s.W));
  s.lam = s.rho / (2.0 * s.p);
  return s;
}
V5 to_cons(double rho, const V3& U, double p, double gamma) {
  return {rho, rho * U[0], rho * U[1], rho * U[2],
          p / (gamma - 1.0) + 0.5 * rho * dot(U, U)};
}
bool physical(const V5& q, double gamma) {
  if (!(q[0] > 0.0) || !std::isfinite(q[4])) return false;
  double p = (gamma - 1.0) * (q[4] - 0.5 * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) / q[0]);
  return p > 0.0 && std::isfinite(p);
}

// ---------------------------------------------------------------------------
// the oracle context
// ---------------------------------------------------------------------------
struct Face {
  int L = -1, R = -1;  // R < 0: boundary face, ghost id -R-1
  int pL = -1, pR = -1;
  V3 n{}, t1{}, t2{}, xc{};
  double S = 0.0;
  int ng = 3;      // Gauss points: 3 on a triangle, 4 on a quadrilateral
  V3 gp[4];
  double gw[4] = {0, 0, 0, 0};  // quadrature weights (quadrilaterals; 1/3 each on triangles)
  int kind = -1;  // boundary kind, -1 interior
};

struct Ghost {
  int owner, face;
  V3 c;
  M33 m2;
  double vol;
};

}  // namespace

struct orc_ctx {
  orc_options o;
  double K;  // internal degrees of freedom (5-3 gamma)/(gamma-1), A2
  V5 qinf;
  V3 uinf;
  double rhoinf, pinf;
  int N = 0;
  std::vector<double> vol, hcell, hdt;
  std::vector<V3> cen;
  std::vector<M33> m2;
  std::vector<Face> faces;
  int nf = 4;  // faces per cell: 4 tetrahedra, 6 hexahedra
  std::vector<std::array<int, 6>> cf, nb;
  std::vector<Ghost> ghosts;
  std::vector<std::vector<int>> big;
  std::vector<std::vector<std::vector<int>>> sub;  // non-compact sub-stencils per cell

  bool is_ghost(int e) const { return e >= N; }
  const V3& c_of(int e) const { return e < N ? cen[e] : ghosts[e - N].c; }
  const M33& m2_of(int e) const { return e < N ? m2[e] : ghosts[e - N].m2; }
  double vol_of(int e) const { return e < N ? vol[e] : ghosts[e - N].vol; }
};

namespace {

int nthreads_req = 1;

// Tangent rule of reading A4: t1 = normalise(n x e_k) with e_k the axis of the
// smallest |n_k| (ties -> lowest k), t2 = n x t1.
void tangents(const V3& n, V3& t1, V3& t2) {
  int k = 0;
  for (int j = 1; j < 3; ++j)
    if (std::fabs(n[j]) < std::fabs(n[k])) k = j;
  V3 e{0, 0, 0};
  e[k] = 1.0;
  t1 = cross(n, e);
  t1 = scl(1.0 / norm(t1), t1);
  t2 = cross(n, t1);
}

// local frame rotation of a conserved state (momentum onto n, t1, t2)
V5 to_local(const V5& q, const Face& f) {
  V3 m{q[1], q[2], q[3]};
  return {q[0], dot(m, f.n), dot(m, f.t1), dot(m, f.t2), q[4]};
}
V5 to_global(const V5& q, const Face& f) {
  V5 r;
  r[0] = q[0];
  for (int d = 0; d < 3; ++d) r[1 + d] = q[1] * f.n[d] + q[2] * f.t1[d] + q[3] * f.t2[d];
  r[4] = q[4];
  return r;
}

// Far-field state from local Riemann invariants along the normal nn (reading
// A16): supersonic in -> free stream, supersonic out -> interior; otherwise
// R+ from the interior, R- from the free stream; entropy and tangential
// velocity from the upwind side.
V5 farfield_state(const orc_ctx& C, const V5& qi, const V3& nn, const V3& uinf) {
  double g = C.o.gamma;
  Prim s = to_prim(qi, g);
  V3 Ui{s.U, s.V, s.W};
  double ci = std::sqrt(g * s.p / s.rho);
  double uni = dot(Ui, nn);
  V5 qinf = to_cons(C.rhoinf, uinf, C.pinf, g);
  if (uni <= -ci) return qinf;
  if (uni >= ci) return qi;
  double cinf = std::sqrt(g * C.pinf / C.rhoinf);
  double uninf = dot(uinf, nn);
  double Rp = uni + 2.0 * ci / (g - 1.0);
  double Rm = uninf - 2.0 * cinf / (g - 1.0);
  double unb = 0.5 * (Rp + Rm);
  double cb = 0.25 * (g - 1.0) * (Rp - Rm);
  double ent;
  V3 Ut;
  if (unb < 0.0) {
    ent = C.pinf / std::pow(C.rhoinf, g);
    Ut = sub(uinf, scl(uninf, nn));
  } else {
    ent = s.p / std::pow(s.rho, g);
    Ut = sub(Ui, scl(uni, nn));
  }
  double rb = std::pow(cb * cb / (g * ent), 1.0 / (g - 1.0));
  double pb = rb * cb * cb / g;
  return to_cons(rb, add(Ut, scl(unb, nn)), pb, g);
}

// ghost cell average (global frame) of a boundary face, reading A16
V5 ghost_state(const orc_ctx& C, const Face& f, const V5& qo) {
  V5 q = qo;
  V3 m{qo[1], qo[2], qo[3]};
  switch (f.kind) {
    case ORC_SLIP: {
      V3 r = sub(m, scl(2.0 * dot(m, f.n), f.n));
      q[1] = r[0]; q[2] = r[1]; q[3] = r[2];
      break;
    }
    case ORC_NOSLIP:
      q[1] = -m[0]; q[2] = -m[1]; q[3] = -m[2];
      break;
    case ORC_FARFIELD:
      q = farfield_state(C, qo, f.n, C.uinf);
      break;
    case ORC_SUP_IN:
      q = C.qinf;
      break;
    default:
      break;
  }
  return q;
}

// ghost cell-averaged gradient (rows var, columns x,y,z), reading A16
void ghost_gradient(const Face& f, const double* Go /*15*/, double* Gg /*15*/) {
  if (f.kind == ORC_FARFIELD || f.kind == ORC_SUP_IN) {
    for (int k = 0; k < 15; ++k) Gg[k] = 0.0;
    return;
  }
  if (f.kind == ORC_SUP_OUT) {
    for (int k = 0; k < 15; ++k) Gg[k] = Go[k];
    return;
  }
  // mirror: x -> Rm x with Rm = I - 2 n n^T; grad of q(Rm x) = grad q . Rm
  double Rm[3][3];
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) Rm[a][b] = (a == b ? 1.0 : 0.0) - 2.0 * f.n[a] * f.n[b];
  double GR[5][3];
  for (int v = 0; v < 5; ++v)
    for (int b = 0; b < 3; ++b) {
      double s = 0.0;
      for (int a = 0; a < 3; ++a) s += Go[v * 3 + a] * Rm[a][b];
      GR[v][b] = s;
    }
  for (int b = 0; b < 3; ++b) {
    Gg[0 * 3 + b] = GR[0][b];
    Gg[4 * 3 + b] = GR[4][b];
  }
  if (f.kind == ORC_SLIP) {
    for (int b = 0; b < 3; ++b)
      for (int a = 0; a < 3; ++a) {
        double s = 0.0;
        for (int k = 0; k < 3; ++k) s += Rm[a][k] * GR[1 + k][b];
        Gg[(1 + a) * 3 + b] = s;
      }
  } else {  // no-slip: momentum negated
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) Gg[(1 + a) * 3 + b] = -GR[1 + a][b];
  }
}

// state of an extended cell index (real cell or ghost)
V5 state_of(const orc_ctx& C, const double* Q, int e) {
  if (e < C.N) {
    V5 q;
    for (int v = 0; v < 5; ++v) q[v] = Q[(size_t)v * C.N + e];
    return q;
  }
  const Ghost& g = C.ghosts[e - C.N];
  V5 qo;
  for (int v = 0; v < 5; ++v) qo[v] = Q[(size_t)v * C.N + g.owner];
  return ghost_state(C, C.faces[g.face], qo);
}
void grad_of(const orc_ctx& C, const double* G, int e, double* out /*15*/) {
  if (e < C.N) {
    for (int k = 0; k < 15; ++k) out[k] = G[(size_t)k * C.N + e];
    return;
  }
  const Ghost& g = C.ghosts[e - C.N];
  double go[15];
  for (int k = 0; k < 15; ++k) go[k] = G[(size_t)k * C.N + g.owner];
  ghost_gradient(C.faces[g.face], go, out);
}

// ---------------------------------------------------------------------------
// characteristic projection (Sec. 5, characteristic variables): right
// eigenvectors of the x-split Euler flux Jacobian at Q*, reading A5 order
// (u-c, u, u, u, u+c)
// ---------------------------------------------------------------------------
void right_eigenvectors(const V5& qloc, double gamma, double R[5][5]) {
  Prim s = to_prim(qloc, gamma);
  double c = std::sqrt(gamma * s.p / s.rho);
  double H = (qloc[4] + s.p) / s.rho;
  double k2 = 0.5 * (s.U * s.U + s.V * s.V + s.W * s.W);
  double cols[5][5] = {{1.0, s.U - c, s.V, s.W, H - s.U * c},
                       {1.0, s.U, s.V, s.W, k2},
                       {0.0, 0.0, 1.0, 0.0, s.V},
                       {0.0, 0.0, 0.0, 1.0, s.W},
                       {1.0, s.U + c, s.V, s.W, H + s.U * c}};
  for (int r = 0; r < 5; ++r)
    for (int k = 0; k < 5; ++k) R[r][k] = cols[k][r];
}

void invert5(const double R[5][5], double Ri[5][5]) {
  std::vector<double> A(25), B(25, 0.0), X;
  for (int r = 0; r < 5; ++r)
    for (int c = 0; c < 5; ++c) A[r * 5 + c] = R[r][c];
  for (int r = 0; r < 5; ++r) B[r * 5 + r] = 1.0;
  gauss_solve(A, B, 5, 5, X);
  for (int r = 0; r < 5; ++r)
    for (int c = 0; c < 5; ++c) Ri[r][c] = X[r * 5 + c];
}

// ---------------------------------------------------------------------------
// reconstruction on one side of a face, literally in characteristic variables
// (Sec. 3.2-3.4 and Sec. 5): project all stencil data with R*^{-1}, fit P0 and
// P_m, compute beta_m and the WENO-Z type weights, evaluate Eq. (weno) at the
// Gauss points and project back.
// ---------------------------------------------------------------------------
struct Poly {           // one characteristic component
  double q0;            // cell average
  double a[9];          // P0: linear (3) and quadratic (xx,yy,zz,xy,xz,yz) in xi = (x-c)/h
  double b[8][3];       // P_m gradients (physical units); up to 8 sub-stencils (hexahedra)
  bool ok[8];
};

// mean over cell e of the scaled basis of cell i (xi = (x - c_i)/h_i)
void basis_means(const orc_ctx& C, int i, int e, double out[9]) {
  double h = C.hcell[i];
  V3 d = scl(1.0 / h, sub(C.c_of(e), C.cen[i]));
  const M33& Me = C.m2_of(e);
  const M33& Mi = C.m2[i];
  out[0] = d[0]; out[1] = d[1]; out[2] = d[2];
  const int pa[6] = {0, 1, 2, 0, 0, 1}, pb[6] = {0, 1, 2, 1, 2, 2};
  for (int k = 0; k < 6; ++k) {
    int a = pa[k], b = pb[k];
    out[3 + k] = (Me[a][b] + (C.c_of(e)[a] - C.cen[i][a]) * (C.c_of(e)[b] - C.cen[i][b]) - Mi[a][b]) / (h * h);
  }
}

// physical gradient of P0 at point x (for the 9-coefficient scaled basis)
V3 p0_grad(const orc_ctx& C, int i, const double a[9], const V3& x) {
  double h = C.hcell[i];
  V3 xi = scl(1.0 / h, sub(x, C.cen[i]));
  V3 g;
  g[0] = a[0] + 2.0 * a[3] * xi[0] + a[6] * xi[1] + a[7] * xi[2];
  g[1] = a[1] + 2.0 * a[4] * xi[1] + a[6] * xi[0] + a[8] * xi[2];
  g[2] = a[2] + 2.0 * a[5] * xi[2] + a[7] * xi[0] + a[8] * xi[1];
  return scl(1.0 / h, g);
}
double p0_value(const orc_ctx& C, int i, double q0, const double a[9], const V3& x) {
  double h = C.hcell[i];
  V3 xi = scl(1.0 / h, sub(x, C.cen[i]));
  const M33& M = C.m2[i];
  double hh = h * h;
  return q0 + a[0] * xi[0] + a[1] * xi[1] + a[2] * xi[2] +
         a[3] * (xi[0] * xi[0] - M[0][0] / hh) + a[4] * (xi[1] * xi[1] - M[1][1] / hh) +
         a[5] * (xi[2] * xi[2] - M[2][2] / hh) + a[6] * (xi[0] * xi[1] - M[0][1] / hh) +
         a[7] * (xi[0] * xi[2] - M[0][2] / hh) + a[8] * (xi[1] * xi[2] - M[1][2] / hh);
}

// smoothness indicator of P0 (Sec. 3.4), integrals over cell i written out
double beta_p0(const orc_ctx& C, int i, const double a[9]) {
  double vol = C.vol[i], h = C.hcell[i];
  const M33& M = C.m2[i];
  // first derivatives: d_k P0 = g_k + s_k . (x - c) (linear), so
  // int (d_k P0)^2 = vol (g_k^2 + s_k^T M2 s_k)
  double g[3] = {a[0] / h, a[1] / h, a[2] / h};
  double s[3][3] = {{2 * a[3], a[6], a[7]}, {a[6], 2 * a[4], a[8]}, {a[7], a[8], 2 * a[5]}};
  double first = 0.0;
  for (int k = 0; k < 3; ++k) {
    double sk[3] = {s[k][0] / (h * h), s[k][1] / (h * h), s[k][2] / (h * h)};
    double q = 0.0;
    for (int x = 0; x < 3; ++x)
      for (int y = 0; y < 3; ++y) q += sk[x] * M[x][y] * sk[y];
    first += vol * (g[k] * g[k] + q);
  }
  // second derivatives (each distinct multi-index once, reading A9)
  double d2[6] = {2 * a[3] / (h * h), 2 * a[4] / (h * h), 2 * a[5] / (h * h),
                  a[6] / (h * h), a[7] / (h * h), a[8] / (h * h)};
  double second = 0.0;
  for (int k = 0; k < 6; ++k) second += vol * d2[k] * d2[k];
  return std::pow(vol, 2.0 / 3.0 - 1.0) * first + std::pow(vol, 4.0 / 3.0 - 1.0) * second;
}
double beta_lin(const orc_ctx& C, int i, const double b[3]) {
  double vol = C.vol[i];
  return std::pow(vol, 2.0 / 3.0 - 1.0) * vol * (b[0] * b[0] + b[1] * b[1] + b[2] * b[2]);
}

void fit_subs(const orc_ctx& C, int i, const std::vector<int>& big, const std::vector<std::vector<int>>& subs,
              const std::vector<V5>& qs, Poly P[5]);

// Reading A36: a cell with two boundary faces whose planes meet at more than
// 45 degrees (a cell on an edge or at a corner of the boundary) takes the
// linear fit for P0.  With the quadratic fit there, the residual linearised
// at a uniform stream in a box or a channel has eigenvalues with positive real
// part, localised at those cells.
static bool edge_cell(const orc_ctx& C, int i) {
  const double c45 = std::sqrt(0.5);
  for (int p = 0; p < C.nf; ++p) {
    const Face& fp = C.faces[C.cf[i][p]];
    if (fp.R >= 0) continue;
    for (int q = 0; q < p; ++q) {
      const Face& fq = C.faces[C.cf[i][q]];
      if (fq.R < 0 && std::fabs(dot(fp.n, fq.n)) < c45) return true;
    }
  }
  return false;
}

// Non-compact WENO fits (Sec. 3.2): q[e] are projected averages keyed by
// position in the big stencil list.
void fit_weno(const orc_ctx& C, int i, const std::vector<int>& big,
              const std::vector<std::vector<int>>& subs, const std::vector<V5>& qs, Poly P[5]) {
  int m = (int)big.size() - 1;
  std::vector<double> A(m * 9), B(m * 5), X;
  for (int r = 0; r < m; ++r) {
    double row[9];
    basis_means(C, i, big[r + 1], row);
    for (int k = 0; k < 9; ++k) A[r * 9 + k] = row[k];
    for (int c = 0; c < 5; ++c) B[r * 5 + c] = qs[r + 1][c] - qs[0][c];
  }
  for (int c = 0; c < 5; ++c) P[c].q0 = qs[0][c];
  if (full_rank(A, m, 9) && !edge_cell(C, i)) {
    householder_lsq(A, B, m, 9, 5, X);
    for (int c = 0; c < 5; ++c)
      for (int k = 0; k < 9; ++k) P[c].a[k] = X[k * 5 + c];
  } else {  // readings A17 and A36: linear LS on the big stencil
    std::vector<double> A3(m * 3);
    for (int r = 0; r < m; ++r)
      for (int k = 0; k < 3; ++k) A3[r * 3 + k] = A[r * 9 + k];
    householder_lsq(A3, B, m, 3, 5, X);
    for (int c = 0; c < 5; ++c) {
      for (int k = 0; k < 9; ++k) P[c].a[k] = 0.0;
      for (int k = 0; k < 3; ++k) P[c].a[k] = X[k * 5 + c];
    }
  }
  fit_subs(C, i, big, subs, qs, P);
}

// Linear P_m of Sec. 3.2 on each sub-stencil by least squares on the cell
// averages of its members (positions looked up in the big stencil list);
// rank-deficient sub-stencils are marked unusable (reading A17).
void fit_subs(const orc_ctx& C, int i, const std::vector<int>& big, const std::vector<std::vector<int>>& subs,
              const std::vector<V5>& qs, Poly P[5]) {
  std::vector<double> X;
  for (int s = 0; s < (int)subs.size(); ++s) {
    const std::vector<int>& st = subs[s];
    int ms = (int)st.size() - 1;
    std::vector<double> As(std::max(ms, 0) * 3), Bs(std::max(ms, 0) * 5);
    for (int r = 0; r < ms; ++r) {
      double row[9];
      basis_means(C, i, st[r + 1], row);
      for (int k = 0; k < 3; ++k) As[r * 3 + k] = row[k];
      int pos = (int)(std::find(big.begin(), big.end(), st[r + 1]) - big.begin());
      for (int c = 0; c < 5; ++c) Bs[r * 5 + c] = qs[pos][c] - qs[0][c];
    }
    bool ok = ms >= 3 && full_rank(As, ms, 3);
    for (int c = 0; c < 5; ++c) P[c].ok[s] = ok;
    if (!ok) continue;
    householder_lsq(As, Bs, ms, 3, 5, X);
    double h = C.hcell[i];
    for (int c = 0; c < 5; ++c)
      for (int k = 0; k < 3; ++k) P[c].b[s][k] = X[k * 5 + c] / h;
  }
}

// Compact HWENO fits (Sec. 3.3): constrained least squares, averages exact,
// h-scaled averaged derivatives in the least-squares sense.
// qs[k] projected averages of stencil member k (self first), gs[k][c][d]
// projected averaged derivatives.
void fit_hweno(const orc_ctx& C, int i, const std::vector<int>& big,
               const std::vector<V5>& qs, const std::vector<std::array<V3, 5>>& gs, Poly P[5]) {
  int nn = (int)big.size() - 1;  // neighbours
  double hi = C.hcell[i];
  for (int c = 0; c < 5; ++c) P[c].q0 = qs[0][c];
  // P0: unknowns a[9]; equality rows: means over neighbours; LS rows:
  // h_k * mean_k(dP0/dx_d) = h_k (Q_d)_k for every member k and direction d.
  int ne = nn, nl = 3 * (nn + 1), nu = 9;
  for (int c = 0; c < 5; ++c) {
    std::vector<double> Ce(ne * nu), de(ne), Al(nl * nu), bl(nl);
    for (int r = 0; r < nn; ++r) {
      double row[9];
      basis_means(C, i, big[r + 1], row);
      for (int k = 0; k < 9; ++k) Ce[r * nu + k] = row[k];
      de[r] = qs[r + 1][c] - qs[0][c];
    }
    for (int k = 0; k <= nn; ++k) {
      int e = big[k];
      double hk = std::cbrt(C.vol_of(e));
      V3 d = scl(1.0 / hi, sub(C.c_of(e), C.cen[i]));
      // mean over cell e of d/dx_a of the basis, times h_i
      double rows[3][9] = {{1, 0, 0, 2 * d[0], 0, 0, d[1], d[2], 0},
                           {0, 1, 0, 0, 2 * d[1], 0, d[0], 0, d[2]},
                           {0, 0, 1, 0, 0, 2 * d[2], 0, d[0], d[1]}};
      for (int a = 0; a < 3; ++a) {
        for (int q = 0; q < 9; ++q) Al[(3 * k + a) * nu + q] = hk * rows[a][q] / hi;
        bl[3 * k + a] = hk * gs[k][c][a];
      }
    }
    // KKT: [2 Al^T Al, Ce^T; Ce, 0] [a; mu] = [2 Al^T bl; de]
    int n = nu + ne;
    std::vector<double> K(n * n, 0.0), rhs(n, 0.0), x;
    for (int p = 0; p < nu; ++p) {
      for (int q = 0; q < nu; ++q) {
        double s = 0.0;
        for (int r = 0; r < nl; ++r) s += Al[r * nu + p] * Al[r * nu + q];
        K[p * n + q] = 2.0 * s;
      }
      double s = 0.0;
      for (int r = 0; r < nl; ++r) s += Al[r * nu + p] * bl[r];
      rhs[p] = 2.0 * s;
      for (int r = 0; r < ne; ++r) {
        K[p * n + nu + r] = Ce[r * nu + p];
        K[(nu + r) * n + p] = Ce[r * nu + p];
      }
    }
    for (int r = 0; r < ne; ++r) rhs[nu + r] = de[r];
    gauss_solve(K, rhs, n, 1, x);
    for (int k = 0; k < 9; ++k) P[c].a[k] = x[k];
  }
  // P_m on {i, i_m}: minimise h_i^2|b - g_i|^2 + h_m^2|b - g_m|^2 subject to
  // b . (c_m - c_i) = q_m - q_i
  for (int s = 0; s < nn; ++s) {
    bool ok = true;
    for (int c = 0; c < 5; ++c) P[c].ok[s] = ok;
    if (!ok) continue;
    int e = big[s + 1];
    double hm = std::cbrt(C.vol_of(e));
    V3 d = sub(C.c_of(e), C.cen[i]);
    for (int c = 0; c < 5; ++c) {
      std::vector<double> K(16, 0.0), rhs(4), x;
      for (int a = 0; a < 3; ++a) {
        K[a * 4 + a] = 2.0 * (hi * hi + hm * hm);
        K[a * 4 + 3] = d[a];
        K[3 * 4 + a] = d[a];
        rhs[a] = 2.0 * (hi * hi * gs[0][c][a] + hm * hm * gs[s + 1][c][a]);
      }
      rhs[3] = qs[s + 1][c] - qs[0][c];
      gauss_solve(K, rhs, 4, 1, x);
      for (int a = 0; a < 3; ++a) P[c].b[s][a] = x[a];
    }
  }
}

}  // namespace

// Values and directional derivatives at the 3 Gauss points of face f on side
// s, local frame.  Returns 1 if the positivity fallback (reading A24) was used.
// If dbg is given, it receives per characteristic component c (64 doubles at
// dbg + 64 c): the cell average, the 9 coefficients of P0, the 8 x 3
// gradients of the P_m, their usable flags, beta_0 .. beta_8, tau_Z,
// omega_0 .. omega_8 and M; then R* and its inverse (25 + 25 doubles at
// dbg + 320).  Used by the tests that pin Sec. 3.4 and the projection.
static int side_values(const orc_ctx& C, const double* Q, const double* G, int fidx, int side,
                       double out[4][4][5], double* dbg = nullptr) {
  const Face& f = C.faces[fidx];
  int i = side == 0 ? f.L : f.R;
  int j = side == 0 ? (f.R >= 0 ? f.R : C.N + (-f.R - 1)) : f.L;
  V5 qi = state_of(C, Q, i), qj = state_of(C, Q, j);
  V5 qil = to_local(qi, f), qjl = to_local(qj, f);
  V5 qs_star;
  for (int v = 0; v < 5; ++v) qs_star[v] = 0.5 * (qil[v] + qjl[v]);
  double Rs[5][5], Ls[5][5];
  right_eigenvectors(qs_star, C.o.gamma, Rs);
  invert5(Rs, Ls);
  auto project = [&](const V5& qglob) {
    V5 ql = to_local(qglob, f), r{0, 0, 0, 0, 0};
    for (int c = 0; c < 5; ++c)
      for (int v = 0; v < 5; ++v) r[c] += Ls[c][v] * ql[v];
    return r;
  };
  bool compact = C.o.scheme == 1;
  const std::vector<int>& big = compact ? std::vector<int>() : C.big[i];
  std::vector<int> cbig;
  if (compact) {
    cbig.push_back(i);
    for (int p = 0; p < C.nf; ++p) cbig.push_back(C.nb[i][p]);
  }
  const std::vector<int>& st = compact ? cbig : big;
  std::vector<V5> qs(st.size());
  for (size_t k = 0; k < st.size(); ++k) qs[k] = project(state_of(C, Q, st[k]));
  Poly P[5];
  if (compact) {
    std::vector<std::array<V3, 5>> gs(st.size());
    for (size_t k = 0; k < st.size(); ++k) {
      double g15[15];
      grad_of(C, G, st[k], g15);
      // project each derivative direction like a state: (Q_d) -> R*^{-1} Rot Q_d
      for (int d = 0; d < 3; ++d) {
        V5 qd{g15[0 * 3 + d], g15[1 * 3 + d], g15[2 * 3 + d], g15[3 * 3 + d], g15[4 * 3 + d]};
        V5 pd = project(qd);
        for (int c = 0; c < 5; ++c) gs[k][c][d] = pd[c];
      }
    }
    fit_hweno(C, i, cbig, qs, gs, P);
    // hexahedra, compact sub-stencil option 1: P0 stays the compact fit, the
    // P_m are the averages-only fits on the eight S^WENO sub-stencils, whose
    // members are all face neighbours (Sec. 3.1; the sphere cases of Sec. 5)
    if (C.o.compact_subs == 1 && C.nf == 6) fit_subs(C, i, cbig, C.sub[i], qs, P);
  } else {
    fit_weno(C, i, big, C.sub[i], qs, P);
  }
  // weights and point values per characteristic component (Eq. (weno))
  const int nsub = compact && !(C.o.compact_subs == 1 && C.nf == 6) ? C.nf : (int)C.sub[i].size();
  const int ng = f.ng;
  double qv[4][4][5];
  for (int c = 0; c < 5; ++c) {
    int M = 0;
    for (int s = 0; s < nsub; ++s) M += P[c].ok[s] ? 1 : 0;
    double gm = C.o.gamma_lin, g0 = 1.0 - gm * M;
    double w[9];
    if (C.o.weights == 1) {
      w[0] = g0;
      for (int s = 0; s < nsub; ++s) w[s + 1] = P[c].ok[s] ? gm : 0.0;
    } else {
      double b0 = beta_p0(C, i, P[c].a), bm[8];
      double tz = 0.0;
      for (int s = 0; s < nsub; ++s)
        if (P[c].ok[s]) {
          bm[s] = beta_lin(C, i, P[c].b[s]);
          tz += std::fabs(b0 - bm[s]) / M;
        }
      double eps = C.o.weno_eps;
      double wt[9], sum = 0.0;
      wt[0] = g0 * (1.0 + tz / (b0 + eps));
      sum += wt[0];
      for (int s = 0; s < nsub; ++s) {
        wt[s + 1] = P[c].ok[s] ? gm * (1.0 + tz / (bm[s] + eps)) : 0.0;
        sum += wt[s + 1];
      }
      for (int k = 0; k <= nsub; ++k) w[k] = wt[k] / sum;
      if (dbg) {
        double* d = dbg + 64 * c;
        d[42] = b0;
        for (int s = 0; s < nsub; ++s) d[43 + s] = P[c].ok[s] ? bm[s] : 0.0;
        d[51] = tz;
      }
    }
    if (dbg) {
      double* d = dbg + 64 * c;
      d[0] = P[c].q0;
      for (int k = 0; k < 9; ++k) d[1 + k] = P[c].a[k];
      for (int s = 0; s < nsub; ++s) {
        for (int k = 0; k < 3; ++k) d[10 + 3 * s + k] = P[c].ok[s] ? P[c].b[s][k] : 0.0;
        d[34 + s] = P[c].ok[s] ? 1.0 : 0.0;
      }
      for (int k = 0; k <= nsub; ++k) d[52 + k] = w[k];
      d[61] = M;
    }
    for (int g = 0; g < ng; ++g) {
      const V3& x = f.gp[g];
      double val = w[0] / g0 * p0_value(C, i, P[c].q0, P[c].a, x);
      V3 grd = scl(w[0] / g0, p0_grad(C, i, P[c].a, x));
      for (int s = 0; s < nsub; ++s) {
        if (!P[c].ok[s]) continue;
        double coef = w[s + 1] - w[0] * gm / g0;
        V3 b{P[c].b[s][0], P[c].b[s][1], P[c].b[s][2]};
        val += coef * (P[c].q0 + dot(b, sub(x, C.cen[i])));
        grd = add(grd, scl(coef, b));
      }
      qv[g][0][c] = val;
      qv[g][1][c] = dot(grd, f.n);
      qv[g][2][c] = dot(grd, f.t1);
      qv[g][3][c] = dot(grd, f.t2);
    }
  }
  if (dbg)
    for (int r = 0; r < 5; ++r)
      for (int c = 0; c < 5; ++c) {
        dbg[320 + 5 * r + c] = Rs[r][c];
        dbg[345 + 5 * r + c] = Ls[r][c];
      }
  // back to conservative local-frame variables with R*
  for (int g = 0; g < ng; ++g)
    for (int d = 0; d < 4; ++d)
      for (int v = 0; v < 5; ++v) {
        double s = 0.0;
        for (int c = 0; c < 5; ++c) s += Rs[v][c] * qv[g][d][c];
        out[g][d][v] = s;
      }
  // positivity fallback (reading A24)
  bool bad = false;
  for (int g = 0; g < ng; ++g) {
    V5 w{out[g][0][0], out[g][0][1], out[g][0][2], out[g][0][3], out[g][0][4]};
    if (!physical(w, C.o.gamma)) bad = true;
  }
  if (bad) {
    for (int g = 0; g < ng; ++g) {
      for (int v = 0; v < 5; ++v) out[g][0][v] = qil[v];
      for (int d = 1; d < 4; ++d)
        for (int v = 0; v < 5; ++v) out[g][d][v] = 0.0;
    }
    return 1;
  }
  return 0;
}

// ---------------------------------------------------------------------------
// gas-kinetic flux at one Gauss point (Sec. 2 Eq. (flux) and Sec. 4 time
// average; Sec. 5 collision time; Prandtl fix of reading A19)
// ---------------------------------------------------------------------------
static void gks_point(const orc_ctx& C, const V5& Wl, const V5 dWl[3], const V5& Wr,
                      const V5 dWr[3], double dt, V5& F, V5* QG) {
  const double g = C.o.gamma, K = C.K;
  Prim l = to_prim(Wl, g), r = to_prim(Wr, g);
  Moments Mlh, Mrh, Mlf, Mrf, M0;
  Mlh.init(l.U, l.V, l.W, l.lam, K, +1);
  Mrh.init(r.U, r.V, r.W, r.lam, K, -1);
  Mlf.init(l.U, l.V, l.W, l.lam, K, 0);
  Mrf.init(r.U, r.V, r.W, r.lam, K, 0);
  // interface equilibrium from the compatibility condition
  V5 Q0;
  {
    V5 a = Mlh.psi(0, 0, 0, 0), b = Mrh.psi(0, 0, 0, 0);
    for (int k = 0; k < 5; ++k) Q0[k] = l.rho * a[k] + r.rho * b[k];
  }
  // vacuum interface (reading A34): the two half-space tails that reach the
  // point carry less than 2^-40 of the adjacent densities; no flux, no
  // point value
  if (!(Q0[0] > std::ldexp(1.0, -40) * (l.rho + r.rho))) {
    F = V5{0, 0, 0, 0, 0};
    if (QG) *QG = V5{0, 0, 0, 0, 0};
    return;
  }
  Prim z = to_prim(Q0, g);
  M0.init(z.U, z.V, z.W, z.lam, K, 0);
  // slopes of the initial distributions in the three local directions
  V5 al[3], ar[3], ab[3];
  V5 dWn{0, 0, 0, 0, 0};  // normal derivative of the interface state (for the heat flux)
  for (int d = 0; d < 3; ++d) {
    V5 bl, br;
    for (int k = 0; k < 5; ++k) {
      bl[k] = dWl[d][k] / l.rho;
      br[k] = dWr[d][k] / r.rho;
    }
    al[d] = slope_solve(Mlf, bl);
    ar[d] = slope_solve(Mrf, br);
    // equilibrium slopes from kinetic-weighted derivatives of Q0 (reading A6)
    V5 ql = Mlh.apsi(al[d], 0, 0, 0), qr = Mrh.apsi(ar[d], 0, 0, 0), b0;
    for (int k = 0; k < 5; ++k) b0[k] = (l.rho * ql[k] + r.rho * qr[k]) / z.rho;
    if (d == 0)
      for (int k = 0; k < 5; ++k) dWn[k] = l.rho * ql[k] + r.rho * qr[k];
    ab[d] = slope_solve(M0, b0);
  }
  // time derivatives from <a_1 u + a_2 v + a_3 w + A> = 0
  auto time_slope = [&](const Moments& M, const V5 a[3]) {
    V5 s{0, 0, 0, 0, 0};
    const int e[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    for (int d = 0; d < 3; ++d) {
      V5 t = M.apsi(a[d], e[d][0], e[d][1], e[d][2]);
      for (int k = 0; k < 5; ++k) s[k] -= t[k];
    }
    return slope_solve(M, s);
  };
  V5 Al = time_slope(Mlf, al), Ar = time_slope(Mrf, ar), Ab = time_slope(M0, ab);
  // collision time (Sec. 5)
  double jump = std::fabs((l.p - r.p) / (l.p + r.p));
  double tau = C.o.physics == 1 ? C.o.mu / z.p + C.o.tau_C * jump * dt
                                : C.o.tau_eps * dt + C.o.tau_C * jump * dt;
  // integrals over [0, dt] of the six time coefficients of Eq. (flux)
  double x = dt / tau, e = std::exp(-x), em1 = -std::expm1(-x);
  double T1 = dt - tau * em1;
  double T2 = -tau * dt + 2.0 * tau * tau * em1 - tau * dt * e;
  double T3 = 0.5 * dt * dt - tau * dt + tau * tau * em1;
  double T4 = tau * em1;
  double T5 = -2.0 * tau * tau * em1 + tau * dt * e;
  double T6 = -tau * tau * em1;
  // moment sum of f with an extra velocity weight u^k (k=1 flux, k=0 density)
  auto fmoment = [&](int k, const double c[6]) {
    V5 out{0, 0, 0, 0, 0};
    auto acc = [&](double s, const V5& t) {
      for (int q = 0; q < 5; ++q) out[q] += s * t[q];
    };
    const int e3[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    acc(z.rho * c[0], M0.psi(k, 0, 0, 0));
    for (int d = 0; d < 3; ++d) acc(z.rho * c[1], M0.apsi(ab[d], k + e3[d][0], e3[d][1], e3[d][2]));
    acc(z.rho * c[2], M0.apsi(Ab, k, 0, 0));
    acc(l.rho * c[3], Mlh.psi(k, 0, 0, 0));
    for (int d = 0; d < 3; ++d) acc(l.rho * c[4], Mlh.apsi(al[d], k + e3[d][0], e3[d][1], e3[d][2]));
    acc(l.rho * c[5], Mlh.apsi(Al, k, 0, 0));
    acc(r.rho * c[3], Mrh.psi(k, 0, 0, 0));
    for (int d = 0; d < 3; ++d) acc(r.rho * c[4], Mrh.apsi(ar[d], k + e3[d][0], e3[d][1], e3[d][2]));
    acc(r.rho * c[5], Mrh.apsi(Ar, k, 0, 0));
    return out;
  };
  double Tav[6] = {T1 / dt, T2 / dt, T3 / dt, T4 / dt, T5 / dt, T6 / dt};
  F = fmoment(1, Tav);
  if (C.o.physics == 1) {
    // Prandtl correction (reading A19): the BGK flux carries the heat flux of
    // Pr = 1, -mu c_p dT/dn; add (1/Pr - 1) times that Fourier flux, formed
    // from the normal derivative of the interface state (T = p / rho)
    const double u2 = z.U * z.U + z.V * z.V + z.W * z.W;
    const double dp = (g - 1.0) * (dWn[4] - (z.U * dWn[1] + z.V * dWn[2] + z.W * dWn[3]) + 0.5 * u2 * dWn[0]);
    const double dT = dp / z.rho - z.p * dWn[0] / (z.rho * z.rho);
    const double q = -C.o.mu * g / (g - 1.0) * dT;
    F[4] += (1.0 / C.o.prandtl - 1.0) * q;
  }
  if (QG) {
    // point value of Eq. (point) at t^n, the start of the local time
    // interval, as in the gradient update formula of Sec. 4.2 (reading A15')
    double t = 0.0;
    double et = std::exp(-t / tau), em1t = -std::expm1(-t / tau);
    double c[6] = {em1t, (t + tau) * et - tau, t - tau + tau * et, et, -(tau + t) * et, -tau * et};
    *QG = fmoment(0, c);
  }
}

// Right state and derivatives at a boundary Gauss point (reading A16), local frame.
static void boundary_right(const orc_ctx& C, const Face& f, const V5& Wl, const V5 dWl[3], V5& Wr,
                           V5 dWr[3]) {
  switch (f.kind) {
    case ORC_SLIP:
    case ORC_NOSLIP: {
      double Mv[5] = {1, -1, 1, 1, 1};
      if (f.kind == ORC_NOSLIP) Mv[2] = Mv[3] = -1;
      for (int k = 0; k < 5; ++k) {
        Wr[k] = Mv[k] * Wl[k];
        dWr[0][k] = -Mv[k] * dWl[0][k];
        dWr[1][k] = Mv[k] * dWl[1][k];
        dWr[2][k] = Mv[k] * dWl[2][k];
      }
      return;
    }
    case ORC_FARFIELD: {
      V3 nloc{1, 0, 0};
      V3 uinf_loc{dot(C.uinf, f.n), dot(C.uinf, f.t1), dot(C.uinf, f.t2)};
      Wr = farfield_state(C, Wl, nloc, uinf_loc);
      break;
    }
    case ORC_SUP_IN:
      Wr = to_local(C.qinf, f);
      break;
    case ORC_SUP_OUT:
      Wr = Wl;
      for (int d = 0; d < 3; ++d) dWr[d] = dWl[d];
      return;
  }
  for (int d = 0; d < 3; ++d) dWr[d] = V5{0, 0, 0, 0, 0};
}

// Face flux (global frame, integrated over the face, oriented L -> R) and the
// face sum of Gauss-point values for the gradient update.
// First-order kinetic flux vector splitting: free transport of the two
// half-space Maxwellians of the cell averages, F = rho_l <u psi>_{u>0} +
// rho_r <u psi>_{u<0} (no collision term, no slopes); the point value of the
// gradient update is rho_l <psi>_{u>0} + rho_r <psi>_{u<0}.
static void kfvs_point(const orc_ctx& C, const V5& Wl, const V5& Wr, V5& F, V5* QG) {
  const double g = C.o.gamma, K = C.K;
  Prim l = to_prim(Wl, g), r = to_prim(Wr, g);
  Moments Ml, Mr;
  Ml.init(l.U, l.V, l.W, l.lam, K, +1);
  Mr.init(r.U, r.V, r.W, r.lam, K, -1);
  V5 fl = Ml.psi(1, 0, 0, 0), fr = Mr.psi(1, 0, 0, 0);
  for (int k = 0; k < 5; ++k) F[k] = l.rho * fl[k] + r.rho * fr[k];
  if (QG) {
    V5 ql = Ml.psi(0, 0, 0, 0), qr = Mr.psi(0, 0, 0, 0);
    for (int k = 0; k < 5; ++k) (*QG)[k] = l.rho * ql[k] + r.rho * qr[k];
  }
}

static int face_flux(const orc_ctx& C, const double* Q, const double* G, const double* dt, int fidx,
                     V5& Fout, V5* QGout) {
  const Face& f = C.faces[fidx];
  if (C.o.first_order) {
    // the cell averages in the local frame; the right state of a boundary
    // face from the boundary condition
    V5 Wl = to_local(state_of(C, Q, f.L), f), Wr, dW0[3], dWr[3];
    for (int d = 0; d < 3; ++d) dW0[d] = {0, 0, 0, 0, 0};
    if (f.R < 0) {
      boundary_right(C, f, Wl, dW0, Wr, dWr);
    } else {
      Wr = to_local(state_of(C, Q, f.R), f);
    }
    V5 Fl, QGl;
    kfvs_point(C, Wl, Wr, Fl, QGout ? &QGl : nullptr);
    V5 Fg = to_global(Fl, f);
    for (int v = 0; v < 5; ++v) Fout[v] = f.S * Fg[v];
    if (QGout) {
      V5 Qg = to_global(QGl, f);
      for (int v = 0; v < 5; ++v) (*QGout)[v] = f.S * Qg[v];
    }
    return 0;
  }
  double sl[4][4][5], sr[4][4][5];
  int fb = side_values(C, Q, G, fidx, 0, sl);
  bool bnd = f.R < 0;
  if (!bnd) fb += side_values(C, Q, G, fidx, 1, sr);
  double dtf = bnd ? dt[f.L] : std::min(dt[f.L], dt[f.R]);
  // time interval of the flux average (reading A18'): the local time step at
  // CFL number cfl_flux; the implicit diagonal keeps the step at cfl
  if (C.o.cfl_flux > 0.0) dtf *= C.o.cfl_flux / C.o.cfl;
  V5 Fsum{0, 0, 0, 0, 0}, Qsum{0, 0, 0, 0, 0};
  for (int g = 0; g < f.ng; ++g) {
    V5 Wl, Wr, dWl[3], dWr[3];
    for (int v = 0; v < 5; ++v) {
      Wl[v] = sl[g][0][v];
      for (int d = 0; d < 3; ++d) dWl[d][v] = sl[g][1 + d][v];
    }
    if (bnd) {
      boundary_right(C, f, Wl, dWl, Wr, dWr);
    } else {
      for (int v = 0; v < 5; ++v) {
        Wr[v] = sr[g][0][v];
        for (int d = 0; d < 3; ++d) dWr[d][v] = sr[g][1 + d][v];
      }
    }
    V5 Fg, QGg;
    gks_point(C, Wl, dWl, Wr, dWr, dtf, Fg, QGout ? &QGg : nullptr);
    if (f.ng == 3) {
      for (int v = 0; v < 5; ++v) Fsum[v] += Fg[v] / 3.0;  // weights 1/3, reading A1
      if (QGout)
        for (int v = 0; v < 5; ++v) Qsum[v] += QGg[v] / 3.0;
    } else {
      for (int v = 0; v < 5; ++v) Fsum[v] += f.gw[g] * Fg[v];
      if (QGout)
        for (int v = 0; v < 5; ++v) Qsum[v] += f.gw[g] * QGg[v];
    }
  }
  V5 Fg = to_global(Fsum, f);
  for (int v = 0; v < 5; ++v) Fout[v] = f.S * Fg[v];
  if (QGout) {
    V5 Qg = to_global(Qsum, f);
    for (int v = 0; v < 5; ++v) (*QGout)[v] = f.S * Qg[v];
  }
  return fb;
}

static void compute_dt(const orc_ctx& C, const double* Q, double* dt) {
  // local time step, reading A18
  for (int i = 0; i < C.N; ++i) {
    V5 q;
    for (int v = 0; v < 5; ++v) q[v] = Q[(size_t)v * C.N + i];
    Prim s = to_prim(q, C.o.gamma);
    double c = std::sqrt(C.o.gamma * s.p / s.rho);
    double spd = std::sqrt(s.U * s.U + s.V * s.V + s.W * s.W);
    double nu = C.o.physics == 1 ? C.o.mu / s.rho : 0.0;
    dt[i] = C.o.cfl * C.hdt[i] / (spd + c + 2.0 * nu / C.hdt[i]);
  }
}

static int64_t residual(const orc_ctx& C, const double* Q, const double* G, const double* dt,
                        double* R, double* Gnew) {
  int F = (int)C.faces.size();
  std::vector<V5> FF(F), QQ(Gnew ? F : 0);
  int64_t fb = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : fb) num_threads(nthreads_req)
  for (int f = 0; f < F; ++f) fb += face_flux(C, Q, G, dt, f, FF[f], Gnew ? &QQ[f] : nullptr);
  // L(Q_i) = - sum over faces of the outward flux times area (Eq. (finite))
  for (int i = 0; i < C.N; ++i) {
    for (int v = 0; v < 5; ++v) R[(size_t)v * C.N + i] = 0.0;
    if (Gnew)
      for (int k = 0; k < 15; ++k) Gnew[(size_t)k * C.N + i] = 0.0;
    for (int p = 0; p < C.nf; ++p) {
      int fi = C.cf[i][p];
      const Face& f = C.faces[fi];
      double sg = f.L == i ? 1.0 : -1.0;
      for (int v = 0; v < 5; ++v) R[(size_t)v * C.N + i] -= sg * FF[fi][v];
      if (Gnew) {
        // Eq. (derivative): |Omega| grad Q = sum_f sum_G w_G Q_G n_out S
        for (int v = 0; v < 5; ++v)
          for (int d = 0; d < 3; ++d)
            Gnew[(size_t)(v * 3 + d) * C.N + i] += sg * QQ[fi][v] * f.n[d] / C.vol[i];
      }
    }
  }
  return fb;
}

// Euler flux Jacobian along n applied to x (the J of Eq. (deri-matrix))
static V5 euler_jn(double g, const V5& q, const V3& n, const V5& x) {
  double rho = q[0];
  V3 U{q[1] / rho, q[2] / rho, q[3] / rho};
  double p = (g - 1.0) * (q[4] - 0.5 * rho * dot(U, U));
  double un = dot(U, n);
  V3 dm{x[1], x[2], x[3]};
  double dun = (dot(dm, n) - un * x[0]) / rho;
  double dp = (g - 1.0) * (x[4] - dot(U, dm) + 0.5 * dot(U, U) * x[0]);
  V5 r;
  r[0] = dot(dm, n);
  for (int d = 0; d < 3; ++d) r[1 + d] = dm[d] * un + q[1 + d] * dun + dp * n[d];
  r[4] = (x[4] + dp) * un + (q[4] + p) * dun;
  return r;
}

// |lambda_f| = |U.n| + c from the mean of the two cells' primitives (A23)
static double face_lambda(const orc_ctx& C, const double* Q, int fidx) {
  const Face& f = C.faces[fidx];
  int j = f.R >= 0 ? f.R : C.N + (-f.R - 1);
  Prim a = to_prim(state_of(C, Q, f.L), C.o.gamma), b = to_prim(state_of(C, Q, j), C.o.gamma);
  double rho = 0.5 * (a.rho + b.rho), p = 0.5 * (a.p + b.p);
  V3 U{0.5 * (a.U + b.U), 0.5 * (a.V + b.V), 0.5 * (a.W + b.W)};
  return std::fabs(dot(U, f.n)) + std::sqrt(C.o.gamma * p / rho);
}

static void diag(const orc_ctx& C, const double* Q, const double* dt, double* D) {
  std::vector<double> lam(C.faces.size());
  for (size_t f = 0; f < C.faces.size(); ++f) lam[f] = face_lambda(C, Q, (int)f);
  for (int i = 0; i < C.N; ++i) {
    double s = C.vol[i] / dt[i];
    for (int p = 0; p < C.nf; ++p) s += 0.5 * lam[C.cf[i][p]] * C.faces[C.cf[i][p]].S;
    D[i] = s;
  }
}

// Jacobi iteration of Eq. (precond) with A = D + L + U from Eq. (deri-matrix)
static void precond(const orc_ctx& C, const double* Q, const double* dt, const double* r,
                    double* out) {
  int N = C.N;
  std::vector<double> D(N), lam(C.faces.size());
  diag(C, Q, dt, D.data());
  for (size_t f = 0; f < C.faces.size(); ++f) lam[f] = face_lambda(C, Q, (int)f);
  std::vector<double> b((size_t)5 * N), nb((size_t)5 * N);
  for (int i = 0; i < N; ++i)
    for (int v = 0; v < 5; ++v) b[(size_t)v * N + i] = r[(size_t)v * N + i] / D[i];
  for (int k = 0; k < C.o.jacobi_sweeps; ++k) {
    for (int i = 0; i < N; ++i) {
      V5 off{0, 0, 0, 0, 0};
      for (int p = 0; p < C.nf; ++p) {
        const Face& f = C.faces[C.cf[i][p]];
        if (f.R < 0) continue;  // boundary off-diagonal dropped (A23)
        int j = f.L == i ? f.R : f.L;
        V3 nout = f.L == i ? f.n : scl(-1.0, f.n);
        V5 qj, xj;
        for (int v = 0; v < 5; ++v) {
          qj[v] = Q[(size_t)v * N + j];
          xj[v] = b[(size_t)v * N + j];
        }
        V5 jx = euler_jn(C.o.gamma, qj, nout, xj);
        double l = lam[C.cf[i][p]];
        for (int v = 0; v < 5; ++v) off[v] += 0.5 * f.S * (jx[v] - l * xj[v]);
      }
      for (int v = 0; v < 5; ++v) nb[(size_t)v * N + i] = (r[(size_t)v * N + i] - off[v]) / D[i];
    }
    b.swap(nb);
  }
  std::copy(b.begin(), b.end(), out);
}

// A x with the approximate matrix of Eq. (deri-matrix): the diagonal D plus
// the off-diagonal blocks 1/2 S_f (J_n(Q_j) - |lambda_f| I) of interior faces
static void amatvec(const orc_ctx& C, const double* Q, const double* dt, const double* x, double* out) {
  int N = C.N;
  std::vector<double> D(N), lam(C.faces.size());
  diag(C, Q, dt, D.data());
  for (size_t f = 0; f < C.faces.size(); ++f) lam[f] = face_lambda(C, Q, (int)f);
  for (int i = 0; i < N; ++i) {
    V5 acc;
    for (int v = 0; v < 5; ++v) acc[v] = D[i] * x[(size_t)v * N + i];
    for (int p = 0; p < C.nf; ++p) {
      const Face& f = C.faces[C.cf[i][p]];
      if (f.R < 0) continue;  // boundary off-diagonal dropped (A23)
      int j = f.L == i ? f.R : f.L;
      V3 nout = f.L == i ? f.n : scl(-1.0, f.n);
      V5 qj, xj;
      for (int v = 0; v < 5; ++v) {
        qj[v] = Q[(size_t)v * N + j];
        xj[v] = x[(size_t)v * N + j];
      }
      V5 jx = euler_jn(C.o.gamma, qj, nout, xj);
      double l = lam[C.cf[i][p]];
      for (int v = 0; v < 5; ++v) acc[v] += 0.5 * f.S * (jx[v] - l * xj[v]);
    }
    for (int v = 0; v < 5; ++v) out[(size_t)v * N + i] = acc[v];
  }
}

// Greedy colouring of the face-neighbour graph: cells in index order, each
// takes the smallest colour that none of its already coloured neighbours has.
// Cells of one colour share no face, so a Gauss-Seidel sweep may update a
// whole colour at once.
static int colour_cells(const orc_ctx& C, std::vector<int>& col) {
  col.assign(C.N, -1);
  int ncol = 0;
  for (int i = 0; i < C.N; ++i) {
    bool used[8] = {false, false, false, false, false, false, false, false};
    for (int p = 0; p < C.nf; ++p) {
      const Face& f = C.faces[C.cf[i][p]];
      if (f.R < 0) continue;
      int j = f.L == i ? f.R : f.L;
      if (col[j] >= 0) used[col[j]] = true;
    }
    int c = 0;
    while (used[c]) ++c;  // at most 4 neighbours: c <= 4
    col[i] = c;
    ncol = std::max(ncol, c + 1);
  }
  return ncol;
}

// LU-SGS of the approximate matrix A = D + L + U of Eq. (deri-matrix) (the
// factorisation of Jameson and Yoon on an unstructured mesh, the LUSGS-WENO
// solver the paper compares with in Sec. 5):
//   (D + L) D^-1 (D + U) dQ = R,
// L holding the off-diagonal blocks 1/2 S_f (J_n(Q_j) - |lambda_f| I) to the
// neighbours j of lower colour, U those of higher colour.  Forward sweep:
// (D + L) y = R in increasing colour; backward sweep: (D + U) dQ = D y in
// decreasing colour, dQ_i = y_i - D_i^-1 (U dQ)_i.
static void lusgs(const orc_ctx& C, const double* Q, const double* dt, const double* R, double* dQ) {
  const int N = C.N;
  std::vector<double> D(N), lam(C.faces.size()), y((size_t)5 * N);
  diag(C, Q, dt, D.data());
  for (size_t f = 0; f < C.faces.size(); ++f) lam[f] = face_lambda(C, Q, (int)f);
  std::vector<int> col;
  colour_cells(C, col);
  std::vector<int> order(N);
  for (int i = 0; i < N; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return col[a] < col[b]; });
  // sum over the neighbours j with lower (sgn < 0) or higher (sgn > 0) colour
  auto offdiag = [&](int i, const std::vector<double>& x, int sgn) {
    V5 off{0, 0, 0, 0, 0};
    for (int p = 0; p < C.nf; ++p) {
      const Face& f = C.faces[C.cf[i][p]];
      if (f.R < 0) continue;  // boundary off-diagonal dropped, as in A
      int j = f.L == i ? f.R : f.L;
      if ((sgn < 0) != (col[j] < col[i])) continue;
      V3 nout = f.L == i ? f.n : scl(-1.0, f.n);
      V5 qj, xj;
      for (int v = 0; v < 5; ++v) {
        qj[v] = Q[(size_t)v * N + j];
        xj[v] = x[(size_t)v * N + j];
      }
      V5 jx = euler_jn(C.o.gamma, qj, nout, xj);
      double l = lam[C.cf[i][p]];
      for (int v = 0; v < 5; ++v) off[v] += 0.5 * f.S * (jx[v] - l * xj[v]);
    }
    return off;
  };
  for (int k = 0; k < N; ++k) {
    int i = order[k];
    V5 off = offdiag(i, y, -1);
    for (int v = 0; v < 5; ++v) y[(size_t)v * N + i] = (R[(size_t)v * N + i] - off[v]) / D[i];
  }
  std::vector<double> x((size_t)5 * N, 0.0);
  for (int k = N - 1; k >= 0; --k) {
    int i = order[k];
    V5 off = offdiag(i, x, +1);
    for (int v = 0; v < 5; ++v) x[(size_t)v * N + i] = y[(size_t)v * N + i] - off[v] / D[i];
  }
  std::copy(x.begin(), x.end(), dQ);
}

static double rms(const double* x, size_t n) {
  double s = 0.0;
  for (size_t k = 0; k < n; ++k) s += x[k] * x[k];
  return std::sqrt(s / (double)n);
}

// matrix-free product of Eq. (frechet); sigma rule of reading A22
static double jv(const orc_ctx& C, const double* Q, const double* G, const double* dt,
                 const double* b, const double* v, double sigma, double* Av) {
  size_t n = (size_t)5 * C.N;
  double rv = rms(v, n);
  if (rv == 0.0) {
    std::fill(Av, Av + n, 0.0);
    return 0.0;
  }
  if (sigma <= 0.0) sigma = std::sqrt(std::ldexp(1.0, -52)) * std::max(1.0, rms(Q, n)) / rv;
  std::vector<double> Qp(n), Rp(n);
  for (size_t k = 0; k < n; ++k) Qp[k] = Q[k] + sigma * v[k];
  residual(C, Qp.data(), G, dt, Rp.data(), nullptr);
  for (int i = 0; i < C.N; ++i)
    for (int q = 0; q < 5; ++q) {
      size_t k = (size_t)q * C.N + i;
      Av[k] = C.vol[i] / dt[i] * v[k] - (Rp[k] - b[k]) / sigma;
    }
  return sigma;
}

static double res_norm(const orc_ctx& C, const double* R) {
  double s = 0.0, v = 0.0;
  for (int i = 0; i < C.N; ++i) {
    s += std::fabs(R[i]);
    v += C.vol[i];
  }
  return s / v;
}

// Boundary matching, ghost cells, length scales and stencils, common to both
// cell shapes.  open: faces seen once, keyed by their sorted node ids.
template <typename Key>
static bool finish_mesh(orc_ctx& C, std::map<Key, int>& open, int64_t n_bf, const int32_t* bf,
                        const int32_t* btag, int32_t n_tags, const int32_t* kind_of_tag) {
  const int N = C.N, nv = (int)std::tuple_size<Key>::value;
  std::map<Key, int> btags;
  for (int64_t k = 0; k < n_bf; ++k) {
    Key key;
    for (int q = 0; q < nv; ++q) key[q] = bf[nv * k + q];
    std::sort(key.begin(), key.end());
    btags[key] = btag[k];
  }
  if ((int64_t)open.size() != n_bf) {
    g_err = "boundary face count mismatch";
    return false;
  }
  for (auto& kv : open) {
    auto bt = btags.find(kv.first);
    if (bt == btags.end() || bt->second < 0 || bt->second >= n_tags) {
      g_err = "unmatched boundary face";
      return false;
    }
    Face& f = C.faces[kv.second];
    f.kind = kind_of_tag[bt->second];
    int gid = (int)C.ghosts.size();
    f.R = -gid - 1;
    Ghost g;
    g.owner = f.L;
    g.face = kv.second;
    // mirror image of the owner across the face plane (reading A16)
    V3 cl = C.cen[f.L];
    g.c = sub(cl, scl(2.0 * dot(sub(cl, f.xc), f.n), f.n));
    double Rm[3][3];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) Rm[a][b] = (a == b ? 1.0 : 0.0) - 2.0 * f.n[a] * f.n[b];
    M33 m{};
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b)
        for (int x = 0; x < 3; ++x)
          for (int y = 0; y < 3; ++y) m[a][b] += Rm[a][x] * C.m2[f.L][x][y] * Rm[y][b];
    g.m2 = m;
    g.vol = C.vol[f.L];
    C.ghosts.push_back(g);
    C.nb[f.L][f.pL] = N + gid;
  }
  // length scales: h = |Omega|^(1/3); time-step length 3|Omega|/max S for a
  // tetrahedron (its height), |Omega|/max S for a hexahedron (its width),
  // readings A18 and A31
  C.hcell.resize(N);
  C.hdt.resize(N);
  for (int i = 0; i < N; ++i) {
    C.hcell[i] = std::cbrt(C.vol[i]);
    double smax = 0.0;
    for (int p = 0; p < C.nf; ++p) smax = std::max(smax, C.faces[C.cf[i][p]].S);
    C.hdt[i] = (C.nf == 4 ? 3.0 : 1.0) * C.vol[i] / smax;
  }
  // stencils (Sec. 3.1, reading A13)
  C.big.resize(N);
  C.sub.resize(N);
  auto push_unique = [](std::vector<int>& v, int e) {
    if (std::find(v.begin(), v.end(), e) == v.end()) v.push_back(e);
  };
  for (int i = 0; i < N; ++i) {
    std::vector<int>& b = C.big[i];
    b.push_back(i);
    for (int p = 0; p < C.nf; ++p) push_unique(b, C.nb[i][p]);
    for (int p = 0; p < C.nf; ++p) {
      int j = C.nb[i][p];
      if (j >= N) continue;  // ghosts have no neighbours
      for (int q = 0; q < C.nf; ++q)
        if (C.nb[j][q] != i) push_unique(b, C.nb[j][q]);
    }
    if (C.nf == 4) {
      // S_i1 = {i, i1, i2, i3, nbrs of i1}, S_i2 = {i, i1, i2, i4, nbrs of i2},
      // S_i3 = {i, i2, i3, i4, nbrs of i3}, S_i4 = {i, i3, i1, i4, nbrs of i4}
      const int first[4][3] = {{0, 1, 2}, {0, 1, 3}, {1, 2, 3}, {2, 0, 3}};
      C.sub[i].assign(4, {});
      for (int m = 0; m < 4; ++m) {
        std::vector<int>& st = C.sub[i][m];
        st.push_back(i);
        for (int k = 0; k < 3; ++k) push_unique(st, C.nb[i][first[m][k]]);
        int j = C.nb[i][m];
        if (j < N)
          for (int q = 0; q < 4; ++q)
            if (C.nb[j][q] != i) push_unique(st, C.nb[j][q]);
      }
    } else {
      // hexahedron, faces F1..F6 = local faces 0..5 (F1, F6 opposite, F2..F5
      // around in order): S_m = {i, i1 or i6, two consecutive lateral
      // neighbours}, m = 1..8 (Sec. 3.1)
      const int lat[5] = {1, 2, 3, 4, 1};
      C.sub[i].assign(8, {});
      for (int m = 0; m < 8; ++m) {
        std::vector<int>& st = C.sub[i][m];
        st.push_back(i);
        push_unique(st, C.nb[i][m < 4 ? 0 : 5]);
        push_unique(st, C.nb[i][lat[m % 4]]);
        push_unique(st, C.nb[i][lat[m % 4 + 1]]);
      }
    }
  }
  return true;
}

static bool build(orc_ctx& C, int64_t n_nodes, const double* xyz, int64_t n_tets,
                  const int32_t* tets, int64_t n_bf, const int32_t* bf, const int32_t* btag,
                  int32_t n_tags, const int32_t* kind_of_tag) {
  int N = (int)n_tets;
  C.N = N;
  C.nf = 4;
  auto X = [&](int node) { return V3{xyz[3 * node], xyz[3 * node + 1], xyz[3 * node + 2]}; };
  C.vol.resize(N);
  C.cen.resize(N);
  C.m2.resize(N);
  for (int i = 0; i < N; ++i) {
    V3 v[4];
    for (int k = 0; k < 4; ++k) {
      int nd = tets[4 * i + k];
      if (nd < 0 || nd >= n_nodes) {
        g_err = "tet node index out of range";
        return false;
      }
      v[k] = X(nd);
    }
    double vol6 = dot(cross(sub(v[1], v[0]), sub(v[2], v[0])), sub(v[3], v[0]));
    if (!(vol6 > 0.0)) {
      g_err = "inverted or degenerate tetrahedron " + std::to_string(i);
      return false;
    }
    C.vol[i] = vol6 / 6.0;
    V3 c{0, 0, 0};
    for (int k = 0; k < 4; ++k) c = add(c, scl(0.25, v[k]));
    C.cen[i] = c;
    // second central moment per unit volume of a simplex: (1/20) sum (v-c)(v-c)^T
    M33 m{};
    for (int k = 0; k < 4; ++k) {
      V3 d = sub(v[k], c);
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) m[a][b] += d[a] * d[b] / 20.0;
    }
    C.m2[i] = m;
  }
  // faces: local face p is opposite local vertex p (reading A13)
  std::map<std::array<int, 3>, int> open;
  C.cf.assign(N, {-1, -1, -1, -1, -1, -1});
  C.nb.assign(N, {-1, -1, -1, -1, -1, -1});
  for (int i = 0; i < N; ++i)
    for (int p = 0; p < 4; ++p) {
      std::array<int, 3> nodes;
      int q = 0;
      for (int k = 0; k < 4; ++k)
        if (k != p) nodes[q++] = tets[4 * i + k];
      std::array<int, 3> key = nodes;
      std::sort(key.begin(), key.end());
      auto it = open.find(key);
      if (it == open.end()) {
        Face f;
        f.L = i;
        f.pL = p;
        V3 a = X(nodes[0]), b = X(nodes[1]), c = X(nodes[2]);
        V3 nn = cross(sub(b, a), sub(c, a));
        f.S = 0.5 * norm(nn);
        f.n = scl(1.0 / norm(nn), nn);
        f.xc = scl(1.0 / 3.0, add(add(a, b), c));
        if (dot(f.n, sub(f.xc, C.cen[i])) < 0) f.n = scl(-1.0, f.n);
        tangents(f.n, f.t1, f.t2);
        // 3-point degree-2 rule, barycentric (2/3, 1/6, 1/6), reading A1
        V3 P[3] = {a, b, c};
        f.ng = 3;
        for (int g = 0; g < 3; ++g) {
          f.gp[g] = add(scl(2.0 / 3.0, P[g]), scl(1.0 / 6.0, add(P[(g + 1) % 3], P[(g + 2) % 3])));
          f.gw[g] = 1.0 / 3.0;
        }
        open[key] = (int)C.faces.size();
        C.cf[i][p] = (int)C.faces.size();
        C.faces.push_back(f);
      } else {
        Face& f = C.faces[it->second];
        if (f.R >= 0) {
          g_err = "non-manifold face";
          return false;
        }
        f.R = i;
        f.pR = p;
        C.cf[i][p] = it->second;
        C.nb[i][p] = f.L;
        C.nb[f.L][f.pL] = i;
        open.erase(it);
      }
    }
  return finish_mesh(C, open, n_bf, bf, btag, n_tags, kind_of_tag);
}

// Hexahedral cells (nodes in the usual order: 0-3 the bottom quadrilateral
// counter-clockwise seen from above, 4-7 the top one above them), mapped
// trilinearly from the unit cube.  Cell integrals use the 3-point
// Gauss-Legendre rule per direction, which is exact for the volume, the
// centroid and the second moments of a trilinear cell (integrands of degree
// <= 4 per reference direction).  Faces are the bilinear quadrilaterals; the
// face vector area is exact, (x_c - x_a) x (x_d - x_b) / 2, and its 2x2
// Gauss points carry weights proportional to the normal component of the
// area element (they sum to one exactly) -- reading A30.
static bool build_hex(orc_ctx& C, int64_t n_nodes, const double* xyz, int64_t n_hex,
                      const int32_t* hexes, int64_t n_bf, const int32_t* bf, const int32_t* btag,
                      int32_t n_tags, const int32_t* kind_of_tag) {
  const int N = (int)n_hex;
  C.N = N;
  C.nf = 6;
  auto X = [&](int node) { return V3{xyz[3 * node], xyz[3 * node + 1], xyz[3 * node + 2]}; };
  // reference corners (r, s, t) of the node order
  const int rc[8][3] = {{0, 0, 0}, {1, 0, 0}, {1, 1, 0}, {0, 1, 0}, {0, 0, 1}, {1, 0, 1}, {1, 1, 1}, {0, 1, 1}};
  const double gx[3] = {0.5 - 0.5 * std::sqrt(0.6), 0.5, 0.5 + 0.5 * std::sqrt(0.6)};
  const double gw3[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};
  C.vol.resize(N);
  C.cen.resize(N);
  C.m2.resize(N);
  for (int i = 0; i < N; ++i) {
    V3 v[8];
    for (int k = 0; k < 8; ++k) {
      int nd = hexes[8 * i + k];
      if (nd < 0 || nd >= n_nodes) {
        g_err = "hex node index out of range";
        return false;
      }
      v[k] = X(nd);
    }
    // position and Jacobian of the trilinear map at (r, s, t)
    auto map = [&](double r, double s, double t, V3& x, double& J) {
      V3 dr{0, 0, 0}, ds{0, 0, 0}, dt{0, 0, 0};
      x = {0, 0, 0};
      for (int k = 0; k < 8; ++k) {
        double fr = rc[k][0] ? r : 1.0 - r, fs = rc[k][1] ? s : 1.0 - s, ft = rc[k][2] ? t : 1.0 - t;
        double sr = rc[k][0] ? 1.0 : -1.0, ss = rc[k][1] ? 1.0 : -1.0, st = rc[k][2] ? 1.0 : -1.0;
        x = add(x, scl(fr * fs * ft, v[k]));
        dr = add(dr, scl(sr * fs * ft, v[k]));
        ds = add(ds, scl(fr * ss * ft, v[k]));
        dt = add(dt, scl(fr * fs * st, v[k]));
      }
      J = dot(cross(dr, ds), dt);
    };
    // a valid cell has a positive Jacobian at its corners and Gauss points
    bool ok = true;
    for (int k = 0; k < 8 && ok; ++k) {
      V3 x;
      double J;
      map(rc[k][0], rc[k][1], rc[k][2], x, J);
      ok = J > 0.0 && std::isfinite(J);
    }
    double vol = 0.0;
    V3 c{0, 0, 0};
    std::vector<std::pair<V3, double>> pts;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b)
        for (int d = 0; d < 3; ++d) {
          V3 x;
          double J;
          map(gx[a], gx[b], gx[d], x, J);
          if (!(J > 0.0)) ok = false;
          double w = gw3[a] * gw3[b] * gw3[d] * J;
          pts.push_back({x, w});
          vol += w;
          c = add(c, scl(w, x));
        }
    if (!ok) {
      g_err = "inverted or degenerate hexahedron " + std::to_string(i);
      return false;
    }
    c = scl(1.0 / vol, c);
    M33 m{};
    for (auto& pw : pts) {
      V3 d = sub(pw.first, c);
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) m[a][b] += pw.second * d[a] * d[b] / vol;
    }
    C.vol[i] = vol;
    C.cen[i] = c;
    C.m2[i] = m;
  }
  // local faces F1..F6 = 0..5: bottom, the four sides in order around, top;
  // node lists counter-clockwise seen from outside
  const int fn[6][4] = {{0, 3, 2, 1}, {0, 1, 5, 4}, {1, 2, 6, 5}, {2, 3, 7, 6}, {3, 0, 4, 7}, {4, 5, 6, 7}};
  const double q0 = 0.5 - 0.5 / std::sqrt(3.0), q1 = 0.5 + 0.5 / std::sqrt(3.0);
  const double quv[4][2] = {{q0, q0}, {q1, q0}, {q1, q1}, {q0, q1}};
  std::map<std::array<int, 4>, int> open;
  C.cf.assign(N, {-1, -1, -1, -1, -1, -1});
  C.nb.assign(N, {-1, -1, -1, -1, -1, -1});
  for (int i = 0; i < N; ++i)
    for (int p = 0; p < 6; ++p) {
      std::array<int, 4> nodes;
      for (int k = 0; k < 4; ++k) nodes[k] = hexes[8 * i + fn[p][k]];
      std::array<int, 4> key = nodes;
      std::sort(key.begin(), key.end());
      auto it = open.find(key);
      if (it == open.end()) {
        Face f;
        f.L = i;
        f.pL = p;
        V3 a = X(nodes[0]), b = X(nodes[1]), c = X(nodes[2]), d = X(nodes[3]);
        V3 sv = scl(0.5, cross(sub(c, a), sub(d, b)));
        f.S = norm(sv);
        if (!(f.S > 0.0)) {
          g_err = "degenerate quadrilateral face of hexahedron " + std::to_string(i);
          return false;
        }
        f.n = scl(1.0 / f.S, sv);
        f.ng = 4;
        V3 xc{0, 0, 0};
        for (int g = 0; g < 4; ++g) {
          double u = quv[g][0], w = quv[g][1];
          f.gp[g] = add(add(scl((1 - u) * (1 - w), a), scl(u * (1 - w), b)), add(scl(u * w, c), scl((1 - u) * w, d)));
          V3 xu = add(scl(1 - w, sub(b, a)), scl(w, sub(c, d)));
          V3 xw = add(scl(1 - u, sub(d, a)), scl(u, sub(c, b)));
          f.gw[g] = 0.25 * dot(cross(xu, xw), f.n) / f.S;
          xc = add(xc, scl(f.gw[g], f.gp[g]));
        }
        f.xc = xc;
        if (dot(f.n, sub(f.xc, C.cen[i])) < 0) {
          g_err = "face normal does not point out of hexahedron " + std::to_string(i);
          return false;
        }
        tangents(f.n, f.t1, f.t2);
        open[key] = (int)C.faces.size();
        C.cf[i][p] = (int)C.faces.size();
        C.faces.push_back(f);
      } else {
        Face& f = C.faces[it->second];
        if (f.R >= 0) {
          g_err = "non-manifold face";
          return false;
        }
        f.R = i;
        f.pR = p;
        C.cf[i][p] = it->second;
        C.nb[i][p] = f.L;
        C.nb[f.L][f.pL] = i;
        open.erase(it);
      }
    }
  return finish_mesh(C, open, n_bf, bf, btag, n_tags, kind_of_tag);
}

// Q^{n+1} = Q^n + dQ.  With max_update = theta > 0 (a runtime policy of the
// library for impulsive starts, not in the paper) each cell's change is
// scaled by the largest alpha = 2^-k, k = 0..20, for which its density and
// pressure change by at most theta of their old values; a state with
// L(Q) = 0 is a fixed point either way.  Returns the number of scaled cells.
static int64_t apply_update(const orc_ctx& C, double* Q, const double* dQ) {
  const int N = C.N;
  const double th = C.o.max_update, g = C.o.gamma;
  int64_t limited = 0;
  for (int i = 0; i < N; ++i) {
    V5 q, d;
    for (int v = 0; v < 5; ++v) {
      q[v] = Q[(size_t)v * N + i];
      d[v] = dQ[(size_t)v * N + i];
    }
    double alpha = 1.0;
    if (th > 0.0) {
      const double p0 = to_prim(q, g).p;
      for (int k = 0; k <= 20; ++k) {
        V5 qn;
        for (int v = 0; v < 5; ++v) qn[v] = q[v] + alpha * d[v];
        const double pn = (g - 1.0) * (qn[4] - 0.5 * (qn[1] * qn[1] + qn[2] * qn[2] + qn[3] * qn[3]) / qn[0]);
        if (std::fabs(qn[0] - q[0]) <= th * q[0] && std::fabs(pn - p0) <= th * p0) break;
        if (k == 20) break;
        alpha *= 0.5;
      }
      if (alpha < 1.0) ++limited;
    }
    for (int v = 0; v < 5; ++v) Q[(size_t)v * N + i] = q[v] + alpha * d[v];
  }
  return limited;
}

// ---------------------------------------------------------------------------
// GMRES (Algorithm 1): left-preconditioned, restarted, MGS Arnoldi, Givens QR
// ---------------------------------------------------------------------------
// the gradients after a step: G_new of Sec. 4.2, or with grad_relax = omega < 1
// the relaxed G + omega (G_new - G) (the same fixed point)
static void relax_gradients(const orc_ctx& C, const std::vector<double>& Gn, double* G) {
  const double w = C.o.grad_relax;
  for (size_t k = 0; k < Gn.size(); ++k) G[k] = w >= 1.0 ? Gn[k] : G[k] + w * (Gn[k] - G[k]);
}

static int implicit_step(const orc_ctx& C, double* Q, double* G, orc_step_info* info) {
  int N = C.N;
  size_t n = (size_t)5 * N;
  std::vector<double> dt(N), b(n), Gn(C.o.scheme == 1 ? (size_t)15 * N : 0);
  compute_dt(C, Q, dt.data());
  int64_t evals = 0, fb = 0;
  fb += residual(C, Q, G, dt.data(), b.data(), C.o.scheme == 1 ? Gn.data() : nullptr);
  ++evals;
  info->res = res_norm(C, b.data());
  if (C.o.solver == 1) {
    // one LU-SGS solve of the approximate system per step
    std::vector<double> dQ(n);
    lusgs(C, Q, dt.data(), b.data(), dQ.data());
    info->n_limited = apply_update(C, Q, dQ.data());
    if (C.o.scheme == 1) relax_gradients(C, Gn, G);
    info->gmres_rel = 0.0;
    info->n_resid_evals = evals;
    info->n_fallbacks = fb;
    for (int i = 0; i < N; ++i) {
      V5 q;
      for (int v = 0; v < 5; ++v) q[v] = Q[(size_t)v * N + i];
      if (!physical(q, C.o.gamma)) return -4;
    }
    return 0;
  }
  int m = C.o.krylov_dim;
  std::vector<double> dQ(n, 0.0), r(n), rh(n), w(n), y(n);
  std::vector<std::vector<double>> V(m + 1, std::vector<double>(n));
  double beta0 = -1.0, last = 0.0;
  auto dotv = [&](const std::vector<double>& a, const std::vector<double>& c) {
    double s = 0.0;
    for (size_t k = 0; k < n; ++k) s += a[k] * c[k];
    return s;
  };
  for (int rs = 0; rs < C.o.restarts; ++rs) {
    if (rs == 0) {
      r = b;  // Delta Q^(0) = 0
    } else {
      if (C.o.jv_mode == 1) {
        amatvec(C, Q, dt.data(), dQ.data(), y.data());
      } else {
        jv(C, Q, G, dt.data(), b.data(), dQ.data(), C.o.fd_sigma, y.data());
        ++evals;
      }
      for (size_t k = 0; k < n; ++k) r[k] = b[k] - y[k];
    }
    precond(C, Q, dt.data(), r.data(), rh.data());
    double beta = std::sqrt(dotv(rh, rh));
    if (beta0 < 0) beta0 = beta;
    if (beta == 0.0) break;
    for (size_t k = 0; k < n; ++k) V[0][k] = rh[k] / beta;
    std::vector<double> H((m + 1) * m, 0.0), cs(m), sn(m), gvec(m + 1, 0.0);
    gvec[0] = beta;
    int jdone = 0;
    for (int j = 0; j < m; ++j) {
      if (C.o.jv_mode == 1) {
        amatvec(C, Q, dt.data(), V[j].data(), y.data());
      } else {
        jv(C, Q, G, dt.data(), b.data(), V[j].data(), C.o.fd_sigma, y.data());
        ++evals;
      }
      precond(C, Q, dt.data(), y.data(), w.data());
      for (int i = 0; i <= j; ++i) {
        double h = dotv(w, V[i]);
        H[i * m + j] = h;
        for (size_t k = 0; k < n; ++k) w[k] -= h * V[i][k];
      }
      double hn = std::sqrt(dotv(w, w));
      H[(j + 1) * m + j] = hn;
      // norm of the preconditioned product before orthogonalisation, from the
      // raw column (h_0j, ..., h_jj, h_j+1,j), for the breakdown test below
      double col2 = 0.0;
      for (int i = 0; i <= j + 1; ++i) col2 += H[i * m + j] * H[i * m + j];
      // Givens rotations on the new column
      for (int i = 0; i < j; ++i) {
        double a = H[i * m + j], c = H[(i + 1) * m + j];
        H[i * m + j] = cs[i] * a + sn[i] * c;
        H[(i + 1) * m + j] = -sn[i] * a + cs[i] * c;
      }
      double a = H[j * m + j], c = H[(j + 1) * m + j];
      double rr = std::hypot(a, c);
      cs[j] = a / rr;
      sn[j] = c / rr;
      H[j * m + j] = rr;
      H[(j + 1) * m + j] = 0.0;
      gvec[j + 1] = -sn[j] * gvec[j];
      gvec[j] = cs[j] * gvec[j];
      jdone = j + 1;
      // happy breakdown (reading A21): the new direction is lost to rounding
      // relative to the vector it was orthogonalised from
      if (hn <= 1e-14 * std::sqrt(col2)) break;
      for (size_t k = 0; k < n; ++k) V[j + 1][k] = w[k] / hn;
    }
    // back substitution of the triangular system
    std::vector<double> yy(jdone, 0.0);
    for (int i = jdone - 1; i >= 0; --i) {
      double s = gvec[i];
      for (int k = i + 1; k < jdone; ++k) s -= H[i * m + k] * yy[k];
      yy[i] = s / H[i * m + i];
    }
    for (int i = 0; i < jdone; ++i)
      for (size_t k = 0; k < n; ++k) dQ[k] += yy[i] * V[i][k];
    last = std::fabs(gvec[jdone]);
  }
  info->n_limited = apply_update(C, Q, dQ.data());
  if (C.o.scheme == 1) relax_gradients(C, Gn, G);
  info->gmres_rel = beta0 > 0 ? last / beta0 : 0.0;
  info->n_resid_evals = evals;
  info->n_fallbacks = fb;
  for (int i = 0; i < N; ++i) {
    V5 q;
    for (int v = 0; v < 5; ++v) q[v] = Q[(size_t)v * N + i];
    if (!physical(q, C.o.gamma)) return -4;
  }
  return 0;
}

// ---------------------------------------------------------------------------
// C interface
// ---------------------------------------------------------------------------
extern "C" {

orc_ctx* orc_create(int64_t n_nodes, const double* xyz, int64_t n_tets, const int32_t* tets,
                    int64_t n_bf, const int32_t* bf, const int32_t* btag, int32_t n_tags,
                    const int32_t* kind_of_tag, const double* prim, const orc_options* opts) {
  orc_ctx* C = new orc_ctx;
  C->o = *opts;
  C->K = (5.0 - 3.0 * opts->gamma) / (opts->gamma - 1.0);
  C->rhoinf = prim[0];
  C->uinf = {prim[1], prim[2], prim[3]};
  C->pinf = prim[4];
  C->qinf = to_cons(prim[0], C->uinf, prim[4], opts->gamma);
  if (!build(*C, n_nodes, xyz, n_tets, tets, n_bf, bf, btag, n_tags, kind_of_tag)) {
    delete C;
    return nullptr;
  }
  return C;
}
orc_ctx* orc_create_hex(int64_t n_nodes, const double* xyz, int64_t n_hex, const int32_t* hexes,
                        int64_t n_bf, const int32_t* bf, const int32_t* btag, int32_t n_tags,
                        const int32_t* kind_of_tag, const double* prim, const orc_options* opts) {
  orc_ctx* C = new orc_ctx;
  C->o = *opts;
  C->K = (5.0 - 3.0 * opts->gamma) / (opts->gamma - 1.0);
  C->rhoinf = prim[0];
  C->uinf = {prim[1], prim[2], prim[3]};
  C->pinf = prim[4];
  C->qinf = to_cons(prim[0], C->uinf, prim[4], opts->gamma);
  if (!build_hex(*C, n_nodes, xyz, n_hex, hexes, n_bf, bf, btag, n_tags, kind_of_tag)) {
    delete C;
    return nullptr;
  }
  return C;
}
int32_t orc_face_points(const orc_ctx* C) { return C->faces.empty() ? 0 : C->faces[0].ng; }
int32_t orc_cell_faces(const orc_ctx* C) { return C->nf; }
const char* orc_error(void) { return g_err.c_str(); }
void orc_destroy(orc_ctx* C) { delete C; }
void orc_set_threads(int32_t n) { nthreads_req = n > 0 ? n : 1; }
int64_t orc_n_cells(const orc_ctx* C) { return C->N; }
int64_t orc_n_faces(const orc_ctx* C) { return (int64_t)C->faces.size(); }

void orc_geometry(const orc_ctx* C, double* vol, double* cen, double* m2) {
  int N = C->N;
  for (int i = 0; i < N; ++i) {
    vol[i] = C->vol[i];
    for (int d = 0; d < 3; ++d) cen[(size_t)d * N + i] = C->cen[i][d];
    const M33& m = C->m2[i];
    double s[6] = {m[0][0], m[1][1], m[2][2], m[0][1], m[0][2], m[1][2]};
    for (int k = 0; k < 6; ++k) m2[(size_t)k * N + i] = s[k];
  }
}
void orc_faces(const orc_ctx* C, int32_t* L, int32_t* R, double* area, double* nrm, double* gp) {
  size_t F = C->faces.size();
  for (size_t f = 0; f < F; ++f) {
    const Face& x = C->faces[f];
    L[f] = x.L;
    R[f] = x.R;
    area[f] = x.S;
    for (int d = 0; d < 3; ++d) nrm[d * F + f] = x.n[d];
    for (int g = 0; g < x.ng; ++g)
      for (int d = 0; d < 3; ++d) gp[(g * 3 + d) * F + f] = x.gp[g][d];
  }
}
int32_t orc_stencil(const orc_ctx* C, int64_t cell, int32_t which, int32_t* members, int32_t cap) {
  if (which < 0 || which > (int)C->sub[cell].size()) return -1;
  const std::vector<int>& s = which == 0 ? C->big[cell] : C->sub[cell][which - 1];
  int n = (int)s.size();
  for (int k = 0; k < n && k < cap; ++k) members[k] = s[k];
  return n;
}
void orc_dt(const orc_ctx* C, const double* Q, double* dt) { compute_dt(*C, Q, dt); }
int64_t orc_residual(const orc_ctx* C, const double* Q, const double* G, const double* dt,
                     double* R, double* Gnew) {
  std::vector<double> d;
  if (!dt) {
    d.resize(C->N);
    compute_dt(*C, Q, d.data());
    dt = d.data();
  }
  std::vector<double> zero;
  if (!G) {
    zero.assign((size_t)15 * C->N, 0.0);
    G = zero.data();
  }
  return residual(*C, Q, G, dt, R, Gnew);
}
int32_t orc_side_values(const orc_ctx* C, const double* Q, const double* G, int64_t f, int32_t side,
                        double* out) {
  std::vector<double> zero;
  if (!G) {
    zero.assign((size_t)15 * C->N, 0.0);
    G = zero.data();
  }
  double o[4][4][5];
  int r = side_values(*C, Q, G, (int)f, side, o);
  std::memcpy(out, o, sizeof(double) * 20 * C->faces[f].ng);
  return r;
}
// Residual (and compact gradient update) of the listed cells only: the same
// face sums as the full residual, evaluated for the faces of those cells (a
// face shared by two listed cells is evaluated twice).  R [5][n], Gnew
// [15][n] (may be NULL).  dt NULL: the local time steps of Q.
int64_t orc_residual_cells(const orc_ctx* C, const double* Q, const double* G, const double* dt, int64_t n,
                           const int64_t* cells, double* R, double* Gnew) {
  std::vector<double> d, zero;
  if (!dt) {
    d.resize(C->N);
    compute_dt(*C, Q, d.data());
    dt = d.data();
  }
  if (!G) {
    zero.assign((size_t)15 * C->N, 0.0);
    G = zero.data();
  }
  int64_t fb = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : fb) num_threads(nthreads_req)
  for (int64_t k = 0; k < n; ++k) {
    const int i = (int)cells[k];
    for (int v = 0; v < 5; ++v) R[(size_t)v * n + k] = 0.0;
    if (Gnew)
      for (int q = 0; q < 15; ++q) Gnew[(size_t)q * n + k] = 0.0;
    for (int p = 0; p < C->nf; ++p) {
      int fi = C->cf[i][p];
      const Face& f = C->faces[fi];
      V5 Ff, Qf;
      fb += face_flux(*C, Q, G, dt, fi, Ff, Gnew ? &Qf : nullptr);
      double sg = f.L == i ? 1.0 : -1.0;
      for (int v = 0; v < 5; ++v) R[(size_t)v * n + k] -= sg * Ff[v];
      if (Gnew)
        for (int v = 0; v < 5; ++v)
          for (int dd = 0; dd < 3; ++dd) Gnew[(size_t)(v * 3 + dd) * n + k] += sg * Qf[v] * f.n[dd] / C->vol[i];
    }
  }
  return fb;
}
// Integrated face fluxes (global frame, oriented L -> R) of the listed
// faces: F [5][n].  dt NULL: the local time steps of Q.
int64_t orc_face_fluxes(const orc_ctx* C, const double* Q, const double* G, const double* dt, int64_t n,
                        const int64_t* faces, double* Fout) {
  std::vector<double> d, zero;
  if (!dt) {
    d.resize(C->N);
    compute_dt(*C, Q, d.data());
    dt = d.data();
  }
  if (!G) {
    zero.assign((size_t)15 * C->N, 0.0);
    G = zero.data();
  }
  int64_t fb = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(+ : fb) num_threads(nthreads_req)
  for (int64_t k = 0; k < n; ++k) {
    V5 Ff;
    fb += face_flux(*C, Q, G, dt, (int)faces[k], Ff, nullptr);
    for (int v = 0; v < 5; ++v) Fout[(size_t)v * n + k] = Ff[v];
  }
  return fb;
}
// per-component polynomials, smoothness indicators and weights of one face
// side, and R* with its inverse (layout at side_values)
int32_t orc_side_debug(const orc_ctx* C, const double* Q, const double* G, int64_t f, int32_t side,
                       double* dbg) {
  std::vector<double> zero;
  if (!G) {
    zero.assign((size_t)15 * C->N, 0.0);
    G = zero.data();
  }
  double o[4][4][5];
  for (int k = 0; k < 370; ++k) dbg[k] = 0.0;
  return side_values(*C, Q, G, (int)f, side, o, dbg);
}
// right eigenvectors of the x-split Euler flux Jacobian at a local-frame state
// (columns u-c, u, u, u, u+c), row-major
void orc_right_eigenvectors(double gamma, const double* q, double* R) {
  V5 v{q[0], q[1], q[2], q[3], q[4]};
  double r[5][5];
  right_eigenvectors(v, gamma, r);
  for (int a = 0; a < 5; ++a)
    for (int b = 0; b < 5; ++b) R[5 * a + b] = r[a][b];
}
// ghost cell of boundary face f: its average (global frame), its gradient
// (15, var-major) and its centroid, given the owner's state and gradients
int32_t orc_ghost(const orc_ctx* C, const double* Q, const double* G, int64_t f, double* q, double* g,
                  double* c) {
  const Face& x = C->faces[f];
  if (x.R >= 0) return -1;
  int e = C->N + (-x.R - 1);
  V5 s = state_of(*C, Q, e);
  for (int k = 0; k < 5; ++k) q[k] = s[k];
  if (G) grad_of(*C, G, e, g);
  const V3& cc = C->c_of(e);
  for (int d = 0; d < 3; ++d) c[d] = cc[d];
  return x.kind;
}
// right state and derivatives (n, t1, t2) of a boundary Gauss point in the
// local frame of boundary face f, given the left ones
int32_t orc_boundary_right(const orc_ctx* C, int64_t f, const double* Wl, const double* dWl, double* Wr,
                           double* dWr) {
  const Face& x = C->faces[f];
  if (x.R >= 0) return -1;
  V5 l, r, dl[3], dr[3];
  for (int k = 0; k < 5; ++k) {
    l[k] = Wl[k];
    for (int d = 0; d < 3; ++d) dl[d][k] = dWl[d * 5 + k];
  }
  boundary_right(*C, x, l, dl, r, dr);
  for (int k = 0; k < 5; ++k) {
    Wr[k] = r[k];
    for (int d = 0; d < 3; ++d) dWr[d * 5 + k] = dr[d][k];
  }
  return x.kind;
}
// length scales: h of the scaled basis and the time-step length
void orc_cell_scales(const orc_ctx* C, double* h, double* hdt) {
  for (int i = 0; i < C->N; ++i) {
    h[i] = C->hcell[i];
    hdt[i] = C->hdt[i];
  }
}
void orc_face_frame(const orc_ctx* C, int64_t f, double* out) {
  const Face& x = C->faces[f];
  for (int d = 0; d < 3; ++d) {
    out[d] = x.n[d];
    out[3 + d] = x.t1[d];
    out[6 + d] = x.t2[d];
  }
}
void orc_gks_point(const orc_ctx* C, const double* Wl, const double* dWl, const double* Wr,
                   const double* dWr, double dt, double* F, double* QG) {
  V5 l, r, dl[3], dr[3];
  for (int k = 0; k < 5; ++k) {
    l[k] = Wl[k];
    r[k] = Wr[k];
    for (int d = 0; d < 3; ++d) {
      dl[d][k] = dWl[d * 5 + k];
      dr[d][k] = dWr[d * 5 + k];
    }
  }
  V5 f, q;
  gks_point(*C, l, dl, r, dr, dt, f, QG ? &q : nullptr);
  for (int k = 0; k < 5; ++k) F[k] = f[k];
  if (QG)
    for (int k = 0; k < 5; ++k) QG[k] = q[k];
}
void orc_kfvs_point(const orc_ctx* C, const double* Wl, const double* Wr, double* F, double* QG) {
  V5 l, r, f, q;
  for (int k = 0; k < 5; ++k) {
    l[k] = Wl[k];
    r[k] = Wr[k];
  }
  kfvs_point(*C, l, r, f, QG ? &q : nullptr);
  for (int k = 0; k < 5; ++k) F[k] = f[k];
  if (QG)
    for (int k = 0; k < 5; ++k) QG[k] = q[k];
}
double orc_moment(double U, double V, double W, double lam, double K, int32_t half, int32_t a,
                  int32_t b, int32_t c, int32_t d) {
  Moments M;
  M.init(U, V, W, lam, K, half);
  return M.m(a, b, c, d);
}
void orc_slope_solve(double U, double V, double W, double lam, double K, const double* rhs,
                     double* a) {
  Moments M;
  M.init(U, V, W, lam, K, 0);
  V5 r{rhs[0], rhs[1], rhs[2], rhs[3], rhs[4]};
  V5 x = slope_solve(M, r);
  for (int k = 0; k < 5; ++k) a[k] = x[k];
}
void orc_euler_jn(double gamma, const double* Q, const double* n, const double* x, double* out) {
  V5 q{Q[0], Q[1], Q[2], Q[3], Q[4]}, xx{x[0], x[1], x[2], x[3], x[4]};
  V5 r = euler_jn(gamma, q, V3{n[0], n[1], n[2]}, xx);
  for (int k = 0; k < 5; ++k) out[k] = r[k];
}
void orc_diag(const orc_ctx* C, const double* Q, const double* dt, double* D) { diag(*C, Q, dt, D); }
void orc_precond(const orc_ctx* C, const double* Q, const double* dt, const double* r, double* out) {
  precond(*C, Q, dt, r, out);
}
double orc_jv(const orc_ctx* C, const double* Q, const double* G, const double* dt, const double* b,
              const double* v, double sigma, double* Av) {
  std::vector<double> zero;
  if (!G) {
    zero.assign((size_t)15 * C->N, 0.0);
    G = zero.data();
  }
  return jv(*C, Q, G, dt, b, v, sigma, Av);
}
int32_t orc_implicit_step(const orc_ctx* C, double* Q, double* G, orc_step_info* info) {
  std::vector<double> zero;
  if (!G) {
    zero.assign((size_t)15 * C->N, 0.0);
    G = zero.data();
  }
  return implicit_step(*C, Q, G, info);
}
double orc_res_norm(const orc_ctx* C, const double* R) { return res_norm(*C, R); }
int32_t orc_colours(const orc_ctx* C, int32_t* col) {
  std::vector<int> c;
  int n = colour_cells(*C, c);
  for (int i = 0; i < C->N; ++i) col[i] = c[i];
  return n;
}
void orc_lusgs(const orc_ctx* C, const double* Q, const double* dt, const double* R, double* dQ) {
  lusgs(*C, Q, dt, R, dQ);
}
void orc_amatvec(const orc_ctx* C, const double* Q, const double* dt, const double* x, double* out) {
  amatvec(*C, Q, dt, x, out);
}

}  // extern "C"
