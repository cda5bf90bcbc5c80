// Host preprocessing of tetrahedral meshes for the HGKS kernels.
//
// Geometry (Sec. 2): volumes, centroids, second moments (exact simplex
// formula), face areas and normals, the 3-point degree-2 triangle rule.
// Stencils (Sec. 3.1): big WENO stencil {i, i_p, i_pm}, the four tetrahedral
// sub-stencils of 7 cells, the compact HWENO stencil {i, i_p}.  Boundary faces
// carry a ghost cell: the mirror image of the owner across the face plane.
// Operators (Sec. 3.2, 3.3): the least-squares fits are linear in the data,
// so each cell stores the matrix that maps stencil data to polynomial
// coefficients (basis: xi = (x - c_i)/h_i, quadratic terms with their cell
// mean removed).
#include "mesh_prep.h"

#include <algorithm>
#include <array>
#include <cmath>
#include <cstring>

namespace hgks {
namespace {

struct Vec3 {
  double x, y, z;
};
inline Vec3 operator-(Vec3 a, Vec3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline Vec3 operator+(Vec3 a, Vec3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline Vec3 operator*(double s, Vec3 a) { return {s * a.x, s * a.y, s * a.z}; }
inline double dotp(Vec3 a, Vec3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline Vec3 crossp(Vec3 a, Vec3 b) { return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x}; }
inline double comp(const Vec3& a, int k) { return k == 0 ? a.x : (k == 1 ? a.y : a.z); }

struct Sym3 {
  double a[3][3];
};

// Pseudo-inverse X (n x m, row-major) of a full-column-rank A (m x n,
// row-major) by modified Gram-Schmidt QR with one re-orthogonalisation pass.
void pinv_mgs(const double* A, int m, int n, double* X) {
  std::vector<double> Q(A, A + (size_t)m * n), R((size_t)n * n, 0.0);
  for (int j = 0; j < n; ++j) {
    for (int pass = 0; pass < 2; ++pass)
      for (int k = 0; k < j; ++k) {
        double r = 0.0;
        for (int i = 0; i < m; ++i) r += Q[i * n + k] * Q[i * n + j];
        R[k * n + j] += r;
        for (int i = 0; i < m; ++i) Q[i * n + j] -= r * Q[i * n + k];
      }
    double nr = 0.0;
    for (int i = 0; i < m; ++i) nr += Q[i * n + j] * Q[i * n + j];
    nr = std::sqrt(nr);
    R[j * n + j] = nr;
    for (int i = 0; i < m; ++i) Q[i * n + j] /= nr;
  }
  // X = R^{-1} Q^T: back substitution for each column of Q^T
  for (int i = 0; i < m; ++i)
    for (int r = n - 1; r >= 0; --r) {
      double s = Q[i * n + r];
      for (int c = r + 1; c < n; ++c) s -= R[r * n + c] * X[c * m + i];
      X[r * m + i] = s / R[r * n + r];
    }
}

// Smallest / largest eigenvalue ratio of A^T A by cyclic Jacobi rotations.
double gram_cond_ratio(const double* A, int m, int n) {
  std::vector<double> G((size_t)n * n, 0.0);
  for (int r = 0; r < m; ++r)
    for (int p = 0; p < n; ++p)
      for (int q = 0; q < n; ++q) G[p * n + q] += A[r * n + p] * A[r * n + q];
  for (int it = 0; it < 60; ++it) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += G[p * n + q] * G[p * n + q];
    if (off < 1e-300) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        double gpq = G[p * n + q];
        if (gpq == 0.0) continue;
        double th = 0.5 * (G[q * n + q] - G[p * n + p]) / gpq;
        double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(1.0 + th * th));
        double c = 1.0 / std::sqrt(1.0 + t * t), s = t * c;
        for (int k = 0; k < n; ++k) {
          double gkp = G[k * n + p], gkq = G[k * n + q];
          G[k * n + p] = c * gkp - s * gkq;
          G[k * n + q] = s * gkp + c * gkq;
        }
        for (int k = 0; k < n; ++k) {
          double gpk = G[p * n + k], gqk = G[q * n + k];
          G[p * n + k] = c * gpk - s * gqk;
          G[q * n + k] = s * gpk + c * gqk;
        }
      }
  }
  double mn = G[0], mx = G[0];
  for (int k = 1; k < n; ++k) {
    mn = std::min(mn, G[k * n + k]);
    mx = std::max(mx, G[k * n + k]);
  }
  return mx > 0.0 ? mn / mx : 0.0;
}

// Dense inverse of an n x n matrix by Gauss-Jordan with partial pivoting.
bool invert(std::vector<double> A, int n, std::vector<double>& Ainv) {
  Ainv.assign((size_t)n * n, 0.0);
  for (int k = 0; k < n; ++k) Ainv[k * n + k] = 1.0;
  for (int c = 0; c < n; ++c) {
    int piv = c;
    for (int r = c + 1; r < n; ++r)
      if (std::fabs(A[r * n + c]) > std::fabs(A[piv * n + c])) piv = r;
    if (A[piv * n + c] == 0.0) return false;
    for (int k = 0; k < n; ++k) {
      std::swap(A[c * n + k], A[piv * n + k]);
      std::swap(Ainv[c * n + k], Ainv[piv * n + k]);
    }
    double ip = 1.0 / A[c * n + c];
    for (int k = 0; k < n; ++k) {
      A[c * n + k] *= ip;
      Ainv[c * n + k] *= ip;
    }
    for (int r = 0; r < n; ++r) {
      if (r == c) continue;
      double f = A[r * n + c];
      if (f == 0.0) continue;
      for (int k = 0; k < n; ++k) {
        A[r * n + k] -= f * A[c * n + k];
        Ainv[r * n + k] -= f * Ainv[c * n + k];
      }
    }
  }
  return true;
}

struct FaceRec {
  std::array<int, 3> key;
  int tet, p;
};

}  // namespace

int build_host_mesh(HostMesh& H, int64_t n_nodes, const double* xyz, int64_t n_tets, const int32_t* tet2node,
                    int64_t n_bf, const int32_t* bf, const int32_t* btag, std::string& err) {
  if (n_nodes <= 0 || n_tets <= 0 || !xyz || !tet2node || n_tets > (int64_t)1 << 30) {
    err = "invalid mesh arguments";
    return -1;
  }
  const int N = (int)n_tets;
  H = HostMesh();
  H.N = N;
  auto P = [&](int node) { return Vec3{xyz[3 * (size_t)node], xyz[3 * (size_t)node + 1], xyz[3 * (size_t)node + 2]}; };
  std::vector<Vec3> cen(N);
  std::vector<Sym3> m2(N);
  H.vol.resize(N);
  for (int i = 0; i < N; ++i) {
    Vec3 v[4];
    for (int k = 0; k < 4; ++k) {
      int nd = tet2node[4 * (size_t)i + k];
      if (nd < 0 || nd >= n_nodes) {
        err = "tet node id out of range at tet " + std::to_string(i);
        return -3;
      }
      v[k] = P(nd);
    }
    double d6 = dotp(crossp(v[1] - v[0], v[2] - v[0]), v[3] - v[0]);
    if (!(d6 > 0.0) || !std::isfinite(d6)) {
      err = "inverted or degenerate tet " + std::to_string(i);
      return -3;
    }
    H.vol[i] = d6 / 6.0;
    Vec3 c = 0.25 * (((v[0] + v[1]) + v[2]) + v[3]);
    cen[i] = c;
    Sym3 s;
    std::memset(&s, 0, sizeof(s));
    for (int k = 0; k < 4; ++k) {
      Vec3 d = v[k] - c;
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) s.a[a][b] += comp(d, a) * comp(d, b) / 20.0;
    }
    m2[i] = s;
  }
  // ---- faces: sort the 4N tet faces by their node triple and pair them ----
  std::vector<FaceRec> recs((size_t)4 * N);
  for (int i = 0; i < N; ++i)
    for (int p = 0; p < 4; ++p) {
      std::array<int, 3> k;
      int q = 0;
      for (int c = 0; c < 4; ++c)
        if (c != p) k[q++] = tet2node[4 * (size_t)i + c];
      std::sort(k.begin(), k.end());
      recs[(size_t)4 * i + p] = {k, i, p};
    }
  std::sort(recs.begin(), recs.end(), [](const FaceRec& a, const FaceRec& b) {
    return a.key != b.key ? a.key < b.key : (a.tet != b.tet ? a.tet < b.tet : a.p < b.p);
  });
  std::vector<std::array<int, 3>> bkeys((size_t)n_bf);
  std::vector<std::pair<std::array<int, 3>, int>> bsorted((size_t)n_bf);
  for (int64_t k = 0; k < n_bf; ++k) {
    std::array<int, 3> key{bf[3 * k], bf[3 * k + 1], bf[3 * k + 2]};
    std::sort(key.begin(), key.end());
    bsorted[k] = {key, btag[k]};
  }
  std::sort(bsorted.begin(), bsorted.end());
  H.cface.assign((size_t)4 * N, 0);
  std::vector<std::array<int, 4>> nbr(N, std::array<int, 4>{-1, -1, -1, -1});
  struct FaceTmp {
    int L, pL, R, pR, tag;
  };
  std::vector<FaceTmp> ft;
  ft.reserve((size_t)2 * N + n_bf);
  size_t nb_found = 0;
  for (size_t k = 0; k < recs.size();) {
    size_t e = k + 1;
    while (e < recs.size() && recs[e].key == recs[k].key) ++e;
    if (e - k > 2) {
      err = "non-manifold face";
      return -3;
    }
    FaceTmp f{recs[k].tet, recs[k].p, -1, -1, -1};
    if (e - k == 2) {
      f.R = recs[k + 1].tet;
      f.pR = recs[k + 1].p;
    } else {
      auto it = std::lower_bound(bsorted.begin(), bsorted.end(), std::make_pair(recs[k].key, INT32_MIN));
      if (it == bsorted.end() || it->first != recs[k].key) {
        err = "boundary face without a tag";
        return -3;
      }
      if (it->second < 0 || it->second > 255) {
        err = "boundary tag out of range";
        return -3;
      }
      f.tag = it->second;
      ++nb_found;
    }
    ft.push_back(f);
    k = e;
  }
  if ((int64_t)nb_found != n_bf) {
    err = "boundary face list does not match the mesh boundary";
    return -3;
  }
  // face order: by left cell, then its local face.  Consecutive faces then
  // share or neighbour their left cell, so a wavefront's loads of left-cell
  // data touch few cache lines (the cell order is the caller's).
  std::sort(ft.begin(), ft.end(),
            [](const FaceTmp& a, const FaceTmp& b) { return a.L != b.L ? a.L < b.L : a.pL < b.pL; });
  const int F = (int)ft.size();
  H.F = F;
  H.Nb = (int)nb_found;
  const int NX = N + H.Nb;
  H.fL.resize(F);
  H.fR.resize(F);
  H.ftag.resize(F);
  H.fn.resize((size_t)3 * F);
  H.fS.resize(F);
  H.fxiL.resize((size_t)9 * F);
  H.fxiR.resize((size_t)9 * F);
  H.gowner.resize(H.Nb);
  H.gface.resize(H.Nb);
  std::vector<Vec3> cx(NX);  // centroids incl. ghosts
  std::vector<Sym3> mx(NX);
  std::vector<double> hx(NX);
  for (int i = 0; i < N; ++i) {
    cx[i] = cen[i];
    mx[i] = m2[i];
    hx[i] = std::cbrt(H.vol[i]);
  }
  std::vector<double> smax(N, 0.0);
  std::vector<std::array<Vec3, 3>> gps(F);
  int g = 0;
  for (int f = 0; f < F; ++f) {
    const FaceTmp& t = ft[f];
    Vec3 v[3];
    int q = 0;
    for (int c = 0; c < 4; ++c)
      if (c != t.pL) v[q++] = P(tet2node[4 * (size_t)t.L + c]);
    Vec3 nn = crossp(v[1] - v[0], v[2] - v[0]);
    double len = std::sqrt(dotp(nn, nn));
    if (!(len > 0.0)) {
      err = "degenerate face";
      return -3;
    }
    double S = 0.5 * len;
    Vec3 n = (1.0 / len) * nn;
    Vec3 xc = (1.0 / 3.0) * ((v[0] + v[1]) + v[2]);
    if (dotp(n, xc - cen[t.L]) < 0.0) n = -1.0 * n;
    for (int k = 0; k < 3; ++k) gps[f][k] = (2.0 / 3.0) * v[k] + (1.0 / 6.0) * (v[(k + 1) % 3] + v[(k + 2) % 3]);
    H.fL[f] = t.L;
    H.fn[f] = n.x;
    H.fn[F + f] = n.y;
    H.fn[2 * (size_t)F + f] = n.z;
    H.fS[f] = S;
    smax[t.L] = std::max(smax[t.L], S);
    H.cface[(size_t)t.pL * N + t.L] = f + 1;
    if (t.R >= 0) {
      H.fR[f] = t.R;
      H.ftag[f] = -1;
      smax[t.R] = std::max(smax[t.R], S);
      H.cface[(size_t)t.pR * N + t.R] = -(f + 1);
      nbr[t.L][t.pL] = t.R;
      nbr[t.R][t.pR] = t.L;
    } else {
      int e = N + g;
      H.fR[f] = e;
      H.ftag[f] = t.tag;
      H.gowner[g] = t.L;
      H.gface[g] = f;
      nbr[t.L][t.pL] = e;
      // ghost: mirror image of the owner across the face plane
      Vec3 cl = cen[t.L];
      cx[e] = cl - (2.0 * dotp(cl - xc, n)) * n;
      double Rm[3][3];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) Rm[a][b] = (a == b ? 1.0 : 0.0) - 2.0 * comp(n, a) * comp(n, b);
      Sym3 s;
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
          double acc = 0.0;
          for (int x = 0; x < 3; ++x)
            for (int y = 0; y < 3; ++y) acc += Rm[a][x] * m2[t.L].a[x][y] * Rm[y][b];
          s.a[a][b] = acc;
        }
      mx[e] = s;
      hx[e] = hx[t.L];
      ++g;
    }
  }
  H.h.resize(N);
  H.hdt.resize(N);
  H.m2s.resize((size_t)6 * N);
  H.cen.resize((size_t)3 * N);
  H.total_volume = 0.0;
  for (int i = 0; i < N; ++i) {
    H.h[i] = hx[i];
    H.hdt[i] = 3.0 * H.vol[i] / smax[i];
    double hh = hx[i] * hx[i];
    const double* s = &m2[i].a[0][0];
    double vals[6] = {s[0], s[4], s[8], s[1], s[2], s[5]};
    for (int k = 0; k < 6; ++k) H.m2s[(size_t)k * N + i] = vals[k] / hh;
    H.cen[i] = cen[i].x;
    H.cen[N + i] = cen[i].y;
    H.cen[2 * (size_t)N + i] = cen[i].z;
    H.total_volume += H.vol[i];
  }
  for (int f = 0; f < F; ++f) {
    int L = H.fL[f], R = H.fR[f];
    for (int k = 0; k < 3; ++k) {
      Vec3 dl = (1.0 / hx[L]) * (gps[f][k] - cen[L]);
      for (int d = 0; d < 3; ++d) H.fxiL[(size_t)(k * 3 + d) * F + f] = comp(dl, d);
      Vec3 dr = R < N ? (1.0 / hx[R]) * (gps[f][k] - cen[R]) : Vec3{0, 0, 0};
      for (int d = 0; d < 3; ++d) H.fxiR[(size_t)(k * 3 + d) * F + f] = comp(dr, d);
    }
  }
  // ---- stencils ----
  H.stn.assign((size_t)16 * N, 0);
  H.sstn.assign((size_t)24 * N, 0);
  H.opA.assign((size_t)144 * N, 0.0);
  H.opB.assign((size_t)72 * N, 0.0);
  H.smask.assign(N, 0);
  H.nb4.assign((size_t)4 * N, 0);
  H.opH.assign((size_t)171 * N, 0.0);
  H.hsub.assign((size_t)24 * N, 0.0);
  // basis means of cell e in the frame of cell i (9 values)
  auto row9 = [&](int i, int e, double* r) {
    double hi = hx[i];
    Vec3 d = cx[e] - cx[i];
    r[0] = d.x / hi;
    r[1] = d.y / hi;
    r[2] = d.z / hi;
    const int A[6] = {0, 1, 2, 0, 0, 1}, B[6] = {0, 1, 2, 1, 2, 2};
    for (int k = 0; k < 6; ++k)
      r[3 + k] = (mx[e].a[A[k]][B[k]] + comp(d, A[k]) * comp(d, B[k]) - mx[i].a[A[k]][B[k]]) / (hi * hi);
  };
  int64_t nfb = 0, nsd = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : nfb, nsd)
  for (int i = 0; i < N; ++i) {
    auto add = [](std::vector<int>& v, int e) {
      for (int x : v)
        if (x == e) return;
      v.push_back(e);
    };
    std::vector<int> big;
    big.reserve(17);
    for (int p = 0; p < 4; ++p) add(big, nbr[i][p]);
    for (int p = 0; p < 4; ++p) {
      int j = nbr[i][p];
      if (j >= N) continue;
      for (int q = 0; q < 4; ++q)
        if (nbr[j][q] != i) add(big, nbr[j][q]);
    }
    int m = (int)big.size();
    for (int r = 0; r < 16; ++r) H.stn[(size_t)r * N + i] = r < m ? big[r] : i;
    // P0 operator
    std::vector<double> A((size_t)m * 9), X((size_t)9 * m);
    for (int r = 0; r < m; ++r) row9(i, big[r], &A[(size_t)r * 9]);
    if (m >= 9 && gram_cond_ratio(A.data(), m, 9) > 1e-20) {
      pinv_mgs(A.data(), m, 9, X.data());
      for (int k = 0; k < 9; ++k)
        for (int r = 0; r < m; ++r) H.opA[(size_t)(k * 16 + r) * N + i] = X[(size_t)k * m + r];
    } else {
      // rank-deficient big stencil: linear least squares on it
      ++nfb;
      std::vector<double> A3((size_t)m * 3), X3((size_t)3 * m);
      for (int r = 0; r < m; ++r)
        for (int k = 0; k < 3; ++k) A3[r * 3 + k] = A[r * 9 + k];
      pinv_mgs(A3.data(), m, 3, X3.data());
      for (int k = 0; k < 3; ++k)
        for (int r = 0; r < m; ++r) H.opA[(size_t)(k * 16 + r) * N + i] = X3[(size_t)k * m + r];
    }
    // sub-stencils S_i1..S_i4: faces {1,2,3},{1,2,4},{2,3,4},{3,1,4} plus the
    // neighbours of i_1..i_4 respectively (1-based as in the paper)
    const int first[4][3] = {{0, 1, 2}, {0, 1, 3}, {1, 2, 3}, {2, 0, 3}};
    uint8_t mask = 0;
    for (int s = 0; s < 4; ++s) {
      std::vector<int> sub;
      for (int k = 0; k < 3; ++k) add(sub, nbr[i][first[s][k]]);
      int j = nbr[i][s];
      if (j < N)
        for (int q = 0; q < 4; ++q)
          if (nbr[j][q] != i) add(sub, nbr[j][q]);
      int ms = (int)sub.size();
      for (int r = 0; r < 6; ++r) H.sstn[(size_t)(s * 6 + r) * N + i] = r < ms ? sub[r] : i;
      std::vector<double> As((size_t)ms * 3), Xs((size_t)3 * ms);
      for (int r = 0; r < ms; ++r) {
        double rr[9];
        row9(i, sub[r], rr);
        for (int k = 0; k < 3; ++k) As[r * 3 + k] = rr[k];
      }
      if (ms >= 3 && gram_cond_ratio(As.data(), ms, 3) > 1e-20) {
        pinv_mgs(As.data(), ms, 3, Xs.data());
        for (int t = 0; t < 3; ++t)
          for (int r = 0; r < ms; ++r) H.opB[(size_t)((s * 3 + t) * 6 + r) * N + i] = Xs[(size_t)t * ms + r];
        mask |= (uint8_t)(1u << s);
      } else {
        ++nsd;
      }
    }
    H.smask[i] = mask;
    // ---- compact HWENO: constrained least squares (Sec. 3.3) ----
    for (int k = 0; k < 4; ++k) H.nb4[(size_t)k * N + i] = nbr[i][k];
    {
      const int nu = 9, ne = 4, nl = 15, nk = nu + ne;
      double Ce[4][9], Al[15][9];
      for (int r = 0; r < 4; ++r) row9(i, nbr[i][r], Ce[r]);
      int mem[5] = {i, nbr[i][0], nbr[i][1], nbr[i][2], nbr[i][3]};
      double hk[5];
      for (int k = 0; k < 5; ++k) {
        int e = mem[k];
        hk[k] = hx[e];
        Vec3 d = (1.0 / hx[i]) * (cx[e] - cx[i]);
        double rows[3][9] = {{1, 0, 0, 2 * d.x, 0, 0, d.y, d.z, 0},
                             {0, 1, 0, 0, 2 * d.y, 0, d.x, 0, d.z},
                             {0, 0, 1, 0, 0, 2 * d.z, 0, d.x, d.y}};
        for (int a = 0; a < 3; ++a)
          for (int q = 0; q < 9; ++q) Al[3 * k + a][q] = hk[k] * rows[a][q] / hx[i];
      }
      std::vector<double> K((size_t)nk * nk, 0.0), Ki;
      for (int p = 0; p < nu; ++p) {
        for (int q = 0; q < nu; ++q) {
          double s = 0.0;
          for (int r = 0; r < nl; ++r) s += Al[r][p] * Al[r][q];
          K[p * nk + q] = 2.0 * s;
        }
        for (int r = 0; r < ne; ++r) {
          K[p * nk + nu + r] = Ce[r][p];
          K[(nu + r) * nk + p] = Ce[r][p];
        }
      }
      invert(K, nk, Ki);
      // a = Ki[0:9, 0:9] 2 Al^T (h G) + Ki[0:9, 9:13] dQ
      for (int k = 0; k < 9; ++k) {
        for (int j = 0; j < 4; ++j) H.opH[(size_t)(k * 19 + j) * N + i] = Ki[k * nk + nu + j];
        for (int mk = 0; mk < 5; ++mk)
          for (int a = 0; a < 3; ++a) {
            int row = 3 * mk + a;
            double s = 0.0;
            for (int q = 0; q < nu; ++q) s += Ki[k * nk + q] * 2.0 * Al[row][q];
            s *= hk[mk];
            int j = mk == 0 ? 4 + a : 7 + 3 * (mk - 1) + a;
            H.opH[(size_t)(k * 19 + j) * N + i] = s;
          }
      }
      for (int s = 0; s < 4; ++s) {
        int e = nbr[i][s];
        double h2i = hx[i] * hx[i], h2m = hx[e] * hx[e];
        Vec3 d = cx[e] - cx[i];
        double vals[6] = {h2i / (h2i + h2m), h2m / (h2i + h2m), d.x, d.y, d.z, 1.0 / dotp(d, d)};
        for (int k = 0; k < 6; ++k) H.hsub[(size_t)(s * 6 + k) * N + i] = vals[k];
      }
    }
  }
  H.n_big_fallback = nfb;
  H.n_sub_dropped = nsd;
  return 0;
}

int colour_cells(const HostMesh& H, std::vector<int>& col, std::vector<int>& order, std::vector<int>& start) {
  const int N = H.N;
  col.assign(N, -1);
  int ncol = 0;
  for (int i = 0; i < N; ++i) {
    unsigned taken = 0;  // bit c: a coloured neighbour has colour c
    for (int k = 0; k < 4; ++k) {
      int j = H.nb4[(size_t)k * N + i];
      if (j < N && col[j] >= 0) taken |= 1u << col[j];
    }
    int c = 0;
    while (taken & (1u << c)) ++c;
    col[i] = c;
    if (c + 1 > ncol) ncol = c + 1;
  }
  // counting sort by colour keeps the index order within a colour
  start.assign(ncol + 1, 0);
  for (int i = 0; i < N; ++i) ++start[col[i] + 1];
  for (int c = 0; c < ncol; ++c) start[c + 1] += start[c];
  order.assign(N, 0);
  std::vector<int> next(start.begin(), start.end() - 1);
  for (int i = 0; i < N; ++i) order[next[col[i]]++] = i;
  return ncol;
}

}  // namespace hgks
