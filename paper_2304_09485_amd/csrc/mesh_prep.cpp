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

struct FaceTmp {
  int L, pL, R, pR, tag;
};

// geometry of one face as seen from its left cell
struct FaceGeo {
  Vec3 n{0, 0, 0}, xc{0, 0, 0};
  double S = 0.0;
  Vec3 gp[4];
  double gw[4] = {0, 0, 0, 0};
};

// Pair the nf faces of every cell by their sorted node keys (NV nodes per
// face); unpaired faces must appear in the tagged boundary list.
template <int NV, typename NodesOf>
int pair_faces(int N, int nf, NodesOf nodes_of, int64_t n_bf, const int32_t* bf, const int32_t* btag,
               std::vector<FaceTmp>& ft, int& nb_found, std::string& err) {
  struct Rec {
    std::array<int, NV> key;
    int cell, p;
  };
  std::vector<Rec> recs((size_t)nf * N);
  for (int i = 0; i < N; ++i)
    for (int p = 0; p < nf; ++p) {
      std::array<int, NV> k = nodes_of(i, p);
      std::sort(k.begin(), k.end());
      recs[(size_t)nf * i + p] = {k, i, p};
    }
  std::sort(recs.begin(), recs.end(), [](const Rec& a, const Rec& b) {
    return a.key != b.key ? a.key < b.key : (a.cell != b.cell ? a.cell < b.cell : a.p < b.p);
  });
  std::vector<std::pair<std::array<int, NV>, int>> bsorted((size_t)n_bf);
  for (int64_t k = 0; k < n_bf; ++k) {
    std::array<int, NV> key;
    for (int q = 0; q < NV; ++q) key[q] = bf[NV * k + q];
    std::sort(key.begin(), key.end());
    bsorted[k] = {key, btag[k]};
  }
  std::sort(bsorted.begin(), bsorted.end());
  ft.clear();
  ft.reserve((size_t)nf * N / 2 + n_bf);
  nb_found = 0;
  for (size_t k = 0; k < recs.size();) {
    size_t e = k + 1;
    while (e < recs.size() && recs[e].key == recs[k].key) ++e;
    if (e - k > 2) {
      err = "non-manifold face";
      return -3;
    }
    FaceTmp f{recs[k].cell, recs[k].p, -1, -1, -1};
    if (e - k == 2) {
      f.R = recs[k + 1].cell;
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
  return 0;
}

// Faces, ghosts, length scales, stencils and reconstruction operators, common
// to both cell shapes (H.nf, H.ng, H.nbig, H.nsw, H.msw set by the caller).
template <typename Geo>
int finish_mesh(HostMesh& H, const std::vector<Vec3>& cen, const std::vector<Sym3>& m2, std::vector<FaceTmp>& ft,
                int nb_found, Geo face_geo, std::string& err) {
  const int N = H.N, nf = H.nf, ng = H.ng;
  // face order: by left cell, then its local face.  Consecutive faces then
  // share or neighbour their left cell, so a wavefront's loads of left-cell
  // data touch few cache lines (the cell order is the caller's).
  std::sort(ft.begin(), ft.end(),
            [](const FaceTmp& a, const FaceTmp& b) { return a.L != b.L ? a.L < b.L : a.pL < b.pL; });
  const int F = (int)ft.size();
  H.F = F;
  H.Nb = nb_found;
  const int NX = N + H.Nb;
  H.fL.resize(F);
  H.fR.resize(F);
  H.ftag.resize(F);
  H.fn.resize((size_t)3 * F);
  H.fS.resize(F);
  H.fxiL.resize((size_t)3 * ng * F);
  H.fxiR.resize((size_t)3 * ng * F);
  if (ng == 4) H.fw.resize((size_t)4 * F);
  H.gowner.resize(H.Nb);
  H.gface.resize(H.Nb);
  H.cface.assign((size_t)nf * N, 0);
  std::vector<std::array<int, 6>> nbr(N, std::array<int, 6>{-1, -1, -1, -1, -1, -1});
  std::vector<Vec3> cx(NX);  // centroids incl. ghosts
  std::vector<Sym3> mx(NX);
  std::vector<double> hx(NX);
  for (int i = 0; i < N; ++i) {
    cx[i] = cen[i];
    mx[i] = m2[i];
    hx[i] = std::cbrt(H.vol[i]);
  }
  std::vector<double> smax(N, 0.0);
  std::vector<std::array<Vec3, 4>> gps(F);
  int g = 0;
  for (int f = 0; f < F; ++f) {
    const FaceTmp& t = ft[f];
    FaceGeo G;
    if (!face_geo(t, G)) {
      err = "degenerate face";
      return -3;
    }
    Vec3 n = G.n, xc = G.xc;
    if (dotp(n, xc - cen[t.L]) < 0.0) {
      if (ng == 4) {
        err = "face normal does not point out of hexahedron " + std::to_string(t.L);
        return -3;
      }
      n = -1.0 * n;
    }
    for (int k = 0; k < ng; ++k) gps[f][k] = G.gp[k];
    if (ng == 4)
      for (int k = 0; k < 4; ++k) H.fw[(size_t)k * F + f] = G.gw[k];
    const double S = G.S;
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
    // time-step length: the height of a tetrahedron, the width of a hexahedron
    H.hdt[i] = (nf == 4 ? 3.0 : 1.0) * H.vol[i] / smax[i];
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
    for (int k = 0; k < ng; ++k) {
      Vec3 dl = (1.0 / hx[L]) * (gps[f][k] - cen[L]);
      for (int d = 0; d < 3; ++d) H.fxiL[(size_t)(k * 3 + d) * F + f] = comp(dl, d);
      Vec3 dr = R < N ? (1.0 / hx[R]) * (gps[f][k] - cen[R]) : Vec3{0, 0, 0};
      for (int d = 0; d < 3; ++d) H.fxiR[(size_t)(k * 3 + d) * F + f] = comp(dr, d);
    }
  }
  // ---- stencils: the largest non-compact stencil sets the hexahedral slot count ----
  auto add = [](std::vector<int>& v, int e) {
    for (int x : v)
      if (x == e) return;
    v.push_back(e);
  };
  auto big_of = [&](int i, std::vector<int>& big) {
    big.clear();
    for (int p = 0; p < nf; ++p) add(big, nbr[i][p]);
    for (int p = 0; p < nf; ++p) {
      int j = nbr[i][p];
      if (j >= N) continue;
      for (int q = 0; q < nf; ++q)
        if (nbr[j][q] != i) add(big, nbr[j][q]);
    }
  };
  if (nf == 6) {
    int mx_big = 0;
    std::vector<int> big;
    for (int i = 0; i < N; ++i) {
      big_of(i, big);
      mx_big = std::max(mx_big, (int)big.size());
    }
    H.nbig = std::max(9, mx_big);
  }
  const int nbig = H.nbig, nsw = H.nsw, msw = H.msw, nhrow = nf + 3 * (nf + 1);
  H.stn.assign((size_t)nbig * N, 0);
  H.sstn.assign((size_t)nsw * msw * N, 0);
  H.opA.assign((size_t)9 * nbig * N, 0.0);
  H.opB.assign((size_t)nsw * 3 * msw * N, 0.0);
  H.smask.assign(N, 0);
  H.nbf.assign((size_t)nf * N, 0);
  H.opH.assign((size_t)9 * nhrow * N, 0.0);
  H.hsub.assign((size_t)6 * nf * N, 0.0);
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
  // a cell with two boundary faces whose planes meet at more than 45 degrees
  // (on an edge or at a corner of the boundary) is fitted linearly: the
  // quadratic fit has growing modes there
  auto at_edge = [&](int i) {
    const double c45 = std::sqrt(0.5);
    for (int p = 0; p < nf; ++p) {
      if (nbr[i][p] < N) continue;
      const int fa = H.gface[nbr[i][p] - N];
      for (int q = 0; q < p; ++q) {
        if (nbr[i][q] < N) continue;
        const int fb = H.gface[nbr[i][q] - N];
        double d = 0.0;
        for (int k = 0; k < 3; ++k) d += H.fn[(size_t)k * F + fa] * H.fn[(size_t)k * F + fb];
        if (std::fabs(d) < c45) return true;
      }
    }
    return false;
  };
  int64_t nfb = 0, nsd = 0;
#pragma omp parallel for schedule(dynamic, 256) reduction(+ : nfb, nsd)
  for (int i = 0; i < N; ++i) {
    std::vector<int> big;
    big.reserve(40);
    big_of(i, big);
    int m = (int)big.size();
    for (int r = 0; r < nbig; ++r) H.stn[(size_t)r * N + i] = r < m ? big[r] : i;
    // P0 operator
    std::vector<double> A((size_t)m * 9), X((size_t)9 * m);
    for (int r = 0; r < m; ++r) row9(i, big[r], &A[(size_t)r * 9]);
    if (m >= 9 && gram_cond_ratio(A.data(), m, 9) > 1e-20 && !at_edge(i)) {
      pinv_mgs(A.data(), m, 9, X.data());
      for (int k = 0; k < 9; ++k)
        for (int r = 0; r < m; ++r) H.opA[(size_t)(k * nbig + r) * N + i] = X[(size_t)k * m + r];
    } else {
      // rank-deficient big stencil, or a cell on a boundary edge: linear
      // least squares on the big stencil
      ++nfb;
      std::vector<double> A3((size_t)m * 3), X3((size_t)3 * m);
      for (int r = 0; r < m; ++r)
        for (int k = 0; k < 3; ++k) A3[r * 3 + k] = A[r * 9 + k];
      pinv_mgs(A3.data(), m, 3, X3.data());
      for (int k = 0; k < 3; ++k)
        for (int r = 0; r < m; ++r) H.opA[(size_t)(k * nbig + r) * N + i] = X3[(size_t)k * m + r];
    }
    uint8_t mask = 0;
    for (int s = 0; s < nsw; ++s) {
      std::vector<int> sub;
      if (nf == 4) {
        // sub-stencils S_i1..S_i4: faces {1,2,3},{1,2,4},{2,3,4},{3,1,4} plus
        // the neighbours of i_1..i_4 respectively (1-based as in the paper)
        const int first[4][3] = {{0, 1, 2}, {0, 1, 3}, {1, 2, 3}, {2, 0, 3}};
        for (int k = 0; k < 3; ++k) add(sub, nbr[i][first[s][k]]);
        int j = nbr[i][s];
        if (j < N)
          for (int q = 0; q < 4; ++q)
            if (nbr[j][q] != i) add(sub, nbr[j][q]);
      } else {
        // hexahedron: F1 or F6 with two consecutive lateral faces F2..F5
        const int lat[5] = {1, 2, 3, 4, 1};
        add(sub, nbr[i][s < 4 ? 0 : 5]);
        add(sub, nbr[i][lat[s % 4]]);
        add(sub, nbr[i][lat[s % 4 + 1]]);
      }
      int ms = (int)sub.size();
      for (int r = 0; r < msw; ++r) H.sstn[(size_t)(s * msw + r) * N + i] = r < ms ? sub[r] : i;
      std::vector<double> As((size_t)ms * 3), Xs((size_t)3 * ms);
      for (int r = 0; r < ms; ++r) {
        double rr[9];
        row9(i, sub[r], rr);
        for (int k = 0; k < 3; ++k) As[r * 3 + k] = rr[k];
      }
      if (ms >= 3 && gram_cond_ratio(As.data(), ms, 3) > 1e-20) {
        pinv_mgs(As.data(), ms, 3, Xs.data());
        for (int t = 0; t < 3; ++t)
          for (int r = 0; r < ms; ++r)
            H.opB[(size_t)((s * 3 + t) * msw + r) * N + i] = Xs[(size_t)t * ms + r];
        mask |= (uint8_t)(1u << s);
      } else {
        ++nsd;
      }
    }
    H.smask[i] = mask;
    // ---- compact HWENO: constrained least squares (Sec. 3.3) ----
    for (int k = 0; k < nf; ++k) H.nbf[(size_t)k * N + i] = nbr[i][k];
    {
      const int nu = 9, ne = nf, nl = 3 * (nf + 1), nk = nu + ne;
      std::vector<double> Ce((size_t)ne * 9), Al((size_t)nl * 9);
      for (int r = 0; r < ne; ++r) row9(i, nbr[i][r], &Ce[(size_t)r * 9]);
      int mem[7];
      mem[0] = i;
      for (int k = 0; k < nf; ++k) mem[1 + k] = nbr[i][k];
      double hk[7];
      for (int k = 0; k <= nf; ++k) {
        int e = mem[k];
        hk[k] = hx[e];
        Vec3 d = (1.0 / hx[i]) * (cx[e] - cx[i]);
        double rows[3][9] = {{1, 0, 0, 2 * d.x, 0, 0, d.y, d.z, 0},
                             {0, 1, 0, 0, 2 * d.y, 0, d.x, 0, d.z},
                             {0, 0, 1, 0, 0, 2 * d.z, 0, d.x, d.y}};
        for (int a = 0; a < 3; ++a)
          for (int q = 0; q < 9; ++q) Al[(size_t)(3 * k + a) * 9 + q] = hk[k] * rows[a][q] / hx[i];
      }
      std::vector<double> K((size_t)nk * nk, 0.0), Ki;
      for (int p = 0; p < nu; ++p) {
        for (int q = 0; q < nu; ++q) {
          double s = 0.0;
          for (int r = 0; r < nl; ++r) s += Al[(size_t)r * 9 + p] * Al[(size_t)r * 9 + q];
          K[p * nk + q] = 2.0 * s;
        }
        for (int r = 0; r < ne; ++r) {
          K[p * nk + nu + r] = Ce[(size_t)r * 9 + p];
          K[(nu + r) * nk + p] = Ce[(size_t)r * 9 + p];
        }
      }
      invert(K, nk, Ki);
      // a = Ki[0:9, 0:9] 2 Al^T (h G) + Ki[0:9, 9:9+nf] dQ; rows j < nf the
      // neighbour differences, then the own and the neighbours' gradients
      for (int k = 0; k < 9; ++k) {
        for (int j = 0; j < nf; ++j) H.opH[(size_t)(k * nhrow + j) * N + i] = Ki[k * nk + nu + j];
        for (int mk = 0; mk <= nf; ++mk)
          for (int a = 0; a < 3; ++a) {
            int row = 3 * mk + a;
            double s = 0.0;
            for (int q = 0; q < nu; ++q) s += Ki[k * nk + q] * 2.0 * Al[(size_t)row * 9 + q];
            s *= hk[mk];
            int j = nf + 3 * mk + a;
            H.opH[(size_t)(k * nhrow + j) * N + i] = s;
          }
      }
      for (int s = 0; s < nf; ++s) {
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
  // local face p is the one opposite local vertex p
  auto nodes_of = [&](int i, int p) {
    std::array<int, 3> k;
    int q = 0;
    for (int c = 0; c < 4; ++c)
      if (c != p) k[q++] = tet2node[4 * (size_t)i + c];
    return k;
  };
  std::vector<FaceTmp> ft;
  int nb_found = 0;
  int rc = pair_faces<3>(N, 4, nodes_of, n_bf, bf, btag, ft, nb_found, err);
  if (rc) return rc;
  auto geo = [&](const FaceTmp& t, FaceGeo& G) {
    std::array<int, 3> k = nodes_of(t.L, t.pL);
    Vec3 v[3] = {P(k[0]), P(k[1]), P(k[2])};
    Vec3 nn = crossp(v[1] - v[0], v[2] - v[0]);
    double len = std::sqrt(dotp(nn, nn));
    if (!(len > 0.0)) return false;
    G.S = 0.5 * len;
    G.n = (1.0 / len) * nn;
    G.xc = (1.0 / 3.0) * ((v[0] + v[1]) + v[2]);
    for (int q = 0; q < 3; ++q) G.gp[q] = (2.0 / 3.0) * v[q] + (1.0 / 6.0) * (v[(q + 1) % 3] + v[(q + 2) % 3]);
    return true;
  };
  return finish_mesh(H, cen, m2, ft, nb_found, geo, err);
}

int build_host_hex_mesh(HostMesh& H, int64_t n_nodes, const double* xyz, int64_t n_hex, const int32_t* hex2node,
                        int64_t n_bf, const int32_t* bf, const int32_t* btag, std::string& err) {
  if (n_nodes <= 0 || n_hex <= 0 || !xyz || !hex2node || n_hex > (int64_t)1 << 29) {
    err = "invalid mesh arguments";
    return -1;
  }
  const int N = (int)n_hex;
  H = HostMesh();
  H.N = N;
  H.nf = 6;
  H.ng = 4;
  H.nsw = 8;
  H.msw = 3;
  auto P = [&](int node) { return Vec3{xyz[3 * (size_t)node], xyz[3 * (size_t)node + 1], xyz[3 * (size_t)node + 2]}; };
  // reference corners (r, s, t) of the node order; 3-point Gauss-Legendre
  // per direction integrates volume, centroid and second moments of the
  // trilinear cell exactly
  static const int rc3[8][3] = {{0, 0, 0}, {1, 0, 0}, {1, 1, 0}, {0, 1, 0}, {0, 0, 1}, {1, 0, 1}, {1, 1, 1}, {0, 1, 1}};
  const double gx[3] = {0.5 - 0.5 * std::sqrt(0.6), 0.5, 0.5 + 0.5 * std::sqrt(0.6)};
  const double gw[3] = {5.0 / 18.0, 8.0 / 18.0, 5.0 / 18.0};
  std::vector<Vec3> cen(N);
  std::vector<Sym3> m2(N);
  H.vol.resize(N);
  for (int i = 0; i < N; ++i) {
    Vec3 v[8];
    for (int k = 0; k < 8; ++k) {
      int nd = hex2node[8 * (size_t)i + k];
      if (nd < 0 || nd >= n_nodes) {
        err = "hex node id out of range at hex " + std::to_string(i);
        return -3;
      }
      v[k] = P(nd);
    }
    auto map = [&](double r, double s, double t, Vec3& x) {
      Vec3 dr{0, 0, 0}, ds{0, 0, 0}, dt{0, 0, 0};
      x = Vec3{0, 0, 0};
      for (int k = 0; k < 8; ++k) {
        double fr = rc3[k][0] ? r : 1.0 - r, fs = rc3[k][1] ? s : 1.0 - s, ftt = rc3[k][2] ? t : 1.0 - t;
        double sr = rc3[k][0] ? 1.0 : -1.0, ss = rc3[k][1] ? 1.0 : -1.0, st = rc3[k][2] ? 1.0 : -1.0;
        x = x + (fr * fs * ftt) * v[k];
        dr = dr + (sr * fs * ftt) * v[k];
        ds = ds + (fr * ss * ftt) * v[k];
        dt = dt + (fr * fs * st) * v[k];
      }
      return dotp(crossp(dr, ds), dt);
    };
    bool ok = true;
    Vec3 x;
    for (int k = 0; k < 8; ++k) {
      double J = map(rc3[k][0], rc3[k][1], rc3[k][2], x);
      if (!(J > 0.0) || !std::isfinite(J)) ok = false;
    }
    double vol = 0.0;
    Vec3 c{0, 0, 0};
    Vec3 px[27];
    double pw[27];
    int np = 0;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b)
        for (int d = 0; d < 3; ++d) {
          double J = map(gx[a], gx[b], gx[d], x);
          if (!(J > 0.0)) ok = false;
          pw[np] = gw[a] * gw[b] * gw[d] * J;
          px[np] = x;
          vol += pw[np];
          c = c + pw[np] * x;
          ++np;
        }
    if (!ok) {
      err = "inverted or degenerate hexahedron " + std::to_string(i);
      return -3;
    }
    c = (1.0 / vol) * c;
    Sym3 s;
    std::memset(&s, 0, sizeof(s));
    for (int q = 0; q < 27; ++q) {
      Vec3 d = px[q] - c;
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) s.a[a][b] += pw[q] * comp(d, a) * comp(d, b) / vol;
    }
    H.vol[i] = vol;
    cen[i] = c;
    m2[i] = s;
  }
  // local faces F1..F6 = 0..5: bottom, the four sides in order around, top;
  // node lists counter-clockwise seen from outside
  static const int fq[6][4] = {{0, 3, 2, 1}, {0, 1, 5, 4}, {1, 2, 6, 5}, {2, 3, 7, 6}, {3, 0, 4, 7}, {4, 5, 6, 7}};
  auto nodes_of = [&](int i, int p) {
    std::array<int, 4> k;
    for (int q = 0; q < 4; ++q) k[q] = hex2node[8 * (size_t)i + fq[p][q]];
    return k;
  };
  std::vector<FaceTmp> ft;
  int nb_found = 0;
  int rc = pair_faces<4>(N, 6, nodes_of, n_bf, bf, btag, ft, nb_found, err);
  if (rc) return rc;
  const double q0 = 0.5 - 0.5 / std::sqrt(3.0), q1 = 0.5 + 0.5 / std::sqrt(3.0);
  const double quv[4][2] = {{q0, q0}, {q1, q0}, {q1, q1}, {q0, q1}};
  // bilinear face: exact vector area (x_c - x_a) x (x_d - x_b) / 2; 2x2 Gauss
  // points weighted by the normal component of the area element
  auto geo = [&](const FaceTmp& t, FaceGeo& G) {
    std::array<int, 4> k = nodes_of(t.L, t.pL);
    Vec3 a = P(k[0]), b = P(k[1]), c = P(k[2]), d = P(k[3]);
    Vec3 sv = 0.5 * crossp(c - a, d - b);
    G.S = std::sqrt(dotp(sv, sv));
    if (!(G.S > 0.0)) return false;
    G.n = (1.0 / G.S) * sv;
    Vec3 xc{0, 0, 0};
    for (int q = 0; q < 4; ++q) {
      double u = quv[q][0], w = quv[q][1];
      G.gp[q] = (((1 - u) * (1 - w)) * a + (u * (1 - w)) * b) + ((u * w) * c + ((1 - u) * w) * d);
      Vec3 xu = (1 - w) * (b - a) + w * (c - d);
      Vec3 xw = (1 - u) * (d - a) + u * (c - b);
      G.gw[q] = 0.25 * dotp(crossp(xu, xw), G.n) / G.S;
      xc = xc + G.gw[q] * G.gp[q];
    }
    G.xc = xc;
    return true;
  };
  return finish_mesh(H, cen, m2, ft, nb_found, geo, err);
}

int colour_cells(const HostMesh& H, std::vector<int>& col, std::vector<int>& order, std::vector<int>& start) {
  const int N = H.N;
  col.assign(N, -1);
  int ncol = 0;
  for (int i = 0; i < N; ++i) {
    unsigned taken = 0;  // bit c: a coloured neighbour has colour c
    for (int k = 0; k < H.nf; ++k) {
      int j = H.nbf[(size_t)k * N + i];
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
