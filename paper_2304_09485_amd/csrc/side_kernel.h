// Face-side kernel: characteristic WENO of Sec. 3.4 Eq. (weno) with the
// characteristic projection of Sec. 5, values and (n, t1, t2) derivatives at
// the NG Gauss points of the face (3 on a triangle, 4 on a quadrilateral),
// back-projected to conservative variables in the face's local frame.  One
// lane per face side; the 5 characteristic components are taken in turn
// (projection of the side cell's 9 + 3 NSUB coefficient vectors, smoothness
// indicators, nonlinear weights, combined polynomial at the Gauss points) and
// accumulated into the 20 NG outputs through R*.  NSUB: 4 sub-stencils on a
// tetrahedron, 8 (non-compact) or 6 (compact) on a hexahedron.
// sv layout [20 NG][2F], row (g*4+d)*5+v, column side*F+f.
// Included inside namespace hgks of hgks_kernels.hip.
#pragma once

constexpr int SIDE_SPB = 128;      // face sides per block
constexpr int SIDE_THREADS = 128;  // threads per block

// LPS lanes per side: 1 (each lane evaluates all NG Gauss points), or NG
// (each lane one Gauss point; the projection and the weights are repeated
// per lane, the live output shrinks from 20 NG to 20 values, and the
// positivity decision is shared by the side's lanes through a ballot).
template <typename T, int NSUB, int NG, int LPS>
__global__ void __launch_bounds__(128) k_side(DevMesh<T> M, Params P, const T* __restrict__ Qx,
                                              const T* __restrict__ coef, T* __restrict__ sv,
                                              int* __restrict__ nfall) {
  constexpr int NGL = NG / LPS;  // Gauss points of this lane
  const int tid = xcd_block() * blockDim.x + threadIdx.x;  // contiguous side ranges per XCD
  int sidx = tid / LPS;
  const int g_lo = (tid % LPS) * NGL;
  const int F = M.F, N = M.N, NX = M.NX;
  if (sidx >= 2 * F) return;  // whole lane groups (LPS divides the block)
  int side = sidx >= F;
  int f = side ? sidx - F : sidx;
  int L = M.fL[f], R = M.fR[f];
  if (side && R >= N) return;
  int i = side ? R : L, j = side ? L : R;
  const T g = T(P.gamma);
  T e[3][3];
  e[0][0] = M.fn[f];
  e[0][1] = M.fn[F + f];
  e[0][2] = M.fn[2 * F + f];
  face_frame(e[0][0], e[0][1], e[0][2], e[1], e[2]);
  T qi[5], qj[5], qil[5], qs[5];
  for (int v = 0; v < 5; ++v) {
    qi[v] = Qx[(size_t)v * NX + i];
    qj[v] = Qx[(size_t)v * NX + j];
  }
  qil[0] = qi[0];
  qil[4] = qi[4];
  for (int a = 0; a < 3; ++a) qil[1 + a] = e[a][0] * qi[1] + e[a][1] * qi[2] + e[a][2] * qi[3];
  qs[0] = T(0.5) * (qi[0] + qj[0]);
  qs[4] = T(0.5) * (qi[4] + qj[4]);
  for (int a = 0; a < 3; ++a)
    qs[1 + a] = T(0.5) * (qil[1 + a] + (e[a][0] * qj[1] + e[a][1] * qj[2] + e[a][2] * qj[3]));
  // right/left eigenvectors of the x-split Euler Jacobian at Q* (local frame),
  // columns (u-c, u, u, u, u+c)
  T rho = qs[0], u = qs[1] / rho, vv = qs[2] / rho, w = qs[3] / rho;
  T q2 = u * u + vv * vv + w * w;
  T p = (g - T(1)) * (qs[4] - T(0.5) * rho * q2);
  T c = sqrt(g * p / rho);
  T H = (qs[4] + p) / rho;
  const T b1 = (g - T(1)) / (c * c), b2 = T(0.5) * b1 * q2, ic = T(1) / c;
  const T hh = M.h[i];
  const T ih = T(1) / hh;
  T m2[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) m2[k] = M.m2s[k * N + i];
  const T* xis = side ? M.fxiR : M.fxiL;
  T xi[NGL][3];
#pragma unroll
  for (int k = 0; k < 3 * NGL; ++k) xi[k / 3][k % 3] = xis[(size_t)(3 * g_lo + k) * F + f];
  unsigned mask = P.scheme == 1 ? (1u << NSUB) - 1u : (unsigned)M.smask[i];
  int nsub = __popc(mask);
  const T gl = T(P.gamma_lin);
  const T g0 = T(1) - gl * T(nsub);
  T out[NGL][4][5];
#pragma unroll
  for (int a = 0; a < NGL; ++a)
#pragma unroll
    for (int d = 0; d < 4; ++d)
#pragma unroll
      for (int v = 0; v < 5; ++v) out[a][d][v] = T(0);
  for (int cc = 0; cc < 5; ++cc) {
    // row cc of L* = R*^{-1} and column cc of R* (x-split Euler eigenvectors
    // at Q*, columns u-c, u, u, u, u+c), built from the eigen-system scalars
    // (no per-lane matrices: indexing those by cc would put them in scratch)
    T l[5], r[5];
    switch (cc) {
      case 0:
        l[0] = T(0.5) * (b2 + u * ic); l[1] = T(0.5) * (-b1 * u - ic); l[2] = T(-0.5) * b1 * vv;
        l[3] = T(-0.5) * b1 * w; l[4] = T(0.5) * b1;
        r[0] = T(1); r[1] = u - c; r[2] = vv; r[3] = w; r[4] = H - u * c;
        break;
      case 1:
        l[0] = T(1) - b2; l[1] = b1 * u; l[2] = b1 * vv; l[3] = b1 * w; l[4] = -b1;
        r[0] = T(1); r[1] = u; r[2] = vv; r[3] = w; r[4] = T(0.5) * q2;
        break;
      case 2:
        l[0] = -vv; l[1] = T(0); l[2] = T(1); l[3] = T(0); l[4] = T(0);
        r[0] = T(0); r[1] = T(0); r[2] = T(1); r[3] = T(0); r[4] = vv;
        break;
      case 3:
        l[0] = -w; l[1] = T(0); l[2] = T(0); l[3] = T(1); l[4] = T(0);
        r[0] = T(0); r[1] = T(0); r[2] = T(0); r[3] = T(1); r[4] = w;
        break;
      default:
        l[0] = T(0.5) * (b2 - u * ic); l[1] = T(0.5) * (-b1 * u + ic); l[2] = T(-0.5) * b1 * vv;
        l[3] = T(-0.5) * b1 * w; l[4] = T(0.5) * b1;
        r[0] = T(1); r[1] = u + c; r[2] = vv; r[3] = w; r[4] = H + u * c;
        break;
    }
    // row cc of T = L* . Rot
    T tc[5];
    tc[0] = l[0];
    tc[4] = l[4];
#pragma unroll
    for (int d = 0; d < 3; ++d) tc[1 + d] = l[1] * e[0][d] + l[2] * e[1][d] + l[3] * e[2][d];
    T q0 = tc[0] * qi[0] + tc[1] * qi[1] + tc[2] * qi[2] + tc[3] * qi[3] + tc[4] * qi[4];
    T a[9], b[NSUB][3];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const T* cp = coef + (size_t)(k * 5) * N + i;
      a[k] = tc[0] * cp[0] + tc[1] * cp[N] + tc[2] * cp[2 * N] + tc[3] * cp[3 * N] + tc[4] * cp[4 * N];
    }
#pragma unroll
    for (int s = 0; s < NSUB; ++s)
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        const T* cp = coef + (size_t)((9 + s * 3 + t) * 5) * N + i;
        b[s][t] = tc[0] * cp[0] + tc[1] * cp[N] + tc[2] * cp[2 * N] + tc[3] * cp[3 * N] + tc[4] * cp[4 * N];
      }
    // weights
    T w0, ws[NSUB];
    if (P.weights == 1) {
      w0 = g0;
#pragma unroll
      for (int s = 0; s < NSUB; ++s) ws[s] = (mask >> s) & 1u ? gl : T(0);
    } else {
      T s0[3] = {T(2) * a[3], a[6], a[7]}, s1[3] = {a[6], T(2) * a[4], a[8]}, s2[3] = {a[7], a[8], T(2) * a[5]};
      auto quad = [&](const T* sv3) {
        return m2[0] * sv3[0] * sv3[0] + m2[1] * sv3[1] * sv3[1] + m2[2] * sv3[2] * sv3[2] +
               T(2) * (m2[3] * sv3[0] * sv3[1] + m2[4] * sv3[0] * sv3[2] + m2[5] * sv3[1] * sv3[2]);
      };
      T beta0 = a[0] * a[0] + quad(s0) + a[1] * a[1] + quad(s1) + a[2] * a[2] + quad(s2) +
                T(4) * (a[3] * a[3] + a[4] * a[4] + a[5] * a[5]) + a[6] * a[6] + a[7] * a[7] + a[8] * a[8];
      T bm[NSUB], tz = T(0);
#pragma unroll
      for (int s = 0; s < NSUB; ++s) {
        bm[s] = b[s][0] * b[s][0] + b[s][1] * b[s][1] + b[s][2] * b[s][2];
        if ((mask >> s) & 1u) tz += fabs(beta0 - bm[s]);
      }
      if (nsub > 0) tz /= T(nsub);
      const T eps = T(P.weno_eps);
      T wt0 = g0 * (T(1) + tz / (beta0 + eps));
      T sum = wt0;
#pragma unroll
      for (int s = 0; s < NSUB; ++s) {
        ws[s] = (mask >> s) & 1u ? gl * (T(1) + tz / (bm[s] + eps)) : T(0);
        sum += ws[s];
      }
      T isum = T(1) / sum;
      w0 = wt0 * isum;
#pragma unroll
      for (int s = 0; s < NSUB; ++s) ws[s] *= isum;
    }
    // combined polynomial: q0 + Lc . xi + Qc . (xi xi - m2)
    T r0 = w0 / g0;
    T Lc[3], Qc[6];
#pragma unroll
    for (int t = 0; t < 3; ++t) Lc[t] = r0 * a[t];
#pragma unroll
    for (int s = 0; s < NSUB; ++s) {
      if (!((mask >> s) & 1u)) continue;
      T cs = ws[s] - w0 * gl / g0;
#pragma unroll
      for (int t = 0; t < 3; ++t) Lc[t] += cs * b[s][t];
    }
#pragma unroll
    for (int t = 0; t < 6; ++t) Qc[t] = r0 * a[3 + t];
#pragma unroll
    for (int gp = 0; gp < NGL; ++gp) {
      T x0 = xi[gp][0], x1 = xi[gp][1], x2 = xi[gp][2];
      T val = q0 + Lc[0] * x0 + Lc[1] * x1 + Lc[2] * x2 + Qc[0] * (x0 * x0 - m2[0]) +
              Qc[1] * (x1 * x1 - m2[1]) + Qc[2] * (x2 * x2 - m2[2]) + Qc[3] * (x0 * x1 - m2[3]) +
              Qc[4] * (x0 * x2 - m2[4]) + Qc[5] * (x1 * x2 - m2[5]);
      T gx = Lc[0] + T(2) * Qc[0] * x0 + Qc[3] * x1 + Qc[4] * x2;
      T gy = Lc[1] + T(2) * Qc[1] * x1 + Qc[3] * x0 + Qc[5] * x2;
      T gz = Lc[2] + T(2) * Qc[2] * x2 + Qc[4] * x0 + Qc[5] * x1;
      T dd[4];
      dd[0] = val;
#pragma unroll
      for (int a2 = 0; a2 < 3; ++a2) dd[1 + a2] = (gx * e[a2][0] + gy * e[a2][1] + gz * e[a2][2]) * ih;
#pragma unroll
      for (int d = 0; d < 4; ++d)
#pragma unroll
        for (int v = 0; v < 5; ++v) out[gp][d][v] += r[v] * dd[d];
    }
  }
  bool ok = true;
#pragma unroll
  for (int gp = 0; gp < NGL; ++gp) ok = ok && phys_ok(out[gp][0], g);
  if (LPS > 1) {
    // the side falls back if any of its lanes' Gauss points is non-physical
    const unsigned long long bad = __ballot(!ok);
    const int lane0 = (int)(__lane_id() & ~(unsigned)(LPS - 1));
    ok = ((bad >> lane0) & ((1ull << LPS) - 1ull)) == 0ull;
  }
  if (!ok) {
    // positivity fallback: first order on this side
    if (g_lo == 0) atomicAdd(nfall, 1);
    for (int gp = 0; gp < NGL; ++gp) {
      for (int v = 0; v < 5; ++v) out[gp][0][v] = qil[v];
      for (int d = 1; d < 4; ++d)
        for (int v = 0; v < 5; ++v) out[gp][d][v] = T(0);
    }
  }
  const size_t ld = 2 * (size_t)F;
#pragma unroll
  for (int gp = 0; gp < NGL; ++gp)
#pragma unroll
    for (int d = 0; d < 4; ++d)
#pragma unroll
      for (int v = 0; v < 5; ++v) sv[(size_t)(((g_lo + gp) * 4 + d) * 5 + v) * ld + sidx] = out[gp][d][v];
}

