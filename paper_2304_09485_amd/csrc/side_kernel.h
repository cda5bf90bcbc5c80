// Face-side kernel: characteristic WENO of Sec. 3.4 Eq. (weno) with the
// characteristic projection of Sec. 5, values and (n, t1, t2) derivatives at
// the 3 Gauss points of the face, back-projected to conservative variables in
// the face's local frame.
//
// Five lanes per face side, one per characteristic component c: each lane
// projects the 21 coefficient vectors of the side's cell onto its component,
// computes the smoothness indicators and weights and evaluates the combined
// polynomial (12 values).  The back-projection R* mixes components, so the
// lanes exchange their 12 values through LDS and lane c then produces
// conservative variable c.  12 sides per 64-lane block.
// sv layout [60][2F], row (g*4+d)*5+v, column side*F+f.
// Included inside namespace hgks of hgks_kernels.hip.
#pragma once

constexpr int SIDE_SPB = 12;

template <typename T>
__device__ __forceinline__ T pick5(int c, T a0, T a1, T a2, T a3, T a4) {
  return c == 0 ? a0 : (c == 1 ? a1 : (c == 2 ? a2 : (c == 3 ? a3 : a4)));
}

template <typename T>
__global__ void __launch_bounds__(64) k_side(DevMesh<T> M, Params P, const T* __restrict__ Qx,
                                             const T* __restrict__ coef, T* __restrict__ sv,
                                             int* __restrict__ nfall) {
  __shared__ T s_val[SIDE_SPB][5][12];
  __shared__ T s_out[SIDE_SPB][5][12];
  __shared__ int s_bad[SIDE_SPB];
  const int F = M.F, N = M.N, NX = M.NX;
  const int lane = threadIdx.x;
  const int sl = lane / 5, c = lane % 5;  // side slot in the block; component / output variable
  const bool in_block = lane < 5 * SIDE_SPB;
  const int sidx = blockIdx.x * SIDE_SPB + sl;
  bool active = false;
  int side = 0, f = 0, i = 0, j = 0;
  if (in_block && sidx < 2 * F) {
    side = sidx >= F;
    f = side ? sidx - F : sidx;
    int L = M.fL[f], R = M.fR[f];
    active = !(side && R >= N);  // boundary faces have no reconstructed right side
    i = side ? R : L;
    j = side ? L : R;
  }
  if (lane < SIDE_SPB) s_bad[lane] = 0;
  const T g = T(P.gamma);
  T val[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) val[k] = T(0);
  T Rrow[5] = {0, 0, 0, 0, 0};  // row c of R*: conservative variable c from the components
  T qil_c = T(0);               // local-frame cell average, variable c (fallback)
  if (active) {
    T e[3][3];
    e[0][0] = M.fn[f];
    e[0][1] = M.fn[F + f];
    e[0][2] = M.fn[2 * F + f];
    face_frame(e[0][0], e[0][1], e[0][2], e[1], e[2]);
    T qi[5], qj[5], qil[5], qs[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      qi[v] = Qx[(size_t)v * NX + i];
      qj[v] = Qx[(size_t)v * NX + j];
    }
    qil[0] = qi[0];
    qil[4] = qi[4];
#pragma unroll
    for (int a = 0; a < 3; ++a) qil[1 + a] = e[a][0] * qi[1] + e[a][1] * qi[2] + e[a][2] * qi[3];
    qs[0] = T(0.5) * (qi[0] + qj[0]);
    qs[4] = T(0.5) * (qi[4] + qj[4]);
#pragma unroll
    for (int a = 0; a < 3; ++a)
      qs[1 + a] = T(0.5) * (qil[1 + a] + (e[a][0] * qj[1] + e[a][1] * qj[2] + e[a][2] * qj[3]));
    qil_c = pick5(c, qil[0], qil[1], qil[2], qil[3], qil[4]);
    // eigenvectors of the x-split Euler Jacobian at Q* (local frame), columns
    // (u-c, u, u, u, u+c): row c of R* and row c of L* = R*^{-1}
    T rho = qs[0], u = qs[1] / rho, vv = qs[2] / rho, w = qs[3] / rho;
    T q2 = u * u + vv * vv + w * w;
    T p = (g - T(1)) * (qs[4] - T(0.5) * rho * q2);
    T cs = sqrt(g * p / rho);
    T H = (qs[4] + p) / rho;
    T b1 = (g - T(1)) / (cs * cs), b2 = T(0.5) * b1 * q2, ic = T(1) / cs;
    Rrow[0] = pick5(c, T(1), u - cs, vv, w, H - u * cs);
    Rrow[1] = pick5(c, T(1), u, vv, w, T(0.5) * q2);
    Rrow[2] = pick5(c, T(0), T(0), T(1), T(0), vv);
    Rrow[3] = pick5(c, T(0), T(0), T(0), T(1), w);
    Rrow[4] = pick5(c, T(1), u + cs, vv, w, H + u * cs);
    T Lr[5];
    Lr[0] = pick5(c, T(0.5) * (b2 + u * ic), T(1) - b2, -vv, -w, T(0.5) * (b2 - u * ic));
    Lr[1] = pick5(c, T(0.5) * (-b1 * u - ic), b1 * u, T(0), T(0), T(0.5) * (-b1 * u + ic));
    Lr[2] = pick5(c, T(-0.5) * b1 * vv, b1 * vv, T(1), T(0), T(-0.5) * b1 * vv);
    Lr[3] = pick5(c, T(-0.5) * b1 * w, b1 * w, T(0), T(1), T(-0.5) * b1 * w);
    Lr[4] = pick5(c, T(0.5) * b1, -b1, T(0), T(0), T(0.5) * b1);
    // row c of T = L* . Rot (global conservative -> characteristic)
    T tc[5];
    tc[0] = Lr[0];
    tc[4] = Lr[4];
#pragma unroll
    for (int d = 0; d < 3; ++d) tc[1 + d] = Lr[1] * e[0][d] + Lr[2] * e[1][d] + Lr[3] * e[2][d];
    T q0 = tc[0] * qi[0] + tc[1] * qi[1] + tc[2] * qi[2] + tc[3] * qi[3] + tc[4] * qi[4];
    T a[9], b[4][3];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const T* cp = coef + (size_t)(k * 5) * N + i;
      a[k] = tc[0] * cp[0] + tc[1] * cp[N] + tc[2] * cp[2 * N] + tc[3] * cp[3 * N] + tc[4] * cp[4 * N];
    }
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        const T* cp = coef + (size_t)((9 + s * 3 + t) * 5) * N + i;
        b[s][t] = tc[0] * cp[0] + tc[1] * cp[N] + tc[2] * cp[2 * N] + tc[3] * cp[3 * N] + tc[4] * cp[4 * N];
      }
    T m2[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) m2[k] = M.m2s[k * N + i];
    unsigned mask = P.scheme == 1 ? 15u : (unsigned)M.smask[i];
    int nsub = __popc(mask);
    const T gl = T(P.gamma_lin);
    const T g0 = T(1) - gl * T(nsub);
    T w0, ws[4];
    if (P.weights == 1) {
      w0 = g0;
#pragma unroll
      for (int s = 0; s < 4; ++s) ws[s] = (mask >> s) & 1u ? gl : T(0);
    } else {
      // smoothness indicators (scaled basis: the |Omega| powers cancel)
      T s0[3] = {T(2) * a[3], a[6], a[7]}, s1[3] = {a[6], T(2) * a[4], a[8]}, s2[3] = {a[7], a[8], T(2) * a[5]};
      auto quad = [&](const T* x) {
        return m2[0] * x[0] * x[0] + m2[1] * x[1] * x[1] + m2[2] * x[2] * x[2] +
               T(2) * (m2[3] * x[0] * x[1] + m2[4] * x[0] * x[2] + m2[5] * x[1] * x[2]);
      };
      T beta0 = a[0] * a[0] + quad(s0) + a[1] * a[1] + quad(s1) + a[2] * a[2] + quad(s2) +
                T(4) * (a[3] * a[3] + a[4] * a[4] + a[5] * a[5]) + a[6] * a[6] + a[7] * a[7] + a[8] * a[8];
      T bm[4], tz = T(0);
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        bm[s] = b[s][0] * b[s][0] + b[s][1] * b[s][1] + b[s][2] * b[s][2];
        if ((mask >> s) & 1u) tz += fabs(beta0 - bm[s]);
      }
      if (nsub > 0) tz /= T(nsub);
      const T eps = T(P.weno_eps);
      T wt0 = g0 * (T(1) + tz / (beta0 + eps));
      T sum = wt0;
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        ws[s] = (mask >> s) & 1u ? gl * (T(1) + tz / (bm[s] + eps)) : T(0);
        sum += ws[s];
      }
      T isum = T(1) / sum;
      w0 = wt0 * isum;
#pragma unroll
      for (int s = 0; s < 4; ++s) ws[s] *= isum;
    }
    // combined polynomial: q0 + Lc . xi + Qc . (xi xi - m2)
    T r0 = w0 / g0;
    T Lc[3], Qc[6];
#pragma unroll
    for (int t = 0; t < 3; ++t) Lc[t] = r0 * a[t];
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      if (!((mask >> s) & 1u)) continue;
      T cw = ws[s] - w0 * gl / g0;
#pragma unroll
      for (int t = 0; t < 3; ++t) Lc[t] += cw * b[s][t];
    }
#pragma unroll
    for (int t = 0; t < 6; ++t) Qc[t] = r0 * a[3 + t];
    const T* xis = side ? M.fxiR : M.fxiL;
    const T ih = T(1) / M.h[i];
#pragma unroll
    for (int gp = 0; gp < 3; ++gp) {
      T x0 = xis[(size_t)(gp * 3 + 0) * F + f], x1 = xis[(size_t)(gp * 3 + 1) * F + f];
      T x2 = xis[(size_t)(gp * 3 + 2) * F + f];
      val[gp * 4 + 0] = q0 + Lc[0] * x0 + Lc[1] * x1 + Lc[2] * x2 + Qc[0] * (x0 * x0 - m2[0]) +
                        Qc[1] * (x1 * x1 - m2[1]) + Qc[2] * (x2 * x2 - m2[2]) + Qc[3] * (x0 * x1 - m2[3]) +
                        Qc[4] * (x0 * x2 - m2[4]) + Qc[5] * (x1 * x2 - m2[5]);
      T gx = Lc[0] + T(2) * Qc[0] * x0 + Qc[3] * x1 + Qc[4] * x2;
      T gy = Lc[1] + T(2) * Qc[1] * x1 + Qc[3] * x0 + Qc[5] * x2;
      T gz = Lc[2] + T(2) * Qc[2] * x2 + Qc[4] * x0 + Qc[5] * x1;
#pragma unroll
      for (int a2 = 0; a2 < 3; ++a2) val[gp * 4 + 1 + a2] = (gx * e[a2][0] + gy * e[a2][1] + gz * e[a2][2]) * ih;
    }
  }
  if (in_block)
#pragma unroll
    for (int k = 0; k < 12; ++k) s_val[sl][c][k] = val[k];
  __syncthreads();
  // back projection: conservative variable c = sum over components of R*[c][.]
  T out[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    out[k] = T(0);
    if (in_block)
#pragma unroll
      for (int cc = 0; cc < 5; ++cc) out[k] += Rrow[cc] * s_val[sl][cc][k];
  }
  if (in_block)
#pragma unroll
    for (int k = 0; k < 12; ++k) s_out[sl][c][k] = out[k];
  __syncthreads();
  // positivity of the Gauss-point states; fallback to first order on this side
  if (active && c == 0) {
    bool bad = false;
#pragma unroll
    for (int gp = 0; gp < 3; ++gp) {
      T wv[5] = {s_out[sl][0][gp * 4], s_out[sl][1][gp * 4], s_out[sl][2][gp * 4], s_out[sl][3][gp * 4],
                 s_out[sl][4][gp * 4]};
      if (!phys_ok(wv, g)) bad = true;
    }
    if (bad) {
      s_bad[sl] = 1;
      atomicAdd(nfall, 1);
    }
  }
  __syncthreads();
  if (!active) return;
  const bool bad = s_bad[sl] != 0;
  const size_t ld = 2 * (size_t)F;
#pragma unroll
  for (int gp = 0; gp < 3; ++gp)
#pragma unroll
    for (int d = 0; d < 4; ++d) {
      T o = bad ? (d == 0 ? qil_c : T(0)) : out[gp * 4 + d];
      sv[(size_t)((gp * 4 + d) * 5 + c) * ld + sidx] = o;
    }
}
