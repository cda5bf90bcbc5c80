// Face-side kernel: characteristic WENO of Sec. 3.4 Eq. (weno) with the
// characteristic projection of Sec. 5, values and (n, t1, t2) derivatives at
// the NG Gauss points of the face (3 on a triangle, 4 on a quadrilateral),
// back-projected to conservative variables in the face's local frame.  One
// lane per face side; the 5 characteristic components are taken in turn
// (projection of the side cell's 9 + 3 NSUB coefficient vectors, smoothness
// indicators, nonlinear weights, combined polynomial).  Each component's
// combined polynomial is kept as 10 numbers in LDS (the lane's own column,
// no sharing between lanes), and the 20 NG outputs are formed from them
// through R* after the component loop, so that no output accumulators are
// live while the 105 coefficients are.  NSUB: 4 sub-stencils on a
// tetrahedron, 8 (non-compact) or 6 (compact) on a hexahedron.
// sv layout [20 NG][2F], row (g*4+d)*5+v, column side*F+f.
// Included inside namespace hgks of hgks_kernels.hip.
#pragma once

// Element i of row r of a row-major [rows][N] array, read through a buffer
// resource whose base is the row (uniform, scalar registers) and a 32-bit
// per-lane byte offset (a single VGPR shared by all rows), so that no 64-bit
// address per row is formed or held in vector registers.  The resource's
// range is the row: an offset past it reads 0 instead of faulting.
template <typename T>
__device__ __forceinline__ T row_elem(const T* __restrict__ row0, size_t r, int N, unsigned boff) {
  // word 3 of the buffer resource for gfx9-family (CDNA) parts: raw 32-bit
  // data, no swizzle
  const __amdgpu_buffer_rsrc_t rs =
      __builtin_amdgcn_make_buffer_rsrc((void*)(row0 + r * (size_t)N), (short)0, N * (int)sizeof(T), 0x00020000);
  if constexpr (sizeof(T) == 8)
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b64(rs, boff, 0, 0));
  else
    return __builtin_bit_cast(T, __builtin_amdgcn_raw_buffer_load_b32(rs, boff, 0, 0));
}

constexpr int SIDE_SPB = 128;      // face sides per block
constexpr int SIDE_THREADS = 128;  // threads per block

// LPS lanes per side: 1 (each lane evaluates all NG Gauss points; the form
// launched for triangles and quadrilaterals), or NG (each lane one Gauss
// point; the projection and the weights are repeated per lane, and the
// positivity decision is shared by the side's lanes through a ballot).
template <typename T, int NSUB, int NG, int LPS>
__global__ void __launch_bounds__(128) k_side(DevMesh<T> M, Params P, const T* __restrict__ Qx,
                                              const T* __restrict__ coef, T* __restrict__ sv,
                                              int* __restrict__ nfall) {
  constexpr int NGL = NG / LPS;  // Gauss points of this lane
  const int tid = xcd_block() * blockDim.x + threadIdx.x;  // contiguous side ranges per XCD
  const int q = tid / LPS;
  const int g_lo = (tid % LPS) * NGL;
  const int F = M.F, N = M.N, NX = M.NX;
  if (q >= 2 * F) return;  // whole lane groups (LPS divides the block)
  // the two sides of a face are neighbouring lane groups, so that the side
  // cells' coefficients are read close together in time (the second read of
  // a cell's rows then tends to hit in L2)
  const int side = q & 1;
  const int f = q >> 1;
  const int sidx = side * F + f;
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
  unsigned mask = P.scheme == 1 && !P.csubs ? (1u << NSUB) - 1u : (unsigned)M.smask[i];
  int nsub = __popc(mask);
  const T gl = T(P.gamma_lin);
  const T g0 = T(1) - gl * T(nsub);
  // per characteristic component cc, the combined polynomial in the form
  // q0' + Lc . xi + Qc . (xi xi) with q0' = q0 - Qc . m2 (10 numbers); the
  // outputs are formed from these after the component loop
  __shared__ T pqs[50][SIDE_THREADS];  // [cc * 10 + k][lane of the block]
  const int lt = threadIdx.x;
  const unsigned cbo = (unsigned)i * (unsigned)sizeof(T);  // byte offset of the cell in a coefficient row
#pragma unroll 1
  for (int cc = 0; cc < 5; ++cc) {
    // row cc of L* = R*^{-1} (x-split Euler eigenvectors at Q*, columns
    // u-c, u, u, u, u+c), built from the eigen-system scalars
    T l[5];
    switch (cc) {
      case 0:
        l[0] = T(0.5) * (b2 + u * ic); l[1] = T(0.5) * (-b1 * u - ic); l[2] = T(-0.5) * b1 * vv;
        l[3] = T(-0.5) * b1 * w; l[4] = T(0.5) * b1;
        break;
      case 1:
        l[0] = T(1) - b2; l[1] = b1 * u; l[2] = b1 * vv; l[3] = b1 * w; l[4] = -b1;
        break;
      case 2:
        l[0] = -vv; l[1] = T(0); l[2] = T(1); l[3] = T(0); l[4] = T(0);
        break;
      case 3:
        l[0] = -w; l[1] = T(0); l[2] = T(0); l[3] = T(1); l[4] = T(0);
        break;
      default:
        l[0] = T(0.5) * (b2 - u * ic); l[1] = T(0.5) * (-b1 * u + ic); l[2] = T(-0.5) * b1 * vv;
        l[3] = T(-0.5) * b1 * w; l[4] = T(0.5) * b1;
        break;
    }
    // row cc of T = L* . Rot
    T tc[5];
    tc[0] = l[0];
    tc[4] = l[4];
#pragma unroll
    for (int d = 0; d < 3; ++d) tc[1 + d] = l[1] * e[0][d] + l[2] * e[1][d] + l[3] * e[2][d];
    T q0 = tc[0] * qi[0] + tc[1] * qi[1] + tc[2] * qi[2] + tc[3] * qi[3] + tc[4] * qi[4];
    auto co = [&](int r) { return row_elem(coef, (size_t)r, N, cbo); };
    T a[9], b[NSUB][3];
#pragma unroll
    for (int k = 0; k < 9; ++k)
      a[k] = tc[0] * co(k * 5) + tc[1] * co(k * 5 + 1) + tc[2] * co(k * 5 + 2) + tc[3] * co(k * 5 + 3) +
             tc[4] * co(k * 5 + 4);
#pragma unroll
    for (int s = 0; s < NSUB; ++s)
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        const int r = (9 + s * 3 + t) * 5;
        b[s][t] = tc[0] * co(r) + tc[1] * co(r + 1) + tc[2] * co(r + 2) + tc[3] * co(r + 3) + tc[4] * co(r + 4);
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
    pqs[cc * 10][lt] = q0 - (Qc[0] * m2[0] + Qc[1] * m2[1] + Qc[2] * m2[2] + Qc[3] * m2[3] + Qc[4] * m2[4] + Qc[5] * m2[5]);
#pragma unroll
    for (int t = 0; t < 3; ++t) pqs[cc * 10 + 1 + t][lt] = Lc[t];
#pragma unroll
    for (int t = 0; t < 6; ++t) pqs[cc * 10 + 4 + t][lt] = Qc[t];
  }
  // column cc of R* (conservative components of the characteristic mode cc)
  T rc[5][5];
  rc[0][0] = T(1); rc[0][1] = u - c; rc[0][2] = vv; rc[0][3] = w; rc[0][4] = H - u * c;
  rc[1][0] = T(1); rc[1][1] = u; rc[1][2] = vv; rc[1][3] = w; rc[1][4] = T(0.5) * q2;
  rc[2][0] = T(0); rc[2][1] = T(0); rc[2][2] = T(1); rc[2][3] = T(0); rc[2][4] = vv;
  rc[3][0] = T(0); rc[3][1] = T(0); rc[3][2] = T(0); rc[3][3] = T(1); rc[3][4] = w;
  rc[4][0] = T(1); rc[4][1] = u + c; rc[4][2] = vv; rc[4][3] = w; rc[4][4] = H + u * c;
  // point values first: they decide the side's positivity fallback
  bool ok = true;
#pragma unroll
  for (int gp = 0; gp < NGL; ++gp) {
    const T x0 = xi[gp][0], x1 = xi[gp][1], x2 = xi[gp][2];
    T val[5] = {T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int cc = 0; cc < 5; ++cc) {
      T p[10];
#pragma unroll
      for (int k = 0; k < 10; ++k) p[k] = pqs[cc * 10 + k][lt];
      T pv = p[0] + p[1] * x0 + p[2] * x1 + p[3] * x2 + p[4] * (x0 * x0) + p[5] * (x1 * x1) + p[6] * (x2 * x2) +
             p[7] * (x0 * x1) + p[8] * (x0 * x2) + p[9] * (x1 * x2);
#pragma unroll
      for (int v = 0; v < 5; ++v) val[v] += rc[cc][v] * pv;
    }
    ok = ok && phys_ok(val, g);
  }
  if (LPS > 1) {
    // the side falls back if any of its lanes' Gauss points is non-physical
    const unsigned long long bad = __ballot(!ok);
    const int lane0 = (int)(__lane_id() & ~(unsigned)(LPS - 1));
    ok = ((bad >> lane0) & ((1ull << LPS) - 1ull)) == 0ull;
  }
  const size_t ld = 2 * (size_t)F;
  if (!ok) {
    // positivity fallback: first order on this side
    if (g_lo == 0) atomicAdd(nfall, 1);
    for (int gp = 0; gp < NGL; ++gp)
      for (int d = 0; d < 4; ++d)
        for (int v = 0; v < 5; ++v)
          sv[(size_t)(((g_lo + gp) * 4 + d) * 5 + v) * ld + sidx] = d == 0 ? qil[v] : T(0);
    return;
  }
#pragma unroll
  for (int gp = 0; gp < NGL; ++gp) {
    const T x0 = xi[gp][0], x1 = xi[gp][1], x2 = xi[gp][2];
    T out[4][5];
#pragma unroll
    for (int d = 0; d < 4; ++d)
#pragma unroll
      for (int v = 0; v < 5; ++v) out[d][v] = T(0);
#pragma unroll
    for (int cc = 0; cc < 5; ++cc) {
      T p[10];
#pragma unroll
      for (int k = 0; k < 10; ++k) p[k] = pqs[cc * 10 + k][lt];
      T dd[4];
      dd[0] = p[0] + p[1] * x0 + p[2] * x1 + p[3] * x2 + p[4] * (x0 * x0) + p[5] * (x1 * x1) + p[6] * (x2 * x2) +
              p[7] * (x0 * x1) + p[8] * (x0 * x2) + p[9] * (x1 * x2);
      const T gx = p[1] + T(2) * p[4] * x0 + p[7] * x1 + p[8] * x2;
      const T gy = p[2] + T(2) * p[5] * x1 + p[7] * x0 + p[9] * x2;
      const T gz = p[3] + T(2) * p[6] * x2 + p[8] * x0 + p[9] * x1;
#pragma unroll
      for (int a2 = 0; a2 < 3; ++a2) dd[1 + a2] = (gx * e[a2][0] + gy * e[a2][1] + gz * e[a2][2]) * ih;
#pragma unroll
      for (int d = 0; d < 4; ++d)
#pragma unroll
        for (int v = 0; v < 5; ++v) out[d][v] += rc[cc][v] * dd[d];
    }
#pragma unroll
    for (int d = 0; d < 4; ++d)
#pragma unroll
      for (int v = 0; v < 5; ++v) sv[(size_t)(((g_lo + gp) * 4 + d) * 5 + v) * ld + sidx] = out[d][v];
  }
}

