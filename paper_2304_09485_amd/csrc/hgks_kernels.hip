// HIP kernels of the HGKS residual, FD Jacobian-vector product, Jacobi
// preconditioner and GMRES vector operations (gfx950, wave64).
//
// Residual pipeline (paper Sec. 2-3, Sec. 4.1 time-averaged flux):
//   ghost    one thread per boundary face: ghost-cell state (and gradient)
//   recon    one thread per cell: stencil gather and the stored least-squares
//            operator -> coefficients of P0 and P_m in conservative variables
//   side     one thread per face side: characteristic projection of the
//            coefficients, smoothness indicators, nonlinear weights, values and
//            (n,t1,t2) derivatives at the 3 Gauss points, back projection
//   flux     one thread per face: gas-kinetic flux at the 3 Gauss points,
//            quadrature and rotation to the global frame
//   gather   one thread per cell: sum of its 4 signed face fluxes (atomic-free,
//            deterministic), with the Jv / gradient-update epilogues fused
#include "hgks_kernels.h"

#include <mutex>

#include "gks_flux.h"
#include "hgks_device.h"

namespace hgks {

// Workgroups are dispatched to the 8 XCDs of the chip in turn (workgroup b to
// XCD b mod 8), and each XCD has its own L2.  Kernels whose neighbouring
// workgroups read neighbouring cache lines map the dispatch index to a
// logical block so that each XCD works on one contiguous range of blocks:
// a bijection of [0, nb).
constexpr int NUM_XCD = 8;
__device__ __forceinline__ int xcd_block() {
  const int nb = (int)gridDim.x, b = (int)blockIdx.x;
  const int q = nb / NUM_XCD, r = nb % NUM_XCD, x = b % NUM_XCD;
  return x * q + min(x, r) + b / NUM_XCD;
}

// ---------------------------------------------------------------------------
// boundary states
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ void cons_of(T rho, T u0, T u1, T u2, T p, T g, T q[5]) {
  q[0] = rho;
  q[1] = rho * u0;
  q[2] = rho * u1;
  q[3] = rho * u2;
  q[4] = p / (g - T(1)) + T(0.5) * rho * (u0 * u0 + u1 * u1 + u2 * u2);
}

// Riemann-invariant far field along unit normal nn (any frame; uinf in the
// same frame): supersonic inflow -> free stream, supersonic outflow ->
// interior, otherwise R+ from inside, R- from the free stream, entropy and
// tangential velocity from the upwind side.
template <typename T>
__device__ void farfield_state(const T qi[5], const T nn[3], const T ui[3], T rinf, T pinf, T g,
                               T out[5]) {
  T rho = qi[0];
  T U[3] = {qi[1] / rho, qi[2] / rho, qi[3] / rho};
  T p = (g - T(1)) * (qi[4] - T(0.5) * rho * (U[0] * U[0] + U[1] * U[1] + U[2] * U[2]));
  T ci = sqrt(g * p / rho);
  T uni = U[0] * nn[0] + U[1] * nn[1] + U[2] * nn[2];
  if (uni <= -ci) {
    cons_of(rinf, ui[0], ui[1], ui[2], pinf, g, out);
    return;
  }
  if (uni >= ci) {
    for (int k = 0; k < 5; ++k) out[k] = qi[k];
    return;
  }
  T cinf = sqrt(g * pinf / rinf);
  T uninf = ui[0] * nn[0] + ui[1] * nn[1] + ui[2] * nn[2];
  T Rp = uni + T(2) * ci / (g - T(1));
  T Rm = uninf - T(2) * cinf / (g - T(1));
  T unb = T(0.5) * (Rp + Rm);
  T cb = T(0.25) * (g - T(1)) * (Rp - Rm);
  T ent, ut[3];
  if (unb < T(0)) {
    ent = pinf / pow(rinf, g);
    for (int d = 0; d < 3; ++d) ut[d] = ui[d] - uninf * nn[d];
  } else {
    ent = p / pow(rho, g);
    for (int d = 0; d < 3; ++d) ut[d] = U[d] - uni * nn[d];
  }
  T rb = pow(cb * cb / (g * ent), T(1) / (g - T(1)));
  T pb = rb * cb * cb / g;
  cons_of(rb, ut[0] + unb * nn[0], ut[1] + unb * nn[1], ut[2] + unb * nn[2], pb, g, out);
}

template <typename T>
__global__ void __launch_bounds__(256) k_ghost(DevMesh<T> M, Params P, T* __restrict__ Qx,
                                               T* __restrict__ Gx) {
  int gi = blockIdx.x * blockDim.x + threadIdx.x;
  if (gi >= M.Nb) return;
  const int NX = M.NX;
  int o = M.gowner[gi], f = M.gface[gi], kind = M.fkind[f];
  T n[3] = {M.fn[f], M.fn[M.F + f], M.fn[2 * M.F + f]};
  T q[5], out[5];
  for (int v = 0; v < 5; ++v) q[v] = Qx[(size_t)v * NX + o];
  const T g = T(P.gamma);
  for (int v = 0; v < 5; ++v) out[v] = q[v];
  if (kind == 1) {  // slip wall: reflect the momentum about the face plane
    T mn = q[1] * n[0] + q[2] * n[1] + q[3] * n[2];
    for (int d = 0; d < 3; ++d) out[1 + d] = q[1 + d] - T(2) * mn * n[d];
  } else if (kind == 2) {  // no-slip wall: reverse the momentum
    for (int d = 0; d < 3; ++d) out[1 + d] = -q[1 + d];
  } else if (kind == 0) {
    T ui[3] = {T(P.uinf0), T(P.uinf1), T(P.uinf2)};
    farfield_state(q, n, ui, T(P.rhoinf), T(P.pinf), g, out);
  } else if (kind == 3) {
    cons_of(T(P.rhoinf), T(P.uinf0), T(P.uinf1), T(P.uinf2), T(P.pinf), g, out);
  }
  for (int v = 0; v < 5; ++v) Qx[(size_t)v * NX + M.N + gi] = out[v];
  if (Gx) {
    T G[15], Gg[15];
    for (int k = 0; k < 15; ++k) G[k] = Gx[(size_t)k * NX + o];
    if (kind == 0 || kind == 3) {
      for (int k = 0; k < 15; ++k) Gg[k] = T(0);
    } else if (kind == 4) {
      for (int k = 0; k < 15; ++k) Gg[k] = G[k];
    } else {
      // mirror x -> Rm x, Rm = I - 2 n n^T: gradient of q(Rm x) is G Rm
      T Rm[3][3];
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) Rm[a][b] = (a == b ? T(1) : T(0)) - T(2) * n[a] * n[b];
      T GR[5][3];
      for (int v = 0; v < 5; ++v)
        for (int b = 0; b < 3; ++b)
          GR[v][b] = G[v * 3 + 0] * Rm[0][b] + G[v * 3 + 1] * Rm[1][b] + G[v * 3 + 2] * Rm[2][b];
      for (int b = 0; b < 3; ++b) {
        Gg[b] = GR[0][b];
        Gg[12 + b] = GR[4][b];
      }
      for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
          Gg[(1 + a) * 3 + b] = kind == 1 ? Rm[a][0] * GR[1][b] + Rm[a][1] * GR[2][b] + Rm[a][2] * GR[3][b]
                                          : -GR[1 + a][b];
    }
    for (int k = 0; k < 15; ++k) Gx[(size_t)k * NX + M.N + gi] = Gg[k];
  }
}

// ---------------------------------------------------------------------------
// reconstruction: coefficients in conservative variables (linear in the data)
// coef layout [21*5][N], row k*5+v; k < 9: P0 (xi basis), k = 9+3s+t: P_m
// gradient in the xi basis (xi = (x - c)/h)
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_recon_weno(DevMesh<T> M, const T* __restrict__ Qx,
                                                    T* __restrict__ coef) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M.N) return;
  const int N = M.N, NX = M.NX;
  T q0[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) q0[v] = Qx[(size_t)v * NX + i];
  // differences to the 16 cells of the big stencil, all 5 variables: each
  // operator row is then read once and applied to the 5 variables
  T dq[5][16];
#pragma unroll
  for (int j = 0; j < 16; ++j) {
    const int c = M.stn[j * N + i];
#pragma unroll
    for (int v = 0; v < 5; ++v) dq[v][j] = Qx[(size_t)v * NX + c] - q0[v];
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    T acc[5] = {T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      const T o = M.opA[(size_t)(k * 16 + j) * N + i];
#pragma unroll
      for (int v = 0; v < 5; ++v) acc[v] += o * dq[v][j];
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) coef[(size_t)(k * 5 + v) * N + i] = acc[v];
    __builtin_amdgcn_sched_barrier(0);
  }
  // sub-stencil gradients (6 members each)
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    T ds[5][6];
#pragma unroll
    for (int r = 0; r < 6; ++r) {
      const int c = M.sstn[(s * 6 + r) * N + i];
#pragma unroll
      for (int v = 0; v < 5; ++v) ds[v][r] = Qx[(size_t)v * NX + c] - q0[v];
    }
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      T acc[5] = {T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
      for (int r = 0; r < 6; ++r) {
        const T o = M.opB[(size_t)((s * 3 + t) * 6 + r) * N + i];
#pragma unroll
        for (int v = 0; v < 5; ++v) acc[v] += o * ds[v][r];
      }
#pragma unroll
      for (int v = 0; v < 5; ++v) coef[(size_t)((9 + s * 3 + t) * 5 + v) * N + i] = acc[v];
    }
    __builtin_amdgcn_sched_barrier(0);
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_recon_hweno(DevMesh<T> M, const T* __restrict__ Qx,
                                                     const T* __restrict__ Gx, T* __restrict__ coef) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M.N) return;
  const int N = M.N, NX = M.NX;
  int nb[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) nb[k] = M.nbf[k * N + i];
  const T h = M.h[i];
  // the 19 data of the compact stencil for all 5 variables: 4 neighbour
  // differences, own gradient, the 4 neighbours' gradients
  T x[5][19];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    const T q0 = Qx[(size_t)v * NX + i];
#pragma unroll
    for (int k = 0; k < 4; ++k) x[v][k] = Qx[(size_t)v * NX + nb[k]] - q0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      x[v][4 + d] = Gx[(size_t)(v * 3 + d) * NX + i];
#pragma unroll
      for (int k = 0; k < 4; ++k) x[v][7 + 3 * k + d] = Gx[(size_t)(v * 3 + d) * NX + nb[k]];
    }
  }
#pragma unroll
  for (int k = 0; k < 9; ++k) {
    T acc[5] = {T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int j = 0; j < 19; ++j) {
      const T o = M.opH[(size_t)(k * 19 + j) * N + i];
#pragma unroll
      for (int v = 0; v < 5; ++v) acc[v] += o * x[v][j];
    }
#pragma unroll
    for (int v = 0; v < 5; ++v) coef[(size_t)(k * 5 + v) * N + i] = acc[v];
    __builtin_amdgcn_sched_barrier(0);
  }
  // P_m on {i, i_m}: the constrained minimiser has a closed form
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const T wi = M.hsub[(size_t)(s * 6 + 0) * N + i], wm = M.hsub[(size_t)(s * 6 + 1) * N + i];
    const T d0 = M.hsub[(size_t)(s * 6 + 2) * N + i], d1 = M.hsub[(size_t)(s * 6 + 3) * N + i];
    const T d2 = M.hsub[(size_t)(s * 6 + 4) * N + i], id2 = M.hsub[(size_t)(s * 6 + 5) * N + i];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const T g0 = wi * x[v][4] + wm * x[v][7 + 3 * s];
      const T g1 = wi * x[v][5] + wm * x[v][8 + 3 * s];
      const T g2 = wi * x[v][6] + wm * x[v][9 + 3 * s];
      const T lam = (x[v][s] - (d0 * g0 + d1 * g1 + d2 * g2)) * id2;
      coef[(size_t)((9 + s * 3 + 0) * 5 + v) * N + i] = h * (g0 + lam * d0);
      coef[(size_t)((9 + s * 3 + 1) * 5 + v) * N + i] = h * (g1 + lam * d1);
      coef[(size_t)((9 + s * 3 + 2) * 5 + v) * N + i] = h * (g2 + lam * d2);
    }
  }
}

// Hexahedral reconstruction: the non-compact stencil has up to 36 cells and
// the compact one 27 data per variable, too many to hold per lane for all 5
// variables, so the data are streamed member by member and each operator
// entry is applied to the 5 variables as it is read (45 accumulators).
template <typename T>
__global__ void __launch_bounds__(256) k_recon_weno_hex(DevMesh<T> M, const T* __restrict__ Qx,
                                                        T* __restrict__ coef) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M.N) return;
  const int N = M.N, NX = M.NX, nb = M.nbig;
  T q0[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) q0[v] = Qx[(size_t)v * NX + i];
  T acc[9][5];
#pragma unroll
  for (int k = 0; k < 9; ++k)
#pragma unroll
    for (int v = 0; v < 5; ++v) acc[k][v] = T(0);
  for (int j = 0; j < nb; ++j) {
    const int c = M.stn[(size_t)j * N + i];
    T d[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) d[v] = Qx[(size_t)v * NX + c] - q0[v];
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const T o = M.opA[(size_t)(k * nb + j) * N + i];
#pragma unroll
      for (int v = 0; v < 5; ++v) acc[k][v] += o * d[v];
    }
  }
#pragma unroll
  for (int k = 0; k < 9; ++k)
#pragma unroll
    for (int v = 0; v < 5; ++v) coef[(size_t)(k * 5 + v) * N + i] = acc[k][v];
  // the eight sub-stencils {i, i_1 or i_6, two consecutive lateral neighbours}
  for (int sb = 0; sb < 8; ++sb) {
    T ds[3][5];
#pragma unroll
    for (int r = 0; r < 3; ++r) {
      const int c = M.sstn[(size_t)(sb * 3 + r) * N + i];
#pragma unroll
      for (int v = 0; v < 5; ++v) ds[r][v] = Qx[(size_t)v * NX + c] - q0[v];
    }
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      T a5[5] = {T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const T o = M.opB[(size_t)((sb * 3 + t) * 3 + r) * N + i];
#pragma unroll
        for (int v = 0; v < 5; ++v) a5[v] += o * ds[r][v];
      }
#pragma unroll
      for (int v = 0; v < 5; ++v) coef[(size_t)((9 + sb * 3 + t) * 5 + v) * N + i] = a5[v];
    }
  }
}

// SUBW: the sub-stencil polynomials are the eight non-compact ones fitted
// from the cell averages (sstn / opB, as k_recon_weno_hex) instead of the six
// face pairs {i, i_f} fitted with the gradients
template <typename T, bool SUBW>
__global__ void __launch_bounds__(256) k_recon_hweno_hex(DevMesh<T> M, const T* __restrict__ Qx,
                                                         const T* __restrict__ Gx, T* __restrict__ coef) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M.N) return;
  const int N = M.N, NX = M.NX;
  constexpr int NR = 27;  // 6 neighbour differences, own gradient, 6 neighbour gradients
  int nb[6];
#pragma unroll
  for (int k = 0; k < 6; ++k) nb[k] = M.nbf[k * N + i];
  const T h = M.h[i];
  T q0[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) q0[v] = Qx[(size_t)v * NX + i];
  T acc[9][5];
#pragma unroll
  for (int k = 0; k < 9; ++k)
#pragma unroll
    for (int v = 0; v < 5; ++v) acc[k][v] = T(0);
  for (int j = 0; j < NR; ++j) {
    T x[5];
    if (j < 6) {
#pragma unroll
      for (int v = 0; v < 5; ++v) x[v] = Qx[(size_t)v * NX + nb[j]] - q0[v];
    } else {
      const int m = (j - 6) / 3, d = (j - 6) % 3;  // m = 0: the cell itself, else neighbour m - 1
      const int c = m == 0 ? i : nb[m - 1];
#pragma unroll
      for (int v = 0; v < 5; ++v) x[v] = Gx[(size_t)(v * 3 + d) * NX + c];
    }
#pragma unroll
    for (int k = 0; k < 9; ++k) {
      const T o = M.opH[(size_t)(k * NR + j) * N + i];
#pragma unroll
      for (int v = 0; v < 5; ++v) acc[k][v] += o * x[v];
    }
  }
#pragma unroll
  for (int k = 0; k < 9; ++k)
#pragma unroll
    for (int v = 0; v < 5; ++v) coef[(size_t)(k * 5 + v) * N + i] = acc[k][v];
  if (SUBW) {
    // the eight sub-stencils {i, i_1 or i_6, two consecutive lateral neighbours}
    for (int sb = 0; sb < 8; ++sb) {
      T ds[3][5];
#pragma unroll
      for (int r = 0; r < 3; ++r) {
        const int c = M.sstn[(size_t)(sb * 3 + r) * N + i];
#pragma unroll
        for (int v = 0; v < 5; ++v) ds[r][v] = Qx[(size_t)v * NX + c] - q0[v];
      }
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        T a5[5] = {T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int r = 0; r < 3; ++r) {
          const T o = M.opB[(size_t)((sb * 3 + t) * 3 + r) * N + i];
#pragma unroll
          for (int v = 0; v < 5; ++v) a5[v] += o * ds[r][v];
        }
#pragma unroll
        for (int v = 0; v < 5; ++v) coef[(size_t)((9 + sb * 3 + t) * 5 + v) * N + i] = a5[v];
      }
    }
    return;
  }
  // P_m on {i, i_m}: the constrained minimiser has a closed form
  for (int sb = 0; sb < 6; ++sb) {
    const T wi = M.hsub[(size_t)(sb * 6 + 0) * N + i], wm = M.hsub[(size_t)(sb * 6 + 1) * N + i];
    const T d0 = M.hsub[(size_t)(sb * 6 + 2) * N + i], d1 = M.hsub[(size_t)(sb * 6 + 3) * N + i];
    const T d2 = M.hsub[(size_t)(sb * 6 + 4) * N + i], id2 = M.hsub[(size_t)(sb * 6 + 5) * N + i];
    const int c = nb[sb];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      const T g0 = wi * Gx[(size_t)(v * 3 + 0) * NX + i] + wm * Gx[(size_t)(v * 3 + 0) * NX + c];
      const T g1 = wi * Gx[(size_t)(v * 3 + 1) * NX + i] + wm * Gx[(size_t)(v * 3 + 1) * NX + c];
      const T g2 = wi * Gx[(size_t)(v * 3 + 2) * NX + i] + wm * Gx[(size_t)(v * 3 + 2) * NX + c];
      const T dq = Qx[(size_t)v * NX + c] - q0[v];
      const T lam = (dq - (d0 * g0 + d1 * g1 + d2 * g2)) * id2;
      coef[(size_t)((9 + sb * 3 + 0) * 5 + v) * N + i] = h * (g0 + lam * d0);
      coef[(size_t)((9 + sb * 3 + 1) * 5 + v) * N + i] = h * (g1 + lam * d1);
      coef[(size_t)((9 + sb * 3 + 2) * 5 + v) * N + i] = h * (g2 + lam * d2);
    }
  }
}

// ---------------------------------------------------------------------------
// face side: characteristic WENO (Sec. 3.4 Eq. (weno), Sec. 5 projection)
// sv layout [60][2F], row (g*4+d)*5+v, column side*F+f
// ---------------------------------------------------------------------------
template <typename T>
__device__ __forceinline__ bool phys_ok(const T w[5], T g) {
  if (!(w[0] > T(0))) return false;
  T p = (g - T(1)) * (w[4] - T(0.5) * (w[1] * w[1] + w[2] * w[2] + w[3] * w[3]) / w[0]);
  return p > T(0) && isfinite(p);
}

#include "side_kernel.h"

// ---------------------------------------------------------------------------
// flux at the 3 Gauss points of every face (Sec. 2 Eq. (flux), Sec. 4.1)
// ff layout [5][F] (global frame, times area, oriented L -> R); fq likewise
// for the face sum of Gauss-point values (HWENO gradient update)
// ---------------------------------------------------------------------------
template <typename T>
__device__ void boundary_right(int kind, const T Wl[5], const T dWl[3][5], const T ul[3], T rinf, T pinf,
                               T g, T Wr[5], T dWr[3][5]) {
  if (kind == 1 || kind == 2) {
    T m[5] = {T(1), T(-1), T(1), T(1), T(1)};
    if (kind == 2) m[2] = m[3] = T(-1);
    for (int k = 0; k < 5; ++k) {
      Wr[k] = m[k] * Wl[k];
      dWr[0][k] = -m[k] * dWl[0][k];
      dWr[1][k] = m[k] * dWl[1][k];
      dWr[2][k] = m[k] * dWl[2][k];
    }
    return;
  }
  if (kind == 4) {
    for (int k = 0; k < 5; ++k) {
      Wr[k] = Wl[k];
      for (int d = 0; d < 3; ++d) dWr[d][k] = dWl[d][k];
    }
    return;
  }
  if (kind == 0) {
    T nloc[3] = {T(1), T(0), T(0)};
    farfield_state(Wl, nloc, ul, rinf, pinf, g, Wr);
  } else {
    cons_of(rinf, ul[0], ul[1], ul[2], pinf, g, Wr);
  }
  for (int d = 0; d < 3; ++d)
    for (int k = 0; k < 5; ++k) dWr[d][k] = T(0);
}

// one lane per Gauss point: 64 / NG faces per 64-lane block (21 triangles or
// 16 quadrilaterals), the Gauss-point fluxes of a face are summed through LDS
// by the face's first lane
template <int NG>
constexpr int flux_fpb() { return 64 / NG; }

template <typename T, bool QG, int NG>
__global__ void __launch_bounds__(64) k_flux(DevMesh<T> M, Params P, const T* __restrict__ sv,
                                             const T* __restrict__ dt, T* __restrict__ ff,
                                             T* __restrict__ fq) {
  constexpr int FPB = flux_fpb<NG>();
  __shared__ T red[QG ? 10 : 5][64];
  __shared__ T slopes[64 * 45];  // the 45 slope values of each lane's Gauss point
  const int F = M.F, N = M.N;
  const int lane = threadIdx.x;
  const int f = xcd_block() * FPB + lane / NG;  // contiguous face ranges per XCD
  const int gp = lane % NG;
  const bool active = lane < NG * FPB && f < F;
  T Fg[5] = {0, 0, 0, 0, 0}, Qg[5] = {0, 0, 0, 0, 0};
  if (active) {
    int L = M.fL[f], R = M.fR[f];
    bool bnd = R >= N;
    // the flux is averaged over the local time step at CFL cfl_flux
    T dtf = (bnd ? dt[L] : fmin(dt[L], dt[R])) * T(P.flux_scale);
    FluxParams<T> fp;
    fp.gamma = T(P.gamma);
    fp.K = T(P.K);
    fp.tau_eps = T(P.tau_eps);
    fp.tau_C = T(P.tau_C);
    fp.mu = T(P.mu);
    fp.prandtl = T(P.prandtl);
    fp.physics = P.physics;
    const size_t ld = 2 * (size_t)F;
    T Wl[5], dWl[3][5], Wr[5], dWr[3][5];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      Wl[v] = sv[(size_t)((gp * 4 + 0) * 5 + v) * ld + f];
#pragma unroll
      for (int d = 0; d < 3; ++d) dWl[d][v] = sv[(size_t)((gp * 4 + 1 + d) * 5 + v) * ld + f];
    }
    if (bnd) {
      T n[3] = {M.fn[f], M.fn[F + f], M.fn[2 * F + f]}, t1[3], t2[3];
      face_frame(n[0], n[1], n[2], t1, t2);
      T ui[3] = {T(P.uinf0), T(P.uinf1), T(P.uinf2)};
      T ul[3] = {ui[0] * n[0] + ui[1] * n[1] + ui[2] * n[2], ui[0] * t1[0] + ui[1] * t1[1] + ui[2] * t1[2],
                 ui[0] * t2[0] + ui[1] * t2[1] + ui[2] * t2[2]};
      boundary_right(M.fkind[f], Wl, dWl, ul, T(P.rhoinf), T(P.pinf), fp.gamma, Wr, dWr);
    } else {
      const size_t rc = (size_t)F + f;  // column of the right side
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        Wr[v] = sv[(size_t)((gp * 4 + 0) * 5 + v) * ld + rc];
#pragma unroll
        for (int d = 0; d < 3; ++d) dWr[d][v] = sv[(size_t)((gp * 4 + 1 + d) * 5 + v) * ld + rc];
      }
    }
    gks_flux<T, QG>(Wl, dWl, Wr, dWr, dtf, fp, Fg, Qg, slopes + lane * 45);
  }
#pragma unroll
  for (int v = 0; v < 5; ++v) red[v][lane] = Fg[v];
  if (QG)
#pragma unroll
    for (int v = 0; v < 5; ++v) red[5 + v][lane] = Qg[v];
  __syncthreads();
  if (!active || gp != 0) return;
  // quadrature: weights 1/3 on a triangle, the stored weights on a quadrilateral
  T Fs[5], Qs[5];
  if (NG == 3) {
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      Fs[v] = (red[v][lane] / T(3) + red[v][lane + 1] / T(3)) + red[v][lane + 2] / T(3);
      if (QG) Qs[v] = (red[5 + v][lane] / T(3) + red[5 + v][lane + 1] / T(3)) + red[5 + v][lane + 2] / T(3);
    }
  } else {
    T w[NG];
#pragma unroll
    for (int g2 = 0; g2 < NG; ++g2) w[g2] = M.fw[(size_t)g2 * F + f];
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      Fs[v] = T(0);
      Qs[v] = T(0);
#pragma unroll
      for (int g2 = 0; g2 < NG; ++g2) {
        Fs[v] += w[g2] * red[v][lane + g2];
        if (QG) Qs[v] += w[g2] * red[5 + v][lane + g2];
      }
    }
  }
  T n[3] = {M.fn[f], M.fn[F + f], M.fn[2 * F + f]}, t1[3], t2[3];
  face_frame(n[0], n[1], n[2], t1, t2);
  T S = M.fS[f];
  ff[f] = S * Fs[0];
  ff[4 * (size_t)F + f] = S * Fs[4];
#pragma unroll
  for (int d = 0; d < 3; ++d) ff[(size_t)(1 + d) * F + f] = S * (Fs[1] * n[d] + Fs[2] * t1[d] + Fs[3] * t2[d]);
  if (QG) {
    fq[f] = S * Qs[0];
    fq[4 * (size_t)F + f] = S * Qs[4];
#pragma unroll
    for (int d = 0; d < 3; ++d) fq[(size_t)(1 + d) * F + f] = S * (Qs[1] * n[d] + Qs[2] * t1[d] + Qs[3] * t2[d]);
  }
}

// first-order KFVS flux: one thread per face, the cell averages of both
// sides (boundary faces: the boundary state of the owner's average), rotated
// into the face frame; ff as for k_flux
template <typename T>
__global__ void __launch_bounds__(256) k_flux_kfvs(DevMesh<T> M, Params P, const T* __restrict__ Qx,
                                                   T* __restrict__ ff) {
  const int F = M.F, N = M.N, NX = M.NX;
  const int f = xcd_block() * blockDim.x + threadIdx.x;
  if (f >= F) return;
  const int L = M.fL[f], R = M.fR[f];
  T n[3] = {M.fn[f], M.fn[F + f], M.fn[2 * F + f]}, t1[3], t2[3];
  face_frame(n[0], n[1], n[2], t1, t2);
  const T g = T(P.gamma);
  T Wl[5], Wr[5];
  {
    T q[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) q[v] = Qx[(size_t)v * NX + L];
    Wl[0] = q[0];
    Wl[1] = q[1] * n[0] + q[2] * n[1] + q[3] * n[2];
    Wl[2] = q[1] * t1[0] + q[2] * t1[1] + q[3] * t1[2];
    Wl[3] = q[1] * t2[0] + q[2] * t2[1] + q[3] * t2[2];
    Wl[4] = q[4];
  }
  if (R >= N) {
    T ui[3] = {T(P.uinf0), T(P.uinf1), T(P.uinf2)};
    T ul[3] = {ui[0] * n[0] + ui[1] * n[1] + ui[2] * n[2], ui[0] * t1[0] + ui[1] * t1[1] + ui[2] * t1[2],
               ui[0] * t2[0] + ui[1] * t2[1] + ui[2] * t2[2]};
    T d0[3][5] = {}, d1[3][5];
    boundary_right(M.fkind[f], Wl, d0, ul, T(P.rhoinf), T(P.pinf), g, Wr, d1);
  } else {
    T q[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) q[v] = Qx[(size_t)v * NX + R];
    Wr[0] = q[0];
    Wr[1] = q[1] * n[0] + q[2] * n[1] + q[3] * n[2];
    Wr[2] = q[1] * t1[0] + q[2] * t1[1] + q[3] * t1[2];
    Wr[3] = q[1] * t2[0] + q[2] * t2[1] + q[3] * t2[2];
    Wr[4] = q[4];
  }
  T Fs[5];
  kfvs_flux(Wl, Wr, g, T(P.K), Fs);
  const T S = M.fS[f];
  ff[f] = S * Fs[0];
  ff[4 * (size_t)F + f] = S * Fs[4];
#pragma unroll
  for (int d = 0; d < 3; ++d) ff[(size_t)(1 + d) * F + f] = S * (Fs[1] * n[d] + Fs[2] * t1[d] + Fs[3] * t2[d]);
}

// ---------------------------------------------------------------------------
// gather: L(Q_i) = - sum of outward face fluxes (Eq. (finite)); epilogues
//   MODE 0: R = L(Q)
//   MODE 1: Av = (|Omega|/dt) v - (L(Q + sigma v) - b) / sigma     (Eq. (frechet))
//   MODE 2: R = L(Q) and the gradient update of Eq. (derivative)
// ---------------------------------------------------------------------------
template <typename T, typename TO, int MODE, int NF>
__global__ void __launch_bounds__(256) k_gather(DevMesh<T> M, const T* __restrict__ ff,
                                                const T* __restrict__ fq, TO* __restrict__ out,
                                                const TO* __restrict__ vin, const TO* __restrict__ bin,
                                                const T* __restrict__ dt, const double* __restrict__ sigma,
                                                TO* __restrict__ gout) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int N = M.N, F = M.F;
  if (i >= N) return;
  T r[5] = {0, 0, 0, 0, 0};
  T gq[15];
  if (MODE == 2)
    for (int k = 0; k < 15; ++k) gq[k] = T(0);
#pragma unroll
  for (int p = 0; p < NF; ++p) {
    int cf = M.cface[p * N + i];
    int f = (cf > 0 ? cf : -cf) - 1;
    T s = cf > 0 ? T(1) : T(-1);
#pragma unroll
    for (int v = 0; v < 5; ++v) r[v] -= s * ff[(size_t)v * F + f];
    if (MODE == 2) {
      T n[3] = {M.fn[f], M.fn[F + f], M.fn[2 * F + f]};
      T iv = T(1) / M.vol[i];
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        T qv = s * fq[(size_t)v * F + f];
#pragma unroll
        for (int d = 0; d < 3; ++d) gq[v * 3 + d] += qv * n[d] * iv;
      }
    }
  }
  if (MODE == 1) {
    double sg = sigma[0];
    TO a = TO(M.vol[i] / dt[i]);
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      size_t k = (size_t)v * N + i;
      out[k] = sg > 0.0 ? TO(a * vin[k] - (TO(r[v]) - bin[k]) / TO(sg)) : TO(0);
    }
  } else {
#pragma unroll
    for (int v = 0; v < 5; ++v) out[(size_t)v * N + i] = TO(r[v]);
  }
  if (MODE == 2)
    for (int k = 0; k < 15; ++k) gout[(size_t)k * N + i] = TO(gq[k]);
}

// ---------------------------------------------------------------------------
// time step, approximate matrix and Jacobi sweeps (Sec. 4.1-4.2)
// ---------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) k_dt(DevMesh<T> M, Params P, double cfl, const T* __restrict__ Qx,
                                            T* __restrict__ dt) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M.N) return;
  const int NX = M.NX;
  T rho = Qx[i], U = Qx[NX + i] / rho, V = Qx[2 * (size_t)NX + i] / rho, W = Qx[3 * (size_t)NX + i] / rho;
  T g = T(P.gamma);
  T p = (g - T(1)) * (Qx[4 * (size_t)NX + i] - T(0.5) * rho * (U * U + V * V + W * W));
  T c = sqrt(g * p / rho);
  T nu = P.physics ? T(P.mu) / rho : T(0);
  T hd = M.hdt[i];
  dt[i] = T(cfl) * hd / (sqrt(U * U + V * V + W * W) + c + T(2) * nu / hd);
}

template <typename T>
__global__ void __launch_bounds__(256) k_lambda(DevMesh<T> M, Params P, const T* __restrict__ Qx,
                                                T* __restrict__ lam) {
  int f = blockIdx.x * blockDim.x + threadIdx.x;
  if (f >= M.F) return;
  const int NX = M.NX, F = M.F;
  int a = M.fL[f], b = M.fR[f];
  T g = T(P.gamma);
  T pr[2][5];
  int cells[2] = {a, b};
  for (int s = 0; s < 2; ++s) {
    int c = cells[s];
    T rho = Qx[c];
    T U = Qx[NX + c] / rho, V = Qx[2 * (size_t)NX + c] / rho, W = Qx[3 * (size_t)NX + c] / rho;
    pr[s][0] = rho;
    pr[s][1] = U;
    pr[s][2] = V;
    pr[s][3] = W;
    pr[s][4] = (g - T(1)) * (Qx[4 * (size_t)NX + c] - T(0.5) * rho * (U * U + V * V + W * W));
  }
  T rho = T(0.5) * (pr[0][0] + pr[1][0]), p = T(0.5) * (pr[0][4] + pr[1][4]);
  T un = T(0.5) * (pr[0][1] + pr[1][1]) * M.fn[f] + T(0.5) * (pr[0][2] + pr[1][2]) * M.fn[F + f] +
         T(0.5) * (pr[0][3] + pr[1][3]) * M.fn[2 * F + f];
  lam[f] = fabs(un) + sqrt(g * p / rho);
}

template <typename T, int NF>
__global__ void __launch_bounds__(256) k_diag(DevMesh<T> M, const T* __restrict__ lam, const T* __restrict__ dt,
                                              T* __restrict__ D) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= M.N) return;
  T s = M.vol[i] / dt[i];
#pragma unroll
  for (int p = 0; p < NF; ++p) {
    int cf = M.cface[p * M.N + i];
    int f = (cf > 0 ? cf : -cf) - 1;
    s += T(0.5) * lam[f] * M.fS[f];
  }
  D[i] = s;
}

// Euler flux Jacobian along n applied to x
template <typename T>
__device__ __forceinline__ void euler_jn(T g, const T q[5], const T n[3], const T x[5], T out[5]) {
  T rho = q[0];
  T U[3] = {q[1] / rho, q[2] / rho, q[3] / rho};
  T uu = U[0] * U[0] + U[1] * U[1] + U[2] * U[2];
  T p = (g - T(1)) * (q[4] - T(0.5) * rho * uu);
  T un = U[0] * n[0] + U[1] * n[1] + U[2] * n[2];
  T dmn = x[1] * n[0] + x[2] * n[1] + x[3] * n[2];
  T dun = (dmn - un * x[0]) / rho;
  T dp = (g - T(1)) * (x[4] - (U[0] * x[1] + U[1] * x[2] + U[2] * x[3]) + T(0.5) * uu * x[0]);
  out[0] = dmn;
  for (int d = 0; d < 3; ++d) out[1 + d] = x[1 + d] * un + q[1 + d] * dun + dp * n[d];
  out[4] = (x[4] + dp) * un + (q[4] + p) * dun;
}

// x_new = D^{-1} (r - (L+U) x_old); x_old == nullptr gives D^{-1} r
// A x with the approximate matrix of Eq. (deri-matrix): D_i x_i plus the
// off-diagonal blocks 1/2 S_f (J_n(Q_j) - |lambda_f|) x_j of the cell's
// interior faces (boundary off-diagonal blocks dropped)
template <typename T, int NF>
__global__ void __launch_bounds__(256) k_amatvec(DevMesh<T> M, Params P, const T* __restrict__ Qx,
                                                 const T* __restrict__ lam, const T* __restrict__ D,
                                                 const double* __restrict__ x, double* __restrict__ out) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int N = M.N, NX = M.NX, F = M.F;
  if (i >= N) return;
  const T g = T(P.gamma);
  T acc[5];
  for (int v = 0; v < 5; ++v) acc[v] = D[i] * T(x[(size_t)v * N + i]);
#pragma unroll
  for (int p = 0; p < NF; ++p) {
    const int cf = M.cface[p * N + i];
    const int jn = M.nbf[p * N + i];  // read beside the face id
    if (jn >= N) continue;
    const int f = (cf > 0 ? cf : -cf) - 1;
    T s = cf > 0 ? T(1) : T(-1);
    T n[3] = {s * M.fn[f], s * M.fn[F + f], s * M.fn[2 * F + f]};
    T qj[5], xj[5], jx[5];
    for (int v = 0; v < 5; ++v) {
      qj[v] = Qx[(size_t)v * NX + jn];
      xj[v] = T(x[(size_t)v * N + jn]);
    }
    euler_jn(g, qj, n, xj, jx);
    T hs = T(0.5) * M.fS[f], l = lam[f];
    for (int v = 0; v < 5; ++v) acc[v] += hs * (jx[v] - l * xj[v]);
  }
  for (int v = 0; v < 5; ++v) out[(size_t)v * N + i] = double(acc[v]);
}

// One colour class of an LU-SGS sweep (cells cord[c0 .. c0 + nc), colour
// col): the off-diagonal blocks 1/2 S_f (J_n(Q_j) - |lambda_f|) of the
// approximate matrix to the interior neighbours of lower (forward) or higher
// (backward) colour, applied to their already final values in x;
//   forward  x_i = (b_i - sum) / D_i        ((D + L) y = R, b = R)
//   backward x_i = b_i - sum / D_i          ((D + U) dQ = D y, b = y)
// Cells of one colour share no face, so the class updates in parallel.
template <typename T, bool FWD, int NF>
__global__ void __launch_bounds__(256) k_lusgs(DevMesh<T> M, Params P, const T* __restrict__ Qx,
                                               const T* __restrict__ lam, const T* __restrict__ D, int c0, int nc,
                                               int col, const double* __restrict__ b, double* x) {
  int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nc) return;
  const int N = M.N, NX = M.NX, F = M.F;
  const int i = M.cord[c0 + t];
  const T g = T(P.gamma);
  T off[5] = {0, 0, 0, 0, 0};
#pragma unroll
  for (int p = 0; p < NF; ++p) {
    const int cf = M.cface[p * N + i];
    const int jn = M.nbf[p * N + i];  // read beside the face id
    if (jn >= N) continue;
    const int f = (cf > 0 ? cf : -cf) - 1;
    int cj = M.ccol[jn];
    if (FWD ? cj > col : cj < col) continue;
    T s = cf > 0 ? T(1) : T(-1);
    T n[3] = {s * M.fn[f], s * M.fn[F + f], s * M.fn[2 * F + f]};
    T qj[5], xj[5], jx[5];
    for (int v = 0; v < 5; ++v) {
      qj[v] = Qx[(size_t)v * NX + jn];
      xj[v] = T(x[(size_t)v * N + jn]);
    }
    euler_jn(g, qj, n, xj, jx);
    T hs = T(0.5) * M.fS[f], l = lam[f];
    for (int v = 0; v < 5; ++v) off[v] += hs * (jx[v] - l * xj[v]);
  }
  const T d = D[i];
  for (int v = 0; v < 5; ++v) {
    T bv = T(b[(size_t)v * N + i]);
    x[(size_t)v * N + i] = double(FWD ? (bv - off[v]) / d : bv - off[v] / d);
  }
}

// X0R: the sweep's input is x0 = D^{-1} r, formed on the fly from r and D
// (the first two sweeps in one pass, with the same arithmetic as a stored x0)
template <typename T, int NF, bool X0R>
__global__ void __launch_bounds__(256) k_jacobi(DevMesh<T> M, Params P, const T* __restrict__ Qx,
                                                const T* __restrict__ lam, const T* __restrict__ D,
                                                const double* __restrict__ r, const double* __restrict__ xo,
                                                double* __restrict__ xn) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int N = M.N, NX = M.NX, F = M.F;
  if (i >= N) return;
  T acc[5];
  for (int v = 0; v < 5; ++v) acc[v] = T(r[(size_t)v * N + i]);
  if (xo || X0R) {
    T g = T(P.gamma);
#pragma unroll
    for (int p = 0; p < NF; ++p) {
      // the neighbour id is read beside the face id (not through the face),
      // so the neighbour's data and the face's data are gathered in parallel
      const int cf = M.cface[p * N + i];
      const int jn = M.nbf[p * N + i];
      if (jn >= N) continue;  // boundary off-diagonal blocks are dropped
      const int f = (cf > 0 ? cf : -cf) - 1;
      T s = cf > 0 ? T(1) : T(-1);
      T n[3] = {s * M.fn[f], s * M.fn[F + f], s * M.fn[2 * F + f]};
      T qj[5], xj[5], jx[5];
      const T idj = X0R ? T(1) / D[jn] : T(0);
      for (int v = 0; v < 5; ++v) {
        qj[v] = Qx[(size_t)v * NX + jn];
        xj[v] = X0R ? T(double(T(r[(size_t)v * N + jn]) * idj)) : T(xo[(size_t)v * N + jn]);
      }
      euler_jn(g, qj, n, xj, jx);
      T hs = T(0.5) * M.fS[f], l = lam[f];
      for (int v = 0; v < 5; ++v) acc[v] -= hs * (jx[v] - l * xj[v]);
    }
  }
  T id = T(1) / D[i];
  for (int v = 0; v < 5; ++v) xn[(size_t)v * N + i] = double(acc[v] * id);
}

// ---------------------------------------------------------------------------
// vector kernels (FP64 Krylov space); deterministic two-level reductions
// ---------------------------------------------------------------------------
constexpr int RB = 256;     // reduction block
constexpr int RGRID = REDUCE_PARTS; // fixed grid -> fixed summation order
// relative truncation error of an FD product per unit step length |sigma v|,
// assumed when the step is balanced against the rounding of the inner
// precision (measured 2 to 200 on shells and ramps; the balance is within a
// factor 2 of the best step over that range)
constexpr double FD_TRUNC = 10.0;

// sum over the block in a fixed order: a shuffle tree within each 64-lane
// wave, then the wave sums in index order; every lane gets the result.  A
// second call in the same kernel needs a barrier before it (the wave sums
// are read by all lanes).
__device__ __forceinline__ double block_sum(double x) {
  static_assert(RB % 64 == 0, "whole waves");
  __shared__ double sh[RB / 64];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) x += __shfl_down(x, off, 64);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = x;
  __syncthreads();
  double t = sh[0];
#pragma unroll
  for (int k = 1; k < RB / 64; ++k) t += sh[k];
  return t;
}

// part[blockIdx] = sum over a fixed strided slice of op(x, y) (OP 0: x.y,
// 1: |x|); a second one-block kernel sums the partials in block order, so the
// summation order does not depend on scheduling
template <int OP>
__global__ void __launch_bounds__(RB) k_reduce_part(const double* __restrict__ x, const double* __restrict__ y,
                                                    size_t n, double* __restrict__ part) {
  double s = 0.0;
  for (size_t k = (size_t)blockIdx.x * RB + threadIdx.x; k < n; k += (size_t)RGRID * RB) {
    if (OP == 0) s += x[k] * y[k];
    else if (OP == 1) s += fabs(x[k]);
    else s += (x[k] - y[k]) * (x[k] - y[k]);
  }
  double t = block_sum(s);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// out[0] = sum(part) (SQRT: sqrt of it)
template <bool SQRT>
__global__ void __launch_bounds__(RB) k_reduce_final(const double* __restrict__ part, double* __restrict__ out) {
  double s = 0.0;
  for (int k = threadIdx.x; k < RGRID; k += RB) s += part[k];
  double t = block_sum(s);
  if (threadIdx.x == 0) out[0] = SQRT ? sqrt(t) : t;
}

// out[0] = sqrt(sum(part)) / den[0] (0 if den[0] is 0)
__global__ void __launch_bounds__(RB) k_reduce_norm_ratio(const double* __restrict__ part,
                                                          const double* __restrict__ den, double* __restrict__ out) {
  double s = 0.0;
  for (int k = threadIdx.x; k < RGRID; k += RB) s += part[k];
  double t = block_sum(s);
  if (threadIdx.x == 0) out[0] = den[0] > 0.0 ? sqrt(t) / den[0] : 0.0;
}

// one modified Gram-Schmidt step fused with the partials of the next inner
// product.  Its coefficient h comes from the block partials of the previous
// inner product: every block sums pin in the fixed order of k_reduce_final
// (so h is bitwise the value that kernel would write), and block 0 stores it
// in hout[0] for the Hessenberg column.  Then w -= h v, and pout = block
// partials of w.z, or of w.w if z is null (pin and pout are distinct).
__global__ void __launch_bounds__(RB) k_axpy_dot_chain(const double* __restrict__ pin, double* __restrict__ hout,
                                                       const double* __restrict__ v, double* __restrict__ w, size_t n,
                                                       const double* __restrict__ z, double* __restrict__ pout) {
  double s0 = 0.0;
  for (int k = threadIdx.x; k < RGRID; k += RB) s0 += pin[k];
  const double h = block_sum(s0);
  __syncthreads();  // every lane has read the sum before block_sum's buffer is reused
  if (blockIdx.x == 0 && threadIdx.x == 0) hout[0] = h;
  double s = 0.0;
  for (size_t k = (size_t)blockIdx.x * RB + threadIdx.x; k < n; k += (size_t)RGRID * RB) {
    double wk = w[k] - h * v[k];
    w[k] = wk;
    s += wk * (z ? z[k] : wk);
  }
  double t = block_sum(s);
  if (threadIdx.x == 0) pout[blockIdx.x] = t;
}

// y += alpha * x, alpha = sgn * a[0] (or * 1/a[0] if INV)
__global__ void __launch_bounds__(256) k_axpy_dev(const double* __restrict__ x, double* __restrict__ y,
                                                  size_t n, const double* __restrict__ a, double sgn) {
  size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  y[k] += sgn * a[0] * x[k];
}

// Q += alpha_i dQ per cell, alpha_i the largest 2^-k (k <= 20) for which the
// cell's density and pressure change by at most th of their old values (the
// update limit of impulsive starts); cells with alpha_i < 1 are counted
__global__ void __launch_bounds__(256) k_update_limited(double* __restrict__ Q, const double* __restrict__ dQ, int N,
                                                        double th, double g, int* __restrict__ nlim) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double q[5], d[5];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    q[v] = Q[(size_t)v * N + i];
    d[v] = dQ[(size_t)v * N + i];
  }
  const double p0 = (g - 1.0) * (q[4] - 0.5 * (q[1] * q[1] + q[2] * q[2] + q[3] * q[3]) / q[0]);
  double a = 1.0;
  for (int k = 0; k < 20; ++k) {
    double qn[5];
#pragma unroll
    for (int v = 0; v < 5; ++v) qn[v] = q[v] + a * d[v];
    const double pn = (g - 1.0) * (qn[4] - 0.5 * (qn[1] * qn[1] + qn[2] * qn[2] + qn[3] * qn[3]) / qn[0]);
    if (fabs(qn[0] - q[0]) <= th * q[0] && fabs(pn - p0) <= th * p0) break;
    a *= 0.5;
  }
  if (a < 1.0) atomicAdd(nlim, 1);
#pragma unroll
  for (int v = 0; v < 5; ++v) Q[(size_t)v * N + i] = q[v] + a * d[v];
}

// y = x / a[0]; nothing if skip[0] is set (a finished GMRES cycle)
__global__ void __launch_bounds__(256) k_scale_inv(const double* __restrict__ x, double* __restrict__ y, size_t n,
                                                   const double* __restrict__ a, const int* __restrict__ skip) {
  size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n || (skip && skip[0])) return;
  y[k] = x[k] / a[0];
}

// ---------------------------------------------------------------------------
// GMRES cycle bookkeeping on the device (one thread), so that the Arnoldi
// steps of a restart are queued without a host round trip.  G holds the
// Hessenberg matrix H [(m+1) x m], the Givens cosines and sines [m], the
// rotated right-hand side g [m+1]; st: [0] cycle finished (happy breakdown,
// zero or non-finite data), [1] non-finite data seen, [2] columns done.
// ---------------------------------------------------------------------------
__global__ void k_gmres_start(const double* __restrict__ beta, double* __restrict__ G, int* __restrict__ st,
                              int m) {
  double* g = G + (size_t)(m + 1) * m + 2 * m;
  for (int k = 0; k <= m; ++k) g[k] = 0.0;
  const double b = beta[0];
  g[0] = b;
  const bool fin = isfinite(b);
  st[0] = (!fin || !(b > 0.0)) ? 1 : 0;
  st[1] = fin ? 0 : 1;
  st[2] = 0;
}

// column j of H from the modified Gram-Schmidt coefficients hc[0..j+1]:
// apply the previous rotations, form rotation j, update g
__global__ void k_gmres_column(int j, int m, const double* __restrict__ hc, double* __restrict__ G,
                               int* __restrict__ st) {
  if (st[0]) return;
  double* H = G;
  double* cs = G + (size_t)(m + 1) * m;
  double* sn = cs + m;
  double* g = sn + m;
  for (int i = 0; i <= j + 1; ++i)
    if (!isfinite(hc[i])) {
      st[1] = 1;
      st[0] = 1;
      return;
    }
  for (int i = 0; i <= j + 1; ++i) H[(size_t)i * m + j] = hc[i];
  const double hn = hc[j + 1];
  // |P A v_j| before orthogonalisation, from the raw column, for the
  // breakdown test
  double col2 = 0.0;
  for (int i = 0; i <= j + 1; ++i) col2 += hc[i] * hc[i];
  for (int i = 0; i < j; ++i) {
    double a = H[(size_t)i * m + j], c = H[(size_t)(i + 1) * m + j];
    H[(size_t)i * m + j] = cs[i] * a + sn[i] * c;
    H[(size_t)(i + 1) * m + j] = -sn[i] * a + cs[i] * c;
  }
  double a = H[(size_t)j * m + j], c = H[(size_t)(j + 1) * m + j];
  double rr = hypot(a, c);
  cs[j] = a / rr;
  sn[j] = c / rr;
  H[(size_t)j * m + j] = rr;
  H[(size_t)(j + 1) * m + j] = 0.0;
  g[j + 1] = -sn[j] * g[j];
  g[j] = cs[j] * g[j];
  st[2] = j + 1;
  // happy breakdown: the new direction is lost to rounding relative to the
  // vector it was orthogonalised from
  if (hn <= 1e-14 * sqrt(col2)) st[0] = 1;
}

// back substitution of the triangular system (y = 0 beyond the columns done,
// and for a cycle with non-finite data); out[0] = |g[columns done]|
__global__ void k_gmres_solve(int m, const double* __restrict__ G, const int* __restrict__ st,
                              double* __restrict__ y, double* __restrict__ out) {
  const double* H = G;
  const double* g = G + (size_t)(m + 1) * m + 2 * m;
  const int jd = st[1] ? 0 : st[2];
  for (int i = m - 1; i >= 0; --i) {
    if (i >= jd) {
      y[i] = 0.0;
      continue;
    }
    double sacc = g[i];
    for (int k = i + 1; k < jd; ++k) sacc -= H[(size_t)i * m + k] * y[k];
    y[i] = sacc / H[(size_t)i * m + i];
  }
  out[0] = fabs(g[st[2]]);
}

// y = x + sum_j c[j] V[j]  (V: nv vectors of length n, c on the device)
__global__ void __launch_bounds__(256) k_combine(const double* __restrict__ V, const double* __restrict__ c, int nv,
                                                 size_t n, const double* __restrict__ x, double* __restrict__ y) {
  size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  double s = x ? x[k] : 0.0;
  for (int j = 0; j < nv; ++j) s += c[j] * V[(size_t)j * n + k];
  y[k] = s;
}

// Qp(cells) = Q + sigma v (Q, v: [5][N]), written into an extended array [5][NX]
template <typename T>
__global__ void __launch_bounds__(256) k_perturb(const double* __restrict__ Q, const double* __restrict__ v,
                                                 const double* __restrict__ sigma, int N, int NX,
                                                 T* __restrict__ Qp) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  double s = sigma ? sigma[0] : 0.0;
  for (int q = 0; q < 5; ++q) {
    double val = Q[(size_t)q * N + i] + (v ? s * v[(size_t)q * N + i] : 0.0);
    Qp[(size_t)q * NX + i] = T(val);
  }
}

__global__ void __launch_bounds__(256) k_convert(const double* __restrict__ src, float* __restrict__ dst,
                                                 size_t n) {
  size_t k = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) dst[k] = (float)src[k];
}

// automatic FD step of Eq. (frechet): sqrt(eps) max(1, rms Q) / rms v
// (|v|^2 is summed here from its block partials, in the fixed order of
// k_reduce_final, so no separate reduction launch precedes this one)
// block maxima of the relative size of a direction v against the state Q:
// max over cells of |v_rho| / rho, |v_m| / sqrt(rho E) and |v_E| / E (all
// scales positive in a physical state; the momentum one bounds the change of
// the kinetic energy by a fraction of E)
__global__ void __launch_bounds__(RB) k_ratio_part(const double* __restrict__ Q, const double* __restrict__ v, int N,
                                                   double* __restrict__ part) {
  double m = 0.0;
  for (int i = blockIdx.x * RB + threadIdx.x; i < N; i += RGRID * RB) {
    const double rho = Q[i], E = Q[4 * (size_t)N + i];
    const double v1 = v[(size_t)N + i], v2 = v[2 * (size_t)N + i], v3 = v[3 * (size_t)N + i];
    m = fmax(m, fabs(v[i]) / rho);
    m = fmax(m, fabs(v[4 * (size_t)N + i]) / E);
    m = fmax(m, sqrt((v1 * v1 + v2 * v2 + v3 * v3) / (rho * E)));
  }
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_down(m, off, 64));
  __shared__ double sh[RB / 64];
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = sh[0];
#pragma unroll
    for (int k = 1; k < RB / 64; ++k) t = fmax(t, sh[k]);
    part[blockIdx.x] = t;
  }
}

__global__ void __launch_bounds__(RB) k_sigma(const double* __restrict__ vpart, const double* __restrict__ qq,
                                              double n, double eps, double fixed, double* __restrict__ sigma,
                                              const double* __restrict__ rpart, double eta,
                                              const double* __restrict__ noise, double* __restrict__ vnorm) {
  double s0 = 0.0;
  for (int k = threadIdx.x; k < RGRID; k += RB) s0 += vpart[k];
  const double vv = block_sum(s0);
  // the largest relative perturbation of density and energy a unit step makes
  double r = 0.0;
  if (rpart) {
    __syncthreads();
    __shared__ double shr[RB];
    double m = 0.0;
    for (int k = threadIdx.x; k < RGRID; k += RB) m = fmax(m, rpart[k]);
    shr[threadIdx.x] = m;
    __syncthreads();
    if (threadIdx.x == 0)
      for (int k = 0; k < RB; ++k) r = fmax(r, shr[k]);
  }
  if (threadIdx.x != 0) return;
  if (vnorm) vnorm[0] = sqrt(vv);
  double rv = sqrt(vv / n);
  if (rv == 0.0) {
    sigma[0] = 0.0;
    return;
  }
  if (fixed > 0.0) {
    sigma[0] = fixed;
    return;
  }
  double rq = sqrt(qq[0] / n);
  double sg = sqrt(eps) * fmax(1.0, rq) / rv;
  // no cell's density, momentum or energy moves by more than eta
  if (r > 0.0) sg = fmin(sg, eta / r);
  // rounding-aware step: noise[0] = |L~(Q) - L(Q)| (the rounding of one
  // evaluation in the inner precision), noise[1] = |A u| of the last inner
  // product per unit |u|.  The FD product then carries a rounding error of
  // about sqrt(2) noise[0] / s relative to |A v| / |v| and a truncation error
  // of about FD_TRUNC s, s = sigma |v|; s = sqrt(sqrt(2) noise[0] / (FD_TRUNC
  // noise[1])) balances the two
  if (noise && noise[0] > 0.0 && noise[1] > 0.0) {
    const double st = sqrt(sqrt(2.0) * noise[0] / (FD_TRUNC * noise[1]));
    if (st > 0.0 && isfinite(st)) sg = fmin(sg, st / sqrt(vv));
  }
  sigma[0] = sg;
}

// relaxed gradient update of the compact scheme: G += w (Gnew - G), 15 rows
__global__ void __launch_bounds__(256) k_relax_grad(double* __restrict__ G, const double* __restrict__ Gnew, int N,
                                                    int NX, double w) {
  const size_t t = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (size_t)15 * N) return;
  const size_t k = t / N, i = t - k * N;
  double* g = G + k * NX + i;
  *g += w * (Gnew[t] - *g);
}

template <typename T>
__global__ void __launch_bounds__(256) k_check(const T* __restrict__ Qx, int N, int NX, double gamma,
                                               int* __restrict__ bad) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  T w[5];
  for (int v = 0; v < 5; ++v) w[v] = Qx[(size_t)v * NX + i];
  if (!phys_ok(w, T(gamma))) atomicOr(bad, 1);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline unsigned nblk(size_t n, int b) { return (unsigned)((n + b - 1) / b); }

template <typename T>
void launch_ghost(const DevMesh<T>& M, const Params& P, T* Qx, T* Gx, hipStream_t s) {
  if (M.Nb) hipLaunchKernelGGL(k_ghost<T>, dim3(nblk(M.Nb, 256)), dim3(256), 0, s, M, P, Qx, Gx);
}
template <typename T>
void launch_recon(const DevMesh<T>& M, const Params& P, const T* Qx, const T* Gx, T* coef, hipStream_t s) {
  const dim3 g(nblk(M.N, 256)), b(256);
  if (M.nf == 6) {
    if (P.scheme == 1 && P.csubs)
      hipLaunchKernelGGL((k_recon_hweno_hex<T, true>), g, b, 0, s, M, Qx, Gx, coef);
    else if (P.scheme == 1)
      hipLaunchKernelGGL((k_recon_hweno_hex<T, false>), g, b, 0, s, M, Qx, Gx, coef);
    else
      hipLaunchKernelGGL(k_recon_weno_hex<T>, g, b, 0, s, M, Qx, coef);
  } else if (P.scheme == 1) {
    hipLaunchKernelGGL(k_recon_hweno<T>, g, b, 0, s, M, Qx, Gx, coef);
  } else {
    hipLaunchKernelGGL(k_recon_weno<T>, g, b, 0, s, M, Qx, coef);
  }
}
template <typename T>
void launch_side(const DevMesh<T>& M, const Params& P, const T* Qx, const T* coef, T* sv, int* nfall,
                 hipStream_t s) {
  const dim3 b(SIDE_THREADS), g(nblk(2 * (size_t)M.F, SIDE_SPB));
  if (M.nf == 4) {
    hipLaunchKernelGGL((k_side<T, 4, 3, 1>), g, b, 0, s, M, P, Qx, coef, sv, nfall);
  } else if (P.scheme == 1 && !P.csubs) {
    // quadrilateral faces: one lane per side, its 4 Gauss points evaluated
    // from the combined polynomials after the component loop
    hipLaunchKernelGGL((k_side<T, 6, 4, 1>), g, b, 0, s, M, P, Qx, coef, sv, nfall);
  } else {
    hipLaunchKernelGGL((k_side<T, 8, 4, 1>), g, b, 0, s, M, P, Qx, coef, sv, nfall);
  }
}
template <typename T>
void launch_flux(const DevMesh<T>& M, const Params& P, const T* sv, const T* dt, T* ff, T* fq, bool qg,
                 hipStream_t s) {
  if (M.ng == 3) {
    dim3 grid(nblk(M.F, flux_fpb<3>()));
    if (qg)
      hipLaunchKernelGGL((k_flux<T, true, 3>), grid, dim3(64), 0, s, M, P, sv, dt, ff, fq);
    else
      hipLaunchKernelGGL((k_flux<T, false, 3>), grid, dim3(64), 0, s, M, P, sv, dt, ff, fq);
  } else {
    dim3 grid(nblk(M.F, flux_fpb<4>()));
    if (qg)
      hipLaunchKernelGGL((k_flux<T, true, 4>), grid, dim3(64), 0, s, M, P, sv, dt, ff, fq);
    else
      hipLaunchKernelGGL((k_flux<T, false, 4>), grid, dim3(64), 0, s, M, P, sv, dt, ff, fq);
  }
}
template <typename T>
void launch_flux_kfvs(const DevMesh<T>& M, const Params& P, const T* Qx, T* ff, hipStream_t s) {
  if (M.F) hipLaunchKernelGGL(k_flux_kfvs<T>, dim3(nblk(M.F, 256)), dim3(256), 0, s, M, P, Qx, ff);
}
template <typename T, typename TO>
void launch_gather(const DevMesh<T>& M, int mode, const T* ff, const T* fq, TO* out, const TO* v, const TO* b,
                   const T* dt, const double* sigma, TO* gout, hipStream_t s) {
  dim3 g(nblk(M.N, 256)), bl(256);
  if (M.nf == 4) {
    if (mode == 0)
      hipLaunchKernelGGL((k_gather<T, TO, 0, 4>), g, bl, 0, s, M, ff, fq, out, v, b, dt, sigma, gout);
    else if (mode == 1)
      hipLaunchKernelGGL((k_gather<T, TO, 1, 4>), g, bl, 0, s, M, ff, fq, out, v, b, dt, sigma, gout);
    else
      hipLaunchKernelGGL((k_gather<T, TO, 2, 4>), g, bl, 0, s, M, ff, fq, out, v, b, dt, sigma, gout);
  } else {
    if (mode == 0)
      hipLaunchKernelGGL((k_gather<T, TO, 0, 6>), g, bl, 0, s, M, ff, fq, out, v, b, dt, sigma, gout);
    else if (mode == 1)
      hipLaunchKernelGGL((k_gather<T, TO, 1, 6>), g, bl, 0, s, M, ff, fq, out, v, b, dt, sigma, gout);
    else
      hipLaunchKernelGGL((k_gather<T, TO, 2, 6>), g, bl, 0, s, M, ff, fq, out, v, b, dt, sigma, gout);
  }
}
template <typename T>
void launch_dt(const DevMesh<T>& M, const Params& P, double cfl, const T* Qx, T* dt, hipStream_t s) {
  hipLaunchKernelGGL(k_dt<T>, dim3(nblk(M.N, 256)), dim3(256), 0, s, M, P, cfl, Qx, dt);
}
template <typename T>
void launch_lambda_diag(const DevMesh<T>& M, const Params& P, const T* Qx, const T* dt, T* lam, T* D,
                        hipStream_t s) {
  hipLaunchKernelGGL(k_lambda<T>, dim3(nblk(M.F, 256)), dim3(256), 0, s, M, P, Qx, lam);
  if (M.nf == 4)
    hipLaunchKernelGGL((k_diag<T, 4>), dim3(nblk(M.N, 256)), dim3(256), 0, s, M, lam, dt, D);
  else
    hipLaunchKernelGGL((k_diag<T, 6>), dim3(nblk(M.N, 256)), dim3(256), 0, s, M, lam, dt, D);
}
template <typename T>
void launch_jacobi(const DevMesh<T>& M, const Params& P, const T* Qx, const T* lam, const T* D, const double* r,
                   const double* xo, double* xn, hipStream_t s) {
  // xo == r: the input of the sweep is D^{-1} r (fused first sweep)
  const dim3 g(nblk(M.N, 256)), b(256);
  if (xo == r) {
    if (M.nf == 4)
      hipLaunchKernelGGL((k_jacobi<T, 4, true>), g, b, 0, s, M, P, Qx, lam, D, r, nullptr, xn);
    else
      hipLaunchKernelGGL((k_jacobi<T, 6, true>), g, b, 0, s, M, P, Qx, lam, D, r, nullptr, xn);
  } else if (M.nf == 4) {
    hipLaunchKernelGGL((k_jacobi<T, 4, false>), g, b, 0, s, M, P, Qx, lam, D, r, xo, xn);
  } else {
    hipLaunchKernelGGL((k_jacobi<T, 6, false>), g, b, 0, s, M, P, Qx, lam, D, r, xo, xn);
  }
}
template <typename T>
void launch_amatvec(const DevMesh<T>& M, const Params& P, const T* Qx, const T* lam, const T* D, const double* x,
                    double* out, hipStream_t s) {
  if (M.nf == 4)
    hipLaunchKernelGGL((k_amatvec<T, 4>), dim3(nblk(M.N, 256)), dim3(256), 0, s, M, P, Qx, lam, D, x, out);
  else
    hipLaunchKernelGGL((k_amatvec<T, 6>), dim3(nblk(M.N, 256)), dim3(256), 0, s, M, P, Qx, lam, D, x, out);
}
template <typename T>
void launch_lusgs(const DevMesh<T>& M, const Params& P, const T* Qx, const T* lam, const T* D,
                  const std::vector<int>& start, const double* r, double* y, double* x, hipStream_t s) {
  const int nc = (int)start.size() - 1;
  for (int c = 0; c < nc; ++c) {
    int cnt = start[c + 1] - start[c];
    if (cnt && M.nf == 4)
      hipLaunchKernelGGL((k_lusgs<T, true, 4>), dim3(nblk(cnt, 256)), dim3(256), 0, s, M, P, Qx, lam, D, start[c],
                         cnt, c, r, y);
    else if (cnt)
      hipLaunchKernelGGL((k_lusgs<T, true, 6>), dim3(nblk(cnt, 256)), dim3(256), 0, s, M, P, Qx, lam, D, start[c],
                         cnt, c, r, y);
  }
  for (int c = nc - 1; c >= 0; --c) {
    int cnt = start[c + 1] - start[c];
    if (cnt && M.nf == 4)
      hipLaunchKernelGGL((k_lusgs<T, false, 4>), dim3(nblk(cnt, 256)), dim3(256), 0, s, M, P, Qx, lam, D, start[c],
                         cnt, c, (const double*)y, x);
    else if (cnt)
      hipLaunchKernelGGL((k_lusgs<T, false, 6>), dim3(nblk(cnt, 256)), dim3(256), 0, s, M, P, Qx, lam, D, start[c],
                         cnt, c, (const double*)y, x);
  }
}
template <typename T>
void launch_perturb(const double* Q, const double* v, const double* sigma, int N, int NX, T* Qp, hipStream_t s) {
  hipLaunchKernelGGL(k_perturb<T>, dim3(nblk(N, 256)), dim3(256), 0, s, Q, v, sigma, N, NX, Qp);
}
template <typename T>
void launch_check(const T* Qx, int N, int NX, double gamma, int* bad, hipStream_t s) {
  hipLaunchKernelGGL(k_check<T>, dim3(nblk(N, 256)), dim3(256), 0, s, Qx, N, NX, gamma, bad);
}

void launch_dot(const double* x, const double* y, size_t n, double* part, double* out, bool sq, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_part<0>, dim3(RGRID), dim3(RB), 0, s, x, y, n, part);
  if (sq)
    hipLaunchKernelGGL(k_reduce_final<true>, dim3(1), dim3(RB), 0, s, part, out);
  else
    hipLaunchKernelGGL(k_reduce_final<false>, dim3(1), dim3(RB), 0, s, part, out);
}
void launch_abssum(const double* x, size_t n, double* part, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_part<1>, dim3(RGRID), dim3(RB), 0, s, x, x, n, part);
  hipLaunchKernelGGL(k_reduce_final<false>, dim3(1), dim3(RB), 0, s, part, out);
}
void launch_dot_part(const double* x, const double* y, size_t n, double* part, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_part<0>, dim3(RGRID), dim3(RB), 0, s, x, y, n, part);
}
void launch_reduce_final(const double* part, double* out, bool sq, hipStream_t s) {
  if (sq)
    hipLaunchKernelGGL(k_reduce_final<true>, dim3(1), dim3(RB), 0, s, part, out);
  else
    hipLaunchKernelGGL(k_reduce_final<false>, dim3(1), dim3(RB), 0, s, part, out);
}
void launch_axpy_dot_chain(const double* pin, double* hout, const double* v, double* w, size_t n, const double* z,
                           double* pout, hipStream_t s) {
  hipLaunchKernelGGL(k_axpy_dot_chain, dim3(RGRID), dim3(RB), 0, s, pin, hout, v, w, n, z, pout);
}
void launch_axpy_dev(const double* x, double* y, size_t n, const double* a, double sgn, hipStream_t s) {
  hipLaunchKernelGGL(k_axpy_dev, dim3(nblk(n, 256)), dim3(256), 0, s, x, y, n, a, sgn);
}
void launch_update_limited(double* Q, const double* dQ, int N, double th, double gamma, int* nlim, hipStream_t s) {
  hipLaunchKernelGGL(k_update_limited, dim3(nblk((size_t)N, 256)), dim3(256), 0, s, Q, dQ, N, th, gamma, nlim);
}
void launch_scale_inv(const double* x, double* y, size_t n, const double* a, hipStream_t s, const int* skip) {
  hipLaunchKernelGGL(k_scale_inv, dim3(nblk(n, 256)), dim3(256), 0, s, x, y, n, a, skip);
}
void launch_gmres_start(const double* beta, double* G, int* st, int m, hipStream_t s) {
  hipLaunchKernelGGL(k_gmres_start, dim3(1), dim3(1), 0, s, beta, G, st, m);
}
void launch_gmres_column(int j, int m, const double* hc, double* G, int* st, hipStream_t s) {
  hipLaunchKernelGGL(k_gmres_column, dim3(1), dim3(1), 0, s, j, m, hc, G, st);
}
void launch_gmres_solve(int m, const double* G, const int* st, double* y, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_gmres_solve, dim3(1), dim3(1), 0, s, m, G, st, y, out);
}
void launch_combine(const double* V, const double* c, int nv, size_t n, const double* x, double* y, hipStream_t s) {
  hipLaunchKernelGGL(k_combine, dim3(nblk(n, 256)), dim3(256), 0, s, V, c, nv, n, x, y);
}
void launch_convert(const double* src, float* dst, size_t n, hipStream_t s) {
  if (n) hipLaunchKernelGGL(k_convert, dim3(nblk(n, 256)), dim3(256), 0, s, src, dst, n);
}
void launch_sigma(const double* vpart, const double* qq, double n, double eps, double fixed, double* sigma,
                  hipStream_t s, const double* rpart, double eta, const double* noise, double* vnorm) {
  hipLaunchKernelGGL(k_sigma, dim3(1), dim3(RB), 0, s, vpart, qq, n, eps, fixed, sigma, rpart, eta, noise, vnorm);
}
void launch_diff_norm(const double* x, const double* y, size_t n, double* part, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_part<2>, dim3(RGRID), dim3(RB), 0, s, x, y, n, part);
  hipLaunchKernelGGL(k_reduce_final<true>, dim3(1), dim3(RB), 0, s, part, out);
}
void launch_norm_ratio(const double* x, size_t n, const double* den, double* part, double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_reduce_part<0>, dim3(RGRID), dim3(RB), 0, s, x, x, n, part);
  hipLaunchKernelGGL(k_reduce_norm_ratio, dim3(1), dim3(RB), 0, s, part, den, out);
}
void launch_relax_grad(double* G, const double* Gnew, int N, int NX, double w, hipStream_t s) {
  if (N > 0) hipLaunchKernelGGL(k_relax_grad, dim3(nblk((size_t)15 * N, 256)), dim3(256), 0, s, G, Gnew, N, NX, w);
}
void launch_ratio_part(const double* Q, const double* v, int N, double* part, hipStream_t s) {
  hipLaunchKernelGGL(k_ratio_part, dim3(RGRID), dim3(RB), 0, s, Q, v, N, part);
}

// Work space of the allocation-free residual entry point: one copy per GPU,
// held until the process ends.  Host code never passes the array's name to a
// kernel or a copy: on the host it is a stand-in, not a device address.  The
// device address is looked up once per device (with that device current) and
// cached.
static __device__ __align__(256) unsigned char scratch[STATIC_SCRATCH_BYTES];

hipError_t static_scratch_ptr(void** out) {
  static std::mutex mu;
  static void* ptrs[MAX_DEVICES] = {};
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= MAX_DEVICES) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(mu);
  if (!ptrs[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    ptrs[dev] = p;
  }
  *out = ptrs[dev];
  return hipSuccess;
}

#define HGKS_INST(T)                                                                                              \
  template void launch_ghost<T>(const DevMesh<T>&, const Params&, T*, T*, hipStream_t);                           \
  template void launch_recon<T>(const DevMesh<T>&, const Params&, const T*, const T*, T*, hipStream_t);           \
  template void launch_side<T>(const DevMesh<T>&, const Params&, const T*, const T*, T*, int*, hipStream_t);      \
  template void launch_flux<T>(const DevMesh<T>&, const Params&, const T*, const T*, T*, T*, bool, hipStream_t);  \
  template void launch_flux_kfvs<T>(const DevMesh<T>&, const Params&, const T*, T*, hipStream_t);           \
  template void launch_dt<T>(const DevMesh<T>&, const Params&, double, const T*, T*, hipStream_t);                \
  template void launch_lambda_diag<T>(const DevMesh<T>&, const Params&, const T*, const T*, T*, T*, hipStream_t); \
  template void launch_jacobi<T>(const DevMesh<T>&, const Params&, const T*, const T*, const T*, const double*,   \
                                 const double*, double*, hipStream_t);                                           \
  template void launch_amatvec<T>(const DevMesh<T>&, const Params&, const T*, const T*, const T*, const double*,  \
                                  double*, hipStream_t);                                                         \
  template void launch_lusgs<T>(const DevMesh<T>&, const Params&, const T*, const T*, const T*,                \
                               const std::vector<int>&, const double*, double*, double*, hipStream_t);         \
  template void launch_perturb<T>(const double*, const double*, const double*, int, int, T*, hipStream_t);        \
  template void launch_check<T>(const T*, int, int, double, int*, hipStream_t);
HGKS_INST(double)
HGKS_INST(float)
template void launch_gather<double, double>(const DevMesh<double>&, int, const double*, const double*, double*,
                                            const double*, const double*, const double*, const double*, double*,
                                            hipStream_t);
template void launch_gather<float, double>(const DevMesh<float>&, int, const float*, const float*, double*,
                                           const double*, const double*, const float*, const double*, double*,
                                           hipStream_t);

}  // namespace hgks
