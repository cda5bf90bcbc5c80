// Device data structures and math shared by the HGKS kernels (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hgks {

// Read-only mesh data resident in HBM (SoA, index fastest over cells/faces).
// Floating-point arrays are of type T (double for the plain path, float for
// the inner operator of the mixed-precision form).
template <typename T>
struct DevMesh {
  int N;    // cells
  int F;    // faces; fR >= N marks a boundary face
  int Nb;   // boundary faces = ghost cells
  int NX;   // N + Nb, leading dimension of extended state arrays
  int nf;   // faces per cell: 4 tetrahedra, 6 hexahedra
  int ng;   // Gauss points per face: 3 triangles, 4 quadrilaterals
  int nbig; // slots of the non-compact stencil (16 tetrahedra; the mesh's largest for hexahedra)
  const T* vol;        // [N]
  const T* h;          // [N]   |Omega|^(1/3)
  const T* hdt;        // [N]   3|Omega| / max face area
  const T* m2s;        // [6][N] second central moments / h^2 (xx,yy,zz,xy,xz,yz)
  const int* fL;       // [F]
  const int* fR;       // [F]   >= N: ghost N+g
  const int* fkind;    // [F]   boundary kind, -1 interior
  const T* fn;         // [3][F] unit normal L -> R
  const T* fS;         // [F]
  const T* fxiL;       // [3 ng][F] (gp*3+dir) scaled offsets (x_g - c_L)/h_L
  const T* fxiR;       // [3 ng][F]
  const T* fw;         // [ng][F] Gauss weights of quadrilateral faces (null for tetrahedra)
  const int* cface;    // [nf][N] signed face ids: f+1 if the cell is L, -(f+1) if R
  const int* gowner;   // [Nb]
  const int* gface;    // [Nb]
  // non-compact WENO
  const int* stn;      // [nbig][N] big stencil (extended ids), padded with the cell itself
  const T* opA;        // [9 nbig][N] P0 operator, row k*nbig+j
  const int* sstn;     // [24][N] sub-stencil members (extended ids), padded with the cell:
                       // 4 x 6 (tetrahedra) or 8 x 3 (hexahedra)
  const T* opB;        // [72][N] P_m operators, row (s*3+t)*6+r (tetrahedra), (s*3+t)*3+r (hexahedra)
  const uint8_t* smask;// [N]  bit s set = sub-stencil s usable
  // compact HWENO
  const int* nbf;      // [nf][N] face neighbours (extended ids)
  const T* opH;        // [9 (4 nf + 3)][N] P0 operator: rows k*(4nf+3)+j, j<nf averages, then gradients
  const T* hsub;       // [6 nf][N] per sub s: wi, wm, dx, dy, dz, 1/|d|^2
  // LU-SGS
  const int* ccol;     // [N]  colour of the cell
  const int* cord;     // [N]  cell ids sorted by colour
};

struct Params {
  double gamma, K, tau_eps, tau_C, gamma_lin, weno_eps, mu, prandtl;
  double flux_scale;  // time interval of the flux average / implicit time step
  double rhoinf, uinf0, uinf1, uinf2, pinf;
  int physics, weights, scheme;
  int csubs;  // hexahedra, compact scheme: 1 = the eight S^WENO sub-stencils from the cell averages
};

// Tangent rule: t1 = normalise(n x e_k), e_k the axis of smallest |n_k|
// (ties -> lowest k), t2 = n x t1.
template <typename T>
__device__ __forceinline__ void face_frame(T n0, T n1, T n2, T t1[3], T t2[3]) {
  T a0 = fabs(n0), a1 = fabs(n1), a2 = fabs(n2);
  int k = 0;
  T am = a0;
  if (a1 < am) { k = 1; am = a1; }
  if (a2 < am) { k = 2; }
  T c0, c1, c2;  // n x e_k
  if (k == 0) { c0 = 0; c1 = n2; c2 = -n1; }
  else if (k == 1) { c0 = -n2; c1 = 0; c2 = n0; }
  else { c0 = n1; c1 = -n0; c2 = 0; }
  T inv = T(1) / sqrt(c0 * c0 + c1 * c1 + c2 * c2);
  t1[0] = c0 * inv; t1[1] = c1 * inv; t1[2] = c2 * inv;
  t2[0] = n1 * t1[2] - n2 * t1[1];
  t2[1] = n2 * t1[0] - n0 * t1[2];
  t2[2] = n0 * t1[1] - n1 * t1[0];
}

}  // namespace hgks
