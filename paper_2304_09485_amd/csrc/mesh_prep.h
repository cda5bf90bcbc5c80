// Host preprocessing of a tetrahedral mesh: faces, geometry, ghost cells,
// reconstruction stencils (paper Sec. 3.1) and the per-cell least-squares
// operators of the WENO (Sec. 3.2) and HWENO (Sec. 3.3) reconstructions.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

namespace hgks {

struct HostMesh {
  int N = 0, F = 0, Nb = 0;
  // cell shape: faces per cell, Gauss points per face, slots of the
  // non-compact stencil (cells other than the cell itself), non-compact
  // sub-stencils and their members other than the cell
  int nf = 4, ng = 3, nbig = 16, nsw = 4, msw = 6;
  // cells
  std::vector<double> vol, h, hdt, m2s;  // m2s [6][N]
  std::vector<double> cen;               // [3][N]
  // faces
  std::vector<int> fL, fR, ftag;         // ftag: boundary tag or -1
  std::vector<double> fn, fS, fxiL, fxiR;// fn [3][F], fxi [3 ng][F]
  std::vector<double> fw;                // [ng][F] Gauss weights of quadrilateral faces (empty for tets)
  std::vector<int> cface;                // [nf][N]
  // ghosts
  std::vector<int> gowner, gface;
  // WENO
  std::vector<int> stn, sstn;            // [nbig][N], [nsw msw][N]
  std::vector<double> opA, opB;          // [9 nbig][N], [nsw 3 msw][N]
  std::vector<uint8_t> smask;            // [N]
  // HWENO
  std::vector<int> nbf;                  // [nf][N]
  std::vector<double> opH, hsub;         // [9 (nf + 3 (nf + 1))][N], [6 nf][N]
  // diagnostics
  int64_t n_big_fallback = 0, n_sub_dropped = 0;
  double total_volume = 0.0;
};

// Hexahedral mesh: hex2node [n_hex][8] (0-3 the bottom quadrilateral
// counter-clockwise seen from above, 4-7 the top one above them), boundary
// quadrilaterals bf [n_bf][4].  Trilinear cells, bilinear faces with 2x2
// Gauss points; the eight non-compact sub-stencils of Sec. 3.1.
int build_host_hex_mesh(HostMesh& H, int64_t n_nodes, const double* xyz, int64_t n_hex, const int32_t* hex2node,
                        int64_t n_bf, const int32_t* bf, const int32_t* btag, std::string& err);

// Greedy colouring of the face-neighbour graph for the LU-SGS sweeps: cells
// in index order each take the smallest colour no already coloured face
// neighbour has (at most 5 colours for tets).  col [N]; order: cell ids sorted
// by colour (stable); start [ncol + 1]: offsets of the colour classes in order.
int colour_cells(const HostMesh& H, std::vector<int>& col, std::vector<int>& order, std::vector<int>& start);

// Returns 0 on success, -3 (mesh error) or -1 (bad argument) with err set.
int build_host_mesh(HostMesh& H, int64_t n_nodes, const double* xyz, int64_t n_tets, const int32_t* tet2node,
                    int64_t n_bf, const int32_t* bf, const int32_t* btag, std::string& err);

}  // namespace hgks
