/* CPU FP64 oracle of the implicit high-order gas-kinetic scheme (HGKS) on
 * tetrahedral meshes.
 *
 * TEST INFRASTRUCTURE ONLY.  This is the plain, slow reference the HIP path is
 * checked against; the product library never links, loads or calls it.  It
 * shares no code with the library: it derives geometry, stencils,
 * reconstruction and the gas-kinetic flux on its own, literally following the
 * paper's steps (Sec. 2 Eq. (flux); Sec. 3.1-3.4 Eq. (polys), (compact-big-1/2),
 * (weno); Sec. 4 Eq. (impsystem), (frechet), (deri-matrix), (precond),
 * Algorithm 1).
 *
 * Layouts: conserved state Q is variable-major [5][N] (rho, rho U, rho V,
 * rho W, rho E); cell-averaged gradients are [15][N] with row var*3+dir
 * (Cartesian, global frame).  All arrays are host memory owned by the caller.
 */
#ifndef HGKS_ORACLE_H
#define HGKS_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
  int32_t scheme;        /* 0 non-compact WENO, 1 compact HWENO */
  int32_t physics;       /* 0 Euler, 1 Navier-Stokes */
  int32_t weights;       /* 0 nonlinear WENO-Z type, 1 linear */
  int32_t krylov_dim;    /* 10 */
  int32_t restarts;      /* 3 */
  int32_t jacobi_sweeps; /* 2 */
  double gamma;          /* 1.4 */
  double cfl;            /* 10 */
  double tau_eps;        /* 0.1 */
  double tau_C;          /* 1 */
  double gamma_lin;      /* 0.025 */
  double weno_eps;       /* 1e-5 (reading A8) */
  double mu;             /* dynamic viscosity (NS) */
  double prandtl;        /* NS */
  double fd_sigma;       /* 0 = automatic */
  double cfl_flux;       /* CFL of the flux time average; 0 = same as cfl */
  int32_t jv_mode;       /* GMRES operator: 0 FD product of Eq. (frechet), 1 the approximate
                            matrix A of Eq. (deri-matrix) */
  int32_t first_order;   /* 1: first-order KFVS flux of the cell averages (Sec. 5, the
                            supersonic sphere retested with a first-order flux) */
  int32_t solver;        /* implicit step: 0 GMRES, 1 LU-SGS of the approximate matrix (the
                            LUSGS-WENO comparison solver of Sec. 5) */
  int32_t compact_subs;   /* sub-stencils of the compact scheme: 0 the faces' {i, i_f} (Sec. 3.1,
                            gradient-dominated), 1 on hexahedra the eight S^WENO sub-stencils
                            {i, i_1 or i_6, two consecutive lateral neighbours}, fitted from the
                            cell averages (the hexahedral compact choice of the sphere cases of
                            Sec. 5) */
  double max_update;     /* 0: Q^{n+1} = Q^n + dQ (the paper); theta > 0: each cell's dQ scaled
                            by the largest 2^-k (k <= 20) for which its density and pressure
                            change by at most theta of their old values (a runtime policy of
                            the library for impulsive starts; steady states are unchanged) */
  double grad_relax;     /* compact scheme: G <- G + omega (G_new - G), omega in (0, 1]; 1: G_new
                            (Sec. 4.2); the steady state is the same for every omega */
} orc_options;

/* boundary kinds */
enum { ORC_FARFIELD = 0, ORC_SLIP = 1, ORC_NOSLIP = 2, ORC_SUP_IN = 3, ORC_SUP_OUT = 4 };

typedef struct orc_ctx orc_ctx;

/* kind_of_tag[t] gives the boundary kind of boundary tag t (0 <= t < n_tags).
 * Returns NULL on a bad mesh; orc_error() then holds the reason. */
orc_ctx* orc_create(int64_t n_nodes, const double* xyz, int64_t n_tets, const int32_t* tets,
                    int64_t n_bf, const int32_t* bf, const int32_t* btag, int32_t n_tags,
                    const int32_t* kind_of_tag, const double* freestream_prim,
                    const orc_options* opts);
/* Hexahedral mesh (reading A30): hexes [n_hex][8] with nodes 0-3 the bottom
 * quadrilateral counter-clockwise seen from above and 4-7 the top one above
 * them (positive trilinear Jacobian); boundary quadrilaterals bf [n_bf][4]. */
orc_ctx* orc_create_hex(int64_t n_nodes, const double* xyz, int64_t n_hex, const int32_t* hexes,
                        int64_t n_bf, const int32_t* bf, const int32_t* btag, int32_t n_tags,
                        const int32_t* kind_of_tag, const double* prim, const orc_options* opts);
/* Gauss points per face (3 triangles, 4 quadrilaterals) and faces per cell */
int32_t orc_face_points(const orc_ctx*);
int32_t orc_cell_faces(const orc_ctx*);
const char* orc_error(void);
void orc_destroy(orc_ctx*);
void orc_set_threads(int32_t n);
int64_t orc_n_cells(const orc_ctx*);
int64_t orc_n_faces(const orc_ctx*);

/* per-cell geometry: vol[N], centroid[3][N], second central moment [6][N]
 * (xx,yy,zz,xy,xz,yz per unit volume) */
void orc_geometry(const orc_ctx*, double* vol, double* cen, double* m2);
/* per-face geometry: L[F], R[F] (R<0: boundary, -R-1 = ghost id), area[F],
 * normal[3][F], gauss points [9][F] (gp*3+dir) */
void orc_faces(const orc_ctx*, int32_t* L, int32_t* R, double* area, double* nrm, double* gp);
/* stencil sizes and members (extended index: >= N means ghost N+g) */
int32_t orc_stencil(const orc_ctx*, int64_t cell, int32_t which /* 0 big, 1..4 sub */,
                    int32_t* members, int32_t cap);

/* local time step Delta t_i */
void orc_dt(const orc_ctx*, const double* Q, double* dt);

/* residual L(Q) [5][N]; dt NULL -> computed from Q; gradQ needed for HWENO;
 * gradQ_new (HWENO, may be NULL) receives the gradient update from f.
 * Returns the number of positivity fallbacks. */
int64_t orc_residual(const orc_ctx*, const double* Q, const double* gradQ, const double* dt,
                     double* R, double* gradQ_new);

/* side reconstruction of face f, side s (0 = L, 1 = R): out [3 gp][4][5]
 * (value, d/dn, d/dt1, d/dt2) in the face's local frame; returns fallback flag */
int32_t orc_side_values(const orc_ctx*, const double* Q, const double* gradQ, int64_t f,
                        int32_t side, double* out);
/* face frame: n, t1, t2 (9 doubles) */
void orc_face_frame(const orc_ctx*, int64_t f, double* out9);

/* time-averaged gas-kinetic flux at one point in the local frame; W* are
 * conserved local-frame states, d* are [3][5] derivatives along (n, t1, t2).
 * Outputs F[5] and, if QG != NULL, the point value Q(x_G, dt) of Eq. (point). */
void orc_gks_point(const orc_ctx*, const double* Wl, const double* dWl, const double* Wr,
                   const double* dWr, double dt, double* F, double* QG);

/* first-order KFVS flux of two local-frame conserved states (cell averages):
 * F[5] and, if QG != NULL, the half-space density moments rho_l <psi>_{u>0} +
 * rho_r <psi>_{u<0} */
void orc_kfvs_point(const orc_ctx*, const double* Wl, const double* Wr, double* F, double* QG);

/* normalised Maxwellian velocity moments <u^a v^b w^c xi^(2d)> (half: +1 u>0,
 * -1 u<0, 0 full) and slope solve <a psi> = b of Sec. 2 */
double orc_moment(double U, double V, double W, double lam, double K, int32_t half, int32_t a,
                  int32_t b, int32_t c, int32_t d);
void orc_slope_solve(double U, double V, double W, double lam, double K, const double* rhs,
                     double* a);

/* Euler flux Jacobian times vector J_n(Q) x */
void orc_euler_jn(double gamma, const double* Q, const double* n, const double* x, double* out);

/* approximate-matrix pieces of Eq. (deri-matrix): D[N] and Jacobi P^{-1} */
void orc_diag(const orc_ctx*, const double* Q, const double* dt, double* D);
void orc_precond(const orc_ctx*, const double* Q, const double* dt, const double* r, double* out);
/* A x with A = D + L + U of Eq. (deri-matrix) (boundary off-diagonal blocks dropped) */
void orc_amatvec(const orc_ctx*, const double* Q, const double* dt, const double* x, double* out);

/* FD Jacobian-vector product (|Omega|/dt) v - (L(Q + sigma v) - b)/sigma;
 * sigma <= 0 -> automatic; returns the sigma used */
double orc_jv(const orc_ctx*, const double* Q, const double* gradQ, const double* dt,
              const double* b, const double* v, double sigma, double* Av);

typedef struct {
  double res;            /* L1 density residual of L(Q^n) / sum |Omega| */
  double gmres_rel;      /* final GMRES estimate / initial preconditioned norm */
  int64_t n_resid_evals;
  int64_t n_fallbacks;
  int64_t n_limited;     /* cells whose update was scaled (max_update) */
} orc_step_info;

/* one implicit step (Algorithm 1 body); Q, gradQ updated in place */
int32_t orc_implicit_step(const orc_ctx*, double* Q, double* gradQ, orc_step_info* info);

/* greedy colouring of the cells' face-neighbour graph (col [N]); returns the
 * number of colours */
int32_t orc_colours(const orc_ctx*, int32_t* col);

/* LU-SGS solve (D + L) D^-1 (D + U) dQ = R with the approximate matrix of
 * Eq. (deri-matrix) at state Q and time steps dt; L / U hold the blocks to
 * neighbours of lower / higher colour */
void orc_lusgs(const orc_ctx*, const double* Q, const double* dt, const double* R, double* dQ);

/* L1 density residual norm */
double orc_res_norm(const orc_ctx*, const double* R);

#ifdef __cplusplus
}
#endif
#endif
