/* hgks.h -- C ABI of the MI355X implementation of the implicit high-order
 * gas-kinetic scheme (HGKS) for steady compressible flow on tetrahedral meshes
 * (Yang, Pan, Xu, "Implicit high-order gas-kinetic schemes for compressible
 * flows on three-dimensional unstructured meshes I: steady flows").
 *
 * The library evaluates the residual L(Q) of the semi-discrete finite-volume
 * scheme (Sec. 2, Eq. (semi)-(finite)) with third-order WENO (Sec. 3.2) or
 * compact HWENO (Sec. 3.3) reconstruction and the time-averaged BGK
 * gas-kinetic flux (Sec. 2 Eq. (flux), Sec. 4.1), and drives backward-Euler
 * implicit steps (Sec. 4.1 Eq. (impEuler)-(impsystem)) with restarted,
 * Jacobi-preconditioned GMRES (Sec. 4.2 Eq. (precond), Algorithm 1) whose
 * operator is the matrix-free finite-difference product of Eq. (frechet).
 *
 * Conventions
 *   - Every function returns hgks_status (0 = OK, < 0 = error), never throws
 *     and never aborts; hgks_last_error(ctx) holds a message.
 *   - Conserved state Q is variable-major [5][N] doubles: rho, rho U, rho V,
 *     rho W, rho E, in the caller's tet order.  Cell-averaged gradients are
 *     [15][N] doubles, row var*3 + dir, Cartesian global frame.
 *   - Host arrays passed in are copied during the call and stay owned by the
 *     caller; output arrays are caller-allocated.  Device pointers passed to
 *     the *_dev functions are borrowed for the call, in stream order.
 *   - All compute runs on the current HIP device on the context's stream.
 *   - A context is not thread-safe; use one per thread.
 */
#ifndef HGKS_H
#define HGKS_H
#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HGKS_OK = 0,
  HGKS_EINVAL = -1,  /* bad argument or call order */
  HGKS_ENOMEM = -2,  /* device or host allocation failed */
  HGKS_EMESH = -3,   /* non-manifold, inverted or degenerate tet, unmatched boundary face */
  HGKS_ESTATE = -4,  /* NaN, rho <= 0 or p <= 0 in a state */
  HGKS_ENOCONV = -5, /* solve did not reach the requested drop */
  HGKS_EDEVICE = -6  /* HIP runtime error */
} hgks_status;

/* spatial scheme: non-compact WENO (Sec. 3.2), compact HWENO (Sec. 3.3), or
 * the first-order kinetic flux vector splitting of the cell averages that the
 * Mach 3 sphere case of Sec. 5 is retested with (no reconstruction, free
 * transport of the two half-space Maxwellians; inviscid only) */
enum { HGKS_WENO = 0, HGKS_HWENO = 1, HGKS_KFVS1 = 2 };
enum { HGKS_EULER = 0, HGKS_NS = 1 };                /* collision time of Sec. 5 */
enum { HGKS_FP64 = 0, HGKS_FP32_INNER = 1 };         /* arithmetic of the GMRES inner operator */
enum { HGKS_WEIGHTS_NONLINEAR = 0, HGKS_WEIGHTS_LINEAR = 1 }; /* Sec. 3.4 */
/* GMRES operator of the implicit step: the matrix-free FD product of the
 * high-order residual, Eq. (frechet), or the first-order approximate matrix
 * A of Eq. (deri-matrix), applied without being stored (the paper's solver,
 * Sec. 4.2: one high-order residual evaluation per step) */
enum { HGKS_JV_FD = 0, HGKS_JV_APPROX = 1 };
/* implicit solver of each step: restarted GMRES (Sec. 4.2) on the operator
 * jv_mode selects, or one LU-SGS solve (D + L) D^-1 (D + U) dQ = L(Q^n) of the
 * approximate matrix A = D + L + U of Eq. (deri-matrix), L / U being its
 * blocks to neighbours of lower / higher colour in a greedy colouring of the
 * cells (the LUSGS-WENO solver the paper compares with, Sec. 5); one residual
 * evaluation per step, jv_mode / precision / krylov options unused */
enum { HGKS_SOLVER_GMRES = 0, HGKS_SOLVER_LUSGS = 1 };
enum { HGKS_SUBS_FACES = 0, HGKS_SUBS_HEX_WENO = 1 };
enum { HGKS_FARFIELD = 0, HGKS_SLIP_WALL = 1, HGKS_NOSLIP_ADIABATIC = 2,
       HGKS_SUP_IN = 3, HGKS_SUP_OUT = 4 };          /* Sec. 5 boundary conditions */

typedef struct {
  int32_t scheme;        /* HGKS_WENO | HGKS_HWENO | HGKS_KFVS1 */
  int32_t physics;       /* HGKS_EULER | HGKS_NS */
  int32_t precision;     /* HGKS_FP64 | HGKS_FP32_INNER */
  int32_t weights;       /* HGKS_WEIGHTS_NONLINEAR | HGKS_WEIGHTS_LINEAR */
  int32_t krylov_dim;    /* 10, Sec. 5 (at most 32) */
  int32_t restarts;      /* 3, Sec. 5 */
  int32_t jacobi_sweeps; /* 2, Sec. 5 */
  int32_t jv_mode;       /* GMRES operator: HGKS_JV_FD (default) or HGKS_JV_APPROX */
  int32_t solver;        /* HGKS_SOLVER_GMRES (default) | HGKS_SOLVER_LUSGS */
  int32_t compact_subs;  /* sub-stencils of the compact scheme (Sec. 3.1): HGKS_SUBS_FACES
                            (default) the faces' {i, i_f}, fitted with the cell gradients;
                            HGKS_SUBS_HEX_WENO (hexahedral meshes only) the eight non-compact
                            sub-stencils {i, i_1 or i_6, two consecutive lateral neighbours},
                            fitted from the cell averages alone, as the hexahedral sphere
                            cases of Sec. 5 choose them */
  double gamma;          /* 1.4 */
  double cfl;            /* 10 */
  double tau_eps;        /* 0.1, inviscid collision time, Sec. 5 */
  double tau_C;          /* 1, pressure-jump term of the collision time, Sec. 5 */
  double gamma_lin;      /* 0.025, linear weights gamma_m, Sec. 3.4 */
  double weno_eps;       /* 1e-5, epsilon of the nonlinear weights (Sec. 3.4 leaves it open) */
  double mu;             /* dynamic viscosity (NS) */
  double prandtl;        /* Prandtl number (NS), 1 = plain BGK; otherwise the energy flux
                            gets (1/Pr - 1) times the Fourier heat flux -mu c_p dT/dn of
                            the interface state */
  double fd_sigma;       /* FD step of Eq. (frechet); 0 = sqrt(eps) max(1,rms Q)/rms v with
                            eps = 2^-52 (FP64 products) or 2^-23 (FP32 inner products; then
                            capped so that no cell's density, momentum or energy moves by
                            more than 1 %, and at the step that balances the FD truncation
                            against the measured FP32 rounding of the base residual) */
  double cfl_flux;       /* CFL number of the time interval the flux is averaged over
                            (Sec. 4.1); default 1; 0 = the implicit step's cfl */
  double cfl_start;      /* hgks_solve_steady only: CFL of its first step, multiplied by
                            cfl_growth after every step up to cfl; 0 (default) = cfl
                            throughout, as in the paper */
  double cfl_growth;     /* default 1.5 */
  double max_update;     /* 0 (default): Q^{n+1} = Q^n + dQ, as in the paper; theta > 0: each
                            cell's dQ is scaled by the largest 2^-k (k <= 20) for which its
                            density and pressure change by at most theta of their old values
                            (a runtime policy for impulsive starts, e.g. 0.2; a steady state
                            is a fixed point either way) */
  double grad_relax;     /* compact HWENO: the gradients after a step are G + omega (G_new - G)
                            with omega = grad_relax in (0, 1]; 1 (default) takes G_new of
                            Sec. 4.2 as it is.  The steady state (Q, G) is the same for every
                            omega; omega < 1 damps the step-to-step alternation of the
                            gradient fixed-point iteration (a mesh-dependent choice: 0.7
                            to 0.8 on the 202,752-tet sphere shell, 0.5 on a 3,456-tet
                            one).
                            Values outside (0, 1]: HGKS_EINVAL from hgks_create */
  void* stream;          /* hipStream_t to run on; NULL = library-owned stream */
  /* Device allocator hook: every device buffer of a context (mesh data,
   * state, work space, Krylov basis), and so of every served request, comes
   * from dev_alloc(bytes, alloc_user) and goes back through
   * dev_free(ptr, alloc_user) in hgks_destroy, after the context's stream has
   * drained.  dev_alloc returns device memory of the current device, at least
   * 256-byte aligned, or NULL (HGKS_ENOMEM; a misaligned block is handed back
   * and refused the same way).  Both NULL (the default) = hipMalloc / hipFree;
   * setting only one is HGKS_EINVAL.  The Python binding passes PyTorch's
   * caching allocator here.  The hook may be called from the server's
   * worker threads. */
  void* (*dev_alloc)(size_t bytes, void* alloc_user);
  void (*dev_free)(void* ptr, void* alloc_user);
  void* alloc_user;
} hgks_options;

typedef struct {
  double res;            /* L1 density residual of L(Q^n), divided by the total volume */
  double res_rel;        /* res / res of the first step of this context */
  double gmres_rel;      /* last GMRES residual estimate / initial preconditioned norm */
  int64_t n_resid_evals; /* residual evaluations in the step (33 with m = 10, 3 restarts) */
  int64_t n_fallbacks;   /* face sides that fell back to first order (positivity) */
  int64_t n_limited;     /* cells whose update max_update scaled */
  double t_ms;           /* wall time of the step */
} hgks_step_info;

typedef struct {
  int32_t steps;
  int32_t converged;
  double res0, res_final, drop;
  int64_t n_resid_evals;
  double t_ms;
} hgks_solve_info;

typedef struct hgks_ctx hgks_ctx;

/* Fill *opts with the paper's defaults (Sec. 5): WENO, Euler, FP64,
 * nonlinear weights, m = 10, 3 restarts, 2 Jacobi sweeps, CFL 10. */
void hgks_default_options(hgks_options* opts);

/* Create a context on the current HIP device.  opts is copied.  HGKS_EINVAL
 * on an option out of range, and for HGKS_KFVS1 with HGKS_NS. */
hgks_status hgks_create(const hgks_options* opts, hgks_ctx** out);

/* Load a tetrahedral mesh: xyz [n_nodes][3], tet2node [n_tets][4] (any
 * positively oriented: det(x1-x0, x2-x0, x3-x0) > 0; a tet's local face p is
 * the one opposite its local vertex p, Sec. 3.1), boundary triangles
 * bface2node [n_bfaces][3]
 * with integer tags bface_tag [n_bfaces] (0 <= tag < 256).  Builds faces,
 * geometry, ghost cells, stencils and the least-squares operators and uploads
 * them.  HGKS_EMESH on a bad mesh. */
hgks_status hgks_load_mesh(hgks_ctx* ctx, int64_t n_nodes, const double* xyz, int64_t n_tets,
                           const int32_t* tet2node, int64_t n_bfaces, const int32_t* bface2node,
                           const int32_t* bface_tag);

/* Load a hexahedral mesh (Sec. 3.1; the paper's sphere cases use hexahedra):
 * hex2node [n_hex][8], nodes 0-3 the bottom quadrilateral counter-clockwise
 * seen from above and 4-7 the top one above them (a positive Jacobian of the
 * trilinear map at every corner); boundary quadrilaterals bface2node
 * [n_bfaces][4] with tags as for hgks_load_mesh.  Cells are trilinear, faces
 * bilinear with 2x2 Gauss points weighted by the normal component of their
 * area element; the non-compact scheme uses the eight sub-stencils {i, i_1 or
 * i_6, two consecutive lateral neighbours} (local faces 1-6: bottom, the four
 * sides in order around, top), the compact one the six {i, i_f}.  Everything
 * else (schemes, solvers, precision) works as on tetrahedra; the server takes
 * tetrahedral meshes only.  HGKS_EMESH on a bad mesh. */
hgks_status hgks_load_hex_mesh(hgks_ctx* ctx, int64_t n_nodes, const double* xyz, int64_t n_hex,
                               const int32_t* hex2node, int64_t n_bfaces, const int32_t* bface2node,
                               const int32_t* bface_tag);

/* Free stream (rho, U, V, W, p) used by far-field and supersonic-inflow
 * boundaries (Sec. 5). */
hgks_status hgks_set_freestream(hgks_ctx* ctx, const double prim[5]);

/* Boundary kind for a tag (default HGKS_FARFIELD).  params is unused. */
hgks_status hgks_set_bc(hgks_ctx* ctx, int32_t tag, int32_t kind, const double* params);

/* Set / get the state (host, [5][N] and optional [15][N] gradients). */
hgks_status hgks_set_state(hgks_ctx* ctx, const double* Q, const double* gradQ);
hgks_status hgks_get_state(hgks_ctx* ctx, double* Q, double* gradQ);

/* Residual L(Q) of Eq. (finite) with the time-averaged flux of Sec. 4.1 and
 * the local time step computed from Q (host arrays).  Q == NULL uses the
 * current state; gradQ (HWENO) NULL uses the current gradients.
 * gradQ_new (may be NULL) receives the HWENO gradient update of Eq.
 * (derivative).  On a non-physical state returns HGKS_ESTATE after writing R. */
hgks_status hgks_residual(hgks_ctx* ctx, const double* Q, const double* gradQ, double* R,
                          double* gradQ_new);

/* Local time step Delta t_i of the state Q (host, [N]). */
hgks_status hgks_time_step(hgks_ctx* ctx, const double* Q, double* dt);

/* Finite-difference Jacobian-vector product of Eq. (frechet) at the current
 * state with the time step frozen at its value for the current state:
 * Av = (|Omega|/dt) v - (L(Q + sigma v) - L(Q)) / sigma.  sigma <= 0 selects
 * the automatic step.  Host arrays [5][N].  *sigma_used may be NULL.
 * With jv_mode = HGKS_JV_APPROX it returns A v with the approximate matrix
 * of Eq. (deri-matrix) instead (*sigma_used = 0). */
hgks_status hgks_jv(hgks_ctx* ctx, const double* v, double sigma, double* Av, double* sigma_used);

/* Jacobi preconditioner of Eq. (precond) built on the approximate matrix of
 * Eq. (deri-matrix) at the current state: out = P^{-1} r (host [5][N]). */
hgks_status hgks_precond(hgks_ctx* ctx, const double* r, double* out);

/* One implicit step (body of Algorithm 1); updates the state in place. */
hgks_status hgks_implicit_step(hgks_ctx* ctx, hgks_step_info* info);

/* Implicit steps until res/res0 <= drop or max_steps; HGKS_ENOCONV if not. */
hgks_status hgks_solve_steady(hgks_ctx* ctx, double drop, int32_t max_steps, hgks_solve_info* info);

/* Checkpoint / resume of a steady solve.  hgks_checkpoint writes the state,
 * the cell-averaged gradients (compact scheme), the reference residual of
 * res_rel and the CFL number of the next step (the ramp of
 * hgks_solve_steady) to path (written under path.tmp, then renamed over
 * path), with a 64-bit FNV-1a hash of the content.  hgks_restore reads such a
 * file into a context with the same mesh and scheme loaded; the next
 * hgks_solve_steady then continues the interrupted solve: it keeps the
 * restored reference residual and CFL number instead of starting a new ramp
 * and measuring the drop from the resume point (hgks_set_state cancels
 * this).  A file for another mesh or scheme, of another format version, a
 * truncated or corrupted file gives HGKS_EINVAL and leaves the context's
 * state unchanged.  The file is host-endian and not portable across byte
 * orders. */
hgks_status hgks_checkpoint(hgks_ctx* ctx, const char* path);
hgks_status hgks_restore(hgks_ctx* ctx, const char* path);

/* Device-pointer twins (caller's HIP stream; NULL = context stream):
 * Q_dev [5][N] doubles, R_dev [5][N] doubles. */
hgks_status hgks_residual_dev(hgks_ctx* ctx, const void* Q_dev, void* R_dev, void* stream);
hgks_status hgks_jv_dev(hgks_ctx* ctx, const void* v_dev, double sigma, void* Av_dev, void* stream);

/* Allocation-free twin of hgks_residual_dev, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments and the same kernels and
 * results (bitwise) as hgks_residual_dev, but the residual's work space
 * (extended state, time steps, reconstruction coefficients, side values,
 * face fluxes) lives in one static 64 MiB device buffer per GPU instead of the
 * context, so the call allocates nothing; the buffer's device address is
 * looked up on the first call on a device.  Meshes whose work space exceeds
 * the buffer (hgks_residual_static_bytes; about 3 KB per tetrahedron, so up
 * to roughly 22,000 tetrahedra) give HGKS_EINVAL before anything is queued.
 * All calls on one GPU share the buffer and it keeps the last call's
 * contents: calls that overlap on one GPU (concurrent streams or threads)
 * race and must be serialised by the caller. */
hgks_status hgks_residual_dev_static(hgks_ctx* ctx, const void* Q_dev, void* R_dev, void* stream);
/* Work-space bytes hgks_residual_dev_static needs for the loaded mesh (0 if none). */
size_t hgks_residual_static_bytes(const hgks_ctx* ctx);

/* Number of cells / faces of the loaded mesh. */
int64_t hgks_n_cells(const hgks_ctx* ctx);
int64_t hgks_n_faces(const hgks_ctx* ctx);
/* Implicit steps the context has completed (hgks_implicit_step, and the
 * steps of hgks_solve_steady); safe to call from another thread while the
 * context works, for progress reporting. */
int64_t hgks_steps_done(const hgks_ctx* ctx);

/* Per-kernel timing of the last residual evaluation, in ms (HIP events on
 * the context stream): names[k] and ms[k] for k < *n (cap entries). */
hgks_status hgks_kernel_times(hgks_ctx* ctx, const char** names, double* ms, int32_t* n, int32_t cap);

const char* hgks_last_error(const hgks_ctx* ctx);
void hgks_destroy(hgks_ctx* ctx);

/* ---------------------------------------------------------------------------
 * Serving: continuous batching of steady solves (Algorithm 1 run to a residual
 * drop) on one GPU.  Requests are queued on submission and admitted as soon
 * as a slot is free and their estimated device footprint fits the HBM budget:
 * of the queued requests that fit, the smallest footprint first (ties in
 * arrival order); a request that has waited more than 60 s goes next and is
 * passed by no other.  Every admitted request owns a context (mesh data, state, Krylov
 * basis resident in HBM) and a HIP stream driven by its own host thread, so
 * the work of concurrent requests overlaps on the device.  Results of a
 * request do not depend on what else runs (no shared mutable device state,
 * deterministic kernels and reductions).  All server calls are thread-safe.
 * ------------------------------------------------------------------------- */
typedef struct hgks_server hgks_server;

typedef struct {
  int64_t n_nodes;
  const double* xyz;        /* [n_nodes][3] */
  int64_t n_tets;
  const int32_t* tet2node;  /* [n_tets][4] */
  int64_t n_bfaces;
  const int32_t* bface2node;/* [n_bfaces][3] */
  const int32_t* bface_tag; /* [n_bfaces] */
  int32_t n_bc;             /* boundary kinds per tag */
  const int32_t* bc_tag;
  const int32_t* bc_kind;
  double prim_inf[5];       /* free stream (rho, U, V, W, p); also the initial state */
  hgks_options opts;        /* scheme, physics, precision, ...; stream is ignored */
  double drop;              /* target res/res0, e.g. 1e-8 */
  int32_t max_steps;
} hgks_request;             /* all arrays are copied by hgks_server_submit */

typedef struct {
  int32_t status;           /* hgks_status of the solve (HGKS_ENOCONV if max_steps hit) */
  int32_t steps;
  double res0, res_final;
  int64_t n_cells;
  int64_t n_resid_evals;
  double t_queue_ms;        /* submission -> admission */
  double t_solve_ms;        /* admission -> result (includes mesh preprocessing) */
  double t_total_ms;        /* submission -> result */
  size_t footprint_bytes;   /* estimate used for admission */
} hgks_result;

typedef struct {
  int32_t queued, active, done;
  size_t bytes_in_use, budget;
  int64_t cell_resid_evals; /* sum over finished requests of cells x residual evaluations */
  int64_t steps_done;       /* implicit steps of all requests so far, finished and running */
} hgks_server_info;

/* Device bytes a request of this size needs (the admission estimate). */
size_t hgks_estimate_bytes(int64_t n_tets, int64_t n_bfaces, const hgks_options* opts);

hgks_status hgks_server_create(size_t hbm_budget_bytes, int32_t max_slots, hgks_server** out);
hgks_status hgks_server_submit(hgks_server* srv, const hgks_request* req, int64_t* ticket);
/* *done = 1 and *out filled when the request has finished */
hgks_status hgks_server_poll(hgks_server* srv, int64_t ticket, int32_t* done, hgks_result* out);
hgks_status hgks_server_wait(hgks_server* srv, int64_t ticket, hgks_result* out);
/* final state [5][n_tets] of a finished request (host memory of the caller) */
hgks_status hgks_server_get_state(hgks_server* srv, int64_t ticket, double* Q);
hgks_status hgks_server_release(hgks_server* srv, int64_t ticket);
hgks_status hgks_server_stats(hgks_server* srv, hgks_server_info* out);
/* waits for active requests, drops queued ones */
void hgks_server_destroy(hgks_server* srv);

#ifdef __cplusplus
}
#endif
#endif
