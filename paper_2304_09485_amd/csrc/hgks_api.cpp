// C ABI of the HGKS library: context, device buffers, residual and FD-Jv
// pipelines, Jacobi preconditioner and the restarted GMRES of Algorithm 1
// (Krylov basis resident in HBM, FP64; small Hessenberg least-squares problem
// on the host as in Sec. 4.3).
#include "hgks.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "hgks_device.h"
#include "hgks_kernels.h"
#include "mesh_prep.h"

using namespace hgks;

namespace {

// Device buffers of a context: from the caller's allocator hook if one is
// given (e.g. PyTorch's caching allocator), else hipMalloc; all released in
// hgks_destroy.
struct DevAlloc {
  std::vector<void*> ptrs;
  hipError_t last = hipSuccess;
  void* (*ualloc)(size_t, void*) = nullptr;
  void (*ufree)(void*, void*) = nullptr;
  void* user = nullptr;
  template <typename T>
  T* get(size_t n) {
    void* p = nullptr;
    if (n == 0) n = 1;
    const size_t bytes = n * sizeof(T);
    if (ualloc) {
      p = ualloc(bytes, user);
      if (p && ((uintptr_t)p & 255u) != 0) {  // kernels assume 256-byte aligned buffers
        ufree(p, user);
        p = nullptr;
      }
      if (!p) {
        last = hipErrorOutOfMemory;
        return nullptr;
      }
    } else {
      hipError_t e = hipMalloc(&p, bytes);
      if (e != hipSuccess) {
        last = e;
        return nullptr;
      }
    }
    ptrs.push_back(p);
    return (T*)p;
  }
  void free_all() {
    for (void* p : ptrs) {
      if (ufree)
        ufree(p, user);
      else
        (void)hipFree(p);
    }
    ptrs.clear();
  }
};

template <typename T>
struct Work {  // per-precision residual work space
  T* Qx = nullptr;    // [5][NX] extended state of the evaluation point
  T* coef = nullptr;  // [105][N]
  T* sv = nullptr;    // [60][2F]
  T* ff = nullptr;    // [5][F]
  T* fq = nullptr;    // [5][F]
  T* dt = nullptr;    // [N]
  T* Gx = nullptr;    // [15][NX] (HWENO gradients, frozen)
};

constexpr int MAXM = 32;
const char* KNAMES[5] = {"ghost", "recon", "side", "flux", "gather"};

}  // namespace

struct hgks_ctx {
  hgks_options o{};
  std::atomic<int64_t> n_steps{0};  // implicit steps taken (read by other threads)
  std::string err;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  HostMesh H;
  bool mesh = false;
  double prim_inf[5] = {1.0, 0.0, 0.0, 0.0, 1.0 / 1.4};
  int kind_of_tag[256];
  bool kinds_dirty = true;
  DevAlloc A;
  DevMesh<double> M{};
  DevMesh<float> Mf{};
  bool have_f32 = false;
  int* d_fkind = nullptr;
  Params P{};
  // state
  double* Qc = nullptr;  // [5][N] master state
  double* Gc = nullptr;  // [15][NX] master gradients (with ghost slots), HWENO
  bool have_state = false;
  Work<double> W64;         // W64.Qx holds the base point Q^n with ghosts
  Work<float> W32;
  double* Qp64 = nullptr;   // [5][NX] perturbed state Q + sigma v of a Jv
  float* Qp32 = nullptr;
  double* dtc = nullptr;    // [N] frozen time step of the current step
  double* b = nullptr;      // [5][N] base residual
  double* Gnew = nullptr;   // [15][N]
  double* lam = nullptr;    // [F]
  double* D = nullptr;      // [N]
  double* V = nullptr;      // [(m+1)][5N]
  double* wv = nullptr, *yv = nullptr, *rv = nullptr, *dQ = nullptr, *t1 = nullptr, *t2 = nullptr;
  double* b32 = nullptr;    // [5][N] inner-precision base residual
  double* part = nullptr;   // reduction partials
  double* sc = nullptr;     // device scalars [64]
  double* gm = nullptr;     // GMRES cycle: H, Givens rotations, g (device)
  int* gst = nullptr;       // GMRES cycle state (device)
  int* flags = nullptr;     // [0] positivity fallbacks, [1] bad state
  std::vector<int> cstart;  // LU-SGS colour classes: offsets into M.cord
  double res0 = -1.0;
  double cfl_now = 10.0;  // CFL of the local time steps (o.cfl, or the ramp of solve_steady)
  bool resumed = false;   // restored from a checkpoint: solve_steady keeps res0 and the CFL ramp
  // timing of the residual kernels: a pool of event sextets recorded on the
  // stream, drained (one synchronisation) when full or when read
  bool prof = false;
  std::vector<hipEvent_t> evpool;
  int evused = 0;
  double ksum[5] = {0, 0, 0, 0, 0};
  int64_t kcount = 0;
};

namespace {
constexpr int EVSETS = 128;

void drain_events(hgks_ctx* ctx) {
  if (!ctx->prof || ctx->evused == 0) return;
  (void)hipEventSynchronize(ctx->evpool[6 * ctx->evused - 1]);
  for (int k = 0; k < ctx->evused; ++k)
    for (int j = 0; j < 5; ++j) {
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, ctx->evpool[6 * k + j], ctx->evpool[6 * k + j + 1]);
      ctx->ksum[j] += ms;
    }
  ctx->kcount += ctx->evused;
  ctx->evused = 0;
}

hipEvent_t* next_events(hgks_ctx* ctx) {
  if (!ctx->prof) return nullptr;
  if (ctx->evused == EVSETS) drain_events(ctx);
  return &ctx->evpool[6 * ctx->evused++];
}
}  // namespace

#define HIPCHK(call)                                                 \
  do {                                                               \
    hipError_t e_ = (call);                                          \
    if (e_ != hipSuccess) {                                          \
      ctx->err = std::string("HIP error: ") + hipGetErrorString(e_); \
      return HGKS_EDEVICE;                                           \
    }                                                                \
  } while (0)

namespace {

void set_params(hgks_ctx* ctx) {
  Params& P = ctx->P;
  const hgks_options& o = ctx->o;
  P.gamma = o.gamma;
  P.K = (5.0 - 3.0 * o.gamma) / (o.gamma - 1.0);
  P.tau_eps = o.tau_eps;
  P.tau_C = o.tau_C;
  P.gamma_lin = o.gamma_lin;
  P.weno_eps = o.weno_eps;
  P.mu = o.mu;
  P.prandtl = o.prandtl;
  P.flux_scale = o.cfl_flux > 0.0 ? o.cfl_flux / ctx->cfl_now : 1.0;
  P.rhoinf = ctx->prim_inf[0];
  P.uinf0 = ctx->prim_inf[1];
  P.uinf1 = ctx->prim_inf[2];
  P.uinf2 = ctx->prim_inf[3];
  P.pinf = ctx->prim_inf[4];
  P.physics = o.physics;
  P.weights = o.weights;
  P.scheme = o.scheme;
  P.csubs = o.scheme == HGKS_HWENO && o.compact_subs == HGKS_SUBS_HEX_WENO ? 1 : 0;
}

template <typename T>
hgks_status upload(hgks_ctx* ctx, const std::vector<T>& h, const T*& dst) {
  T* d = ctx->A.get<T>(h.size());
  if (!d) return HGKS_ENOMEM;
  if (!h.empty()) HIPCHK(hipMemcpy(d, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice));
  dst = d;
  return HGKS_OK;
}

template <typename T>
hgks_status upload_conv(hgks_ctx* ctx, const std::vector<double>& h, const T*& dst) {
  std::vector<T> c(h.begin(), h.end());
  return upload(ctx, c, dst);
}

#define TRY(x)                         \
  do {                                 \
    hgks_status s_ = (x);              \
    if (s_ != HGKS_OK) return s_;      \
  } while (0)

// floating-point mesh arrays in precision T (integer arrays shared)
template <typename T>
hgks_status upload_mesh_fp(hgks_ctx* ctx, DevMesh<T>& M) {
  const HostMesh& H = ctx->H;
  TRY(upload_conv(ctx, H.vol, M.vol));
  TRY(upload_conv(ctx, H.h, M.h));
  TRY(upload_conv(ctx, H.hdt, M.hdt));
  TRY(upload_conv(ctx, H.m2s, M.m2s));
  TRY(upload_conv(ctx, H.fn, M.fn));
  TRY(upload_conv(ctx, H.fS, M.fS));
  TRY(upload_conv(ctx, H.fxiL, M.fxiL));
  TRY(upload_conv(ctx, H.fxiR, M.fxiR));
  if (H.ng == 4) TRY(upload_conv(ctx, H.fw, M.fw));
  if (ctx->o.scheme == HGKS_HWENO) {
    TRY(upload_conv(ctx, H.opH, M.opH));
    if (ctx->P.csubs)
      TRY(upload_conv(ctx, H.opB, M.opB));  // the eight non-compact hexahedral sub-stencils
    else
      TRY(upload_conv(ctx, H.hsub, M.hsub));
  } else if (ctx->o.scheme == HGKS_WENO) {
    TRY(upload_conv(ctx, H.opA, M.opA));
    TRY(upload_conv(ctx, H.opB, M.opB));
  }
  return HGKS_OK;
}

template <typename T>
hgks_status alloc_work(hgks_ctx* ctx, Work<T>& w) {
  const HostMesh& H = ctx->H;
  size_t N = H.N, F = H.F, NX = H.N + H.Nb;
  w.Qx = ctx->A.get<T>(5 * NX);
  // the first-order scheme has no reconstruction coefficients or side values
  const bool ho = ctx->o.scheme != HGKS_KFVS1;
  // 9 + 3 M coefficient vectors per cell (M sub-stencils: 4 on a tetrahedron,
  // 8 non-compact or 6 compact on a hexahedron); 20 values per Gauss point
  const size_t nsub = H.nf == 4 ? 4 : (ctx->o.scheme == HGKS_HWENO && !ctx->P.csubs ? 6 : 8);
  w.coef = ho ? ctx->A.get<T>(5 * (9 + 3 * nsub) * N) : nullptr;
  w.sv = ho ? ctx->A.get<T>((size_t)20 * H.ng * 2 * F) : nullptr;
  w.ff = ctx->A.get<T>(5 * F);
  w.fq = ctx->A.get<T>(5 * F);
  w.dt = ctx->A.get<T>(N);
  w.Gx = ctx->o.scheme == HGKS_HWENO ? ctx->A.get<T>(15 * NX) : nullptr;
  if (!w.Qx || (ho && (!w.coef || !w.sv)) || !w.ff || !w.fq || !w.dt || (ctx->o.scheme == HGKS_HWENO && !w.Gx))
    return HGKS_ENOMEM;
  return HGKS_OK;
}

hgks_status sync_kinds(hgks_ctx* ctx) {
  if (!ctx->kinds_dirty) return HGKS_OK;
  const HostMesh& H = ctx->H;
  std::vector<int> k(H.F);
  for (int f = 0; f < H.F; ++f) k[f] = H.ftag[f] < 0 ? -1 : ctx->kind_of_tag[H.ftag[f]];
  HIPCHK(hipMemcpy(ctx->d_fkind, k.data(), k.size() * sizeof(int), hipMemcpyHostToDevice));
  ctx->kinds_dirty = false;
  set_params(ctx);
  return HGKS_OK;
}

inline size_t n5(const hgks_ctx* ctx) { return (size_t)5 * ctx->H.N; }

// residual pipeline of precision T on an extended state whose cell part is
// filled; mode 0: out = L, 1: Jv epilogue, 2: L and gradient update
template <typename T, typename TO>
void residual_pipeline(hgks_ctx* ctx, const DevMesh<T>& M, Work<T>& w, T* Qx, const T* dt, int mode, TO* out,
                       const TO* v, const TO* bb, const double* sigma, TO* gout, hipStream_t s) {
  const Params& P = ctx->P;
  hipEvent_t* ev = next_events(ctx);
  if (ctx->o.scheme == HGKS_KFVS1) {
    // first order: the flux of the cell averages, no ghost, recon or side
    // stage (the four intervals before the flux stay empty)
    for (int k = 0; k < 4; ++k)
      if (ev) (void)hipEventRecord(ev[k], s);
    launch_flux_kfvs<T>(M, P, Qx, w.ff, s);
    if (ev) (void)hipEventRecord(ev[4], s);
    launch_gather<T, TO>(M, mode, w.ff, w.fq, out, v, bb, dt, sigma, gout, s);
    if (ev) (void)hipEventRecord(ev[5], s);
    return;
  }
  if (ev) (void)hipEventRecord(ev[0], s);
  launch_ghost<T>(M, P, Qx, (T*)nullptr, s);
  if (ev) (void)hipEventRecord(ev[1], s);
  launch_recon<T>(M, P, Qx, w.Gx, w.coef, s);
  if (ev) (void)hipEventRecord(ev[2], s);
  launch_side<T>(M, P, Qx, w.coef, w.sv, ctx->flags, s);
  if (ev) (void)hipEventRecord(ev[3], s);
  launch_flux<T>(M, P, w.sv, dt, w.ff, w.fq, mode == 2, s);
  if (ev) (void)hipEventRecord(ev[4], s);
  launch_gather<T, TO>(M, mode, w.ff, w.fq, out, v, bb, dt, sigma, gout, s);
  if (ev) (void)hipEventRecord(ev[5], s);
}

// state expansion into the FP64 work state and its time step
void expand_state(hgks_ctx* ctx, const double* Q, hipStream_t s) {
  launch_perturb<double>(Q, nullptr, nullptr, ctx->H.N, ctx->H.N + ctx->H.Nb, ctx->W64.Qx, s);
}

hgks_status ensure_f32(hgks_ctx* ctx) {
  if (ctx->have_f32) return HGKS_OK;
  DevMesh<float>& Mf = ctx->Mf;
  const DevMesh<double>& M = ctx->M;
  Mf.N = M.N; Mf.F = M.F; Mf.Nb = M.Nb; Mf.NX = M.NX;
  Mf.nf = M.nf; Mf.ng = M.ng; Mf.nbig = M.nbig;
  Mf.fL = M.fL; Mf.fR = M.fR; Mf.fkind = M.fkind; Mf.cface = M.cface; Mf.gowner = M.gowner; Mf.gface = M.gface;
  Mf.stn = M.stn; Mf.sstn = M.sstn; Mf.smask = M.smask; Mf.nbf = M.nbf;
  Mf.ccol = M.ccol; Mf.cord = M.cord;
  TRY(upload_mesh_fp<float>(ctx, Mf));
  TRY(alloc_work<float>(ctx, ctx->W32));

  ctx->Qp32 = ctx->A.get<float>((size_t)5 * M.NX);
  if (!ctx->Qp32) return HGKS_ENOMEM;
  ctx->have_f32 = true;
  if (ctx->o.scheme == HGKS_HWENO)
    launch_convert(ctx->Gc, ctx->W32.Gx, (size_t)15 * (M.N + M.Nb), ctx->stream);
  return HGKS_OK;
}

// FD Jacobian-vector product at the current state: out = A v (Eq. (frechet)
// with the (|Omega|/dt) term of Eq. (impsystem)); uses ctx->dtc, ctx->b.
// In the FP32-inner form the Arnoldi products run in FP32 (inner = true);
// the restart residual b - A dQ of the outer defect correction stays FP64.
hgks_status jv_device(hgks_ctx* ctx, const double* v, double sigma_fixed, double* out, hipStream_t s,
                      bool inner = true) {
  if (ctx->o.jv_mode == HGKS_JV_APPROX) {
    // the approximate matrix at the base point (W64.Qx = Q^n, lam, D)
    launch_amatvec<double>(ctx->M, ctx->P, ctx->W64.Qx, ctx->lam, ctx->D, v, out, s);
    HIPCHK(hipMemsetAsync(ctx->sc + 2, 0, sizeof(double), s));  // sigma: none
    return HGKS_OK;
  }
  size_t n = n5(ctx);
  const int N = ctx->H.N, NX = ctx->H.N + ctx->H.Nb;
  launch_dot_part(v, v, n, ctx->part, s);  // partials of |v|^2, summed by the sigma kernel
  bool f32 = inner && ctx->o.precision == HGKS_FP32_INNER;
  double eps = f32 ? std::ldexp(1.0, -23) : std::ldexp(1.0, -52);
  if (f32) {
    // the FP32 step (sqrt(2^-23) relative) is large enough that a direction
    // concentrated on a few cells could perturb them out of the physical
    // states: cap it so that no cell's density, momentum (against
    // sqrt(rho E)) or energy moves by more than 1 % (the second half of the
    // partials is free here)
    launch_ratio_part(ctx->Qc, v, N, ctx->part + REDUCE_PARTS, s);
    // and balance the FD truncation against the FP32 rounding (sc[41]: the
    // rounding of the base residual, sc[42]: |A u| / |u| of the previous
    // FP32 product; sc[43] receives |v|)
    launch_sigma(ctx->part, ctx->sc + 0, (double)n, eps, sigma_fixed, ctx->sc + 2, s, ctx->part + REDUCE_PARTS,
                 1e-2, ctx->sc + 41, ctx->sc + 43);
  } else {
    launch_sigma(ctx->part, ctx->sc + 0, (double)n, eps, sigma_fixed, ctx->sc + 2, s);
  }
  if (!f32) {
    launch_perturb<double>(ctx->Qc, v, ctx->sc + 2, N, NX, ctx->Qp64, s);
    residual_pipeline<double, double>(ctx, ctx->M, ctx->W64, ctx->Qp64, ctx->W64.dt, 1, out, v, ctx->b,
                                      ctx->sc + 2, (double*)nullptr, s);
  } else {
    launch_perturb<float>(ctx->Qc, v, ctx->sc + 2, N, NX, ctx->Qp32, s);
    residual_pipeline<float, double>(ctx, ctx->Mf, ctx->W32, ctx->Qp32, ctx->W32.dt, 1, out, v, ctx->b32,
                                     ctx->sc + 2, (double*)nullptr, s);
    launch_norm_ratio(out, n, ctx->sc + 43, ctx->part, ctx->sc + 42, s);
  }
  return HGKS_OK;
}

// Jacobi preconditioner: out = P^{-1} r (uses ctx->lam, ctx->D, W64.Qx = Q^n)
void precond_device(hgks_ctx* ctx, const double* r, double* out, hipStream_t s) {
  int K = std::max(0, ctx->o.jacobi_sweeps);
  if (K == 0) {
    launch_jacobi<double>(ctx->M, ctx->P, ctx->W64.Qx, ctx->lam, ctx->D, r, nullptr, out, s);
    return;
  }
  // x0 = D^{-1} r is formed inside the first sweep; ping-pong between t1/t2
  // so that the last sweep lands in out
  double* bufs[2] = {ctx->t1, ctx->t2};
  double* cur = K == 1 ? out : bufs[1];
  launch_jacobi<double>(ctx->M, ctx->P, ctx->W64.Qx, ctx->lam, ctx->D, r, r, cur, s);
  for (int k = 2; k <= K; ++k) {
    double* nxt = k == K ? out : bufs[k % 2];
    launch_jacobi<double>(ctx->M, ctx->P, ctx->W64.Qx, ctx->lam, ctx->D, r, cur, nxt, s);
    cur = nxt;
  }
}

// prepare the base point of an implicit step / Jv: W64.Qx = Q^n with ghosts,
// dt, b = L(Q^n) (HWENO: Gnew), lam, D; the FP32 copies for the inner form.
hgks_status prepare_base(hgks_ctx* ctx, bool want_grad, hipStream_t s) {
  const int N = ctx->H.N, NX = N + ctx->H.Nb;
  TRY(sync_kinds(ctx));
  HIPCHK(hipMemsetAsync(ctx->flags, 0, 3 * sizeof(int), s));
  expand_state(ctx, ctx->Qc, s);
  launch_ghost<double>(ctx->M, ctx->P, ctx->W64.Qx, (double*)nullptr, s);
  launch_dt<double>(ctx->M, ctx->P, ctx->cfl_now, ctx->W64.Qx, ctx->W64.dt, s);
  residual_pipeline<double, double>(ctx, ctx->M, ctx->W64, ctx->W64.Qx, ctx->W64.dt, want_grad ? 2 : 0, ctx->b,
                                    (const double*)nullptr, (const double*)nullptr, (const double*)nullptr,
                                    want_grad ? ctx->Gnew : (double*)nullptr, s);
  // the pipeline rewrote the ghosts of W64.Qx from Q^n: still the base point
  launch_lambda_diag<double>(ctx->M, ctx->P, ctx->W64.Qx, ctx->W64.dt, ctx->lam, ctx->D, s);
  launch_dot(ctx->Qc, ctx->Qc, n5(ctx), ctx->part, ctx->sc + 0, false, s);
  if (ctx->o.precision == HGKS_FP32_INNER && ctx->o.jv_mode == HGKS_JV_FD && ctx->o.solver == HGKS_SOLVER_GMRES) {
    TRY(ensure_f32(ctx));
    launch_perturb<float>(ctx->Qc, nullptr, nullptr, N, NX, ctx->W32.Qx, s);
    launch_dt<float>(ctx->Mf, ctx->P, ctx->cfl_now, ctx->W32.Qx, ctx->W32.dt, s);
    residual_pipeline<float, double>(ctx, ctx->Mf, ctx->W32, ctx->W32.Qx, ctx->W32.dt, 0, ctx->b32,
                                     (const double*)nullptr, (const double*)nullptr, (const double*)nullptr,
                                     (double*)nullptr, s);
    // rounding level of one FP32 residual evaluation at the base point
    launch_diff_norm(ctx->b32, ctx->b, n5(ctx), ctx->part, ctx->sc + 41, s);
  }
  return HGKS_OK;
}

hgks_status check_state(hgks_ctx* ctx, hipStream_t s) {
  int flags[2];
  launch_check<double>(ctx->W64.Qx, ctx->H.N, ctx->H.N + ctx->H.Nb, ctx->o.gamma, ctx->flags + 1, s);
  HIPCHK(hipMemcpyAsync(flags, ctx->flags, sizeof(flags), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (flags[1]) {
    ctx->err = "non-physical state (rho <= 0, p <= 0 or NaN)";
    return HGKS_ESTATE;
  }
  return HGKS_OK;
}

hgks_status require(hgks_ctx* ctx, bool need_state) {
  if (!ctx) return HGKS_EINVAL;
  if (!ctx->mesh) {
    ctx->err = "no mesh loaded";
    return HGKS_EINVAL;
  }
  if (need_state && !ctx->have_state) {
    ctx->err = "no state set";
    return HGKS_EINVAL;
  }
  return HGKS_OK;
}

hgks_status upload_gradients(hgks_ctx* ctx, const double* G, hipStream_t s) {
  // host [15][N] -> Gc [15][NX] cell slots, then ghost gradients
  const int N = ctx->H.N, NX = N + ctx->H.Nb;
  for (int k = 0; k < 15; ++k) {
    if (G)
      HIPCHK(hipMemcpyAsync(ctx->Gc + (size_t)k * NX, G + (size_t)k * N, (size_t)N * sizeof(double),
                            hipMemcpyHostToDevice, s));
    else
      HIPCHK(hipMemsetAsync(ctx->Gc + (size_t)k * NX, 0, (size_t)N * sizeof(double), s));
  }
  return HGKS_OK;
}

// ghost gradients of Gc and copies into the work spaces
hgks_status refresh_gradients(hgks_ctx* ctx, hipStream_t s) {
  if (ctx->o.scheme != HGKS_HWENO) return HGKS_OK;
  TRY(sync_kinds(ctx));
  const int N = ctx->H.N, NX = N + ctx->H.Nb;
  // the ghost kernel fills the state ghosts too; use a scratch state copy
  expand_state(ctx, ctx->Qc, s);
  launch_ghost<double>(ctx->M, ctx->P, ctx->W64.Qx, ctx->Gc, s);
  HIPCHK(hipMemcpyAsync(ctx->W64.Gx, ctx->Gc, (size_t)15 * NX * sizeof(double), hipMemcpyDeviceToDevice, s));
  // frozen gradients (with ghosts) in the inner precision
  if (ctx->have_f32) launch_convert(ctx->Gc, ctx->W32.Gx, (size_t)15 * NX, s);
  (void)N;
  return HGKS_OK;
}

}  // namespace

// ===========================================================================
extern "C" {

void hgks_default_options(hgks_options* o) {
  std::memset(o, 0, sizeof(*o));
  o->scheme = HGKS_WENO;
  o->physics = HGKS_EULER;
  o->precision = HGKS_FP64;
  o->weights = HGKS_WEIGHTS_NONLINEAR;
  o->krylov_dim = 10;
  o->restarts = 3;
  o->jacobi_sweeps = 2;
  o->gamma = 1.4;
  o->cfl = 10.0;
  o->tau_eps = 0.1;
  o->tau_C = 1.0;
  o->gamma_lin = 0.025;
  o->weno_eps = 1e-5;
  o->mu = 0.0;
  o->prandtl = 1.0;
  o->fd_sigma = 0.0;
  o->cfl_flux = 1.0;
  o->cfl_start = 0.0;
  o->cfl_growth = 1.5;
  o->grad_relax = 1.0;
  o->stream = nullptr;
}

hgks_status hgks_create(const hgks_options* opts, hgks_ctx** out) {
  if (!opts || !out) return HGKS_EINVAL;
  *out = nullptr;
  if (opts->krylov_dim < 1 || opts->krylov_dim > MAXM || opts->restarts < 1 || opts->jacobi_sweeps < 0 ||
      !(opts->gamma > 1.0) || !(opts->cfl > 0.0) || !(opts->max_update >= 0.0) ||
      !(opts->grad_relax > 0.0 && opts->grad_relax <= 1.0) || opts->scheme < 0 || opts->scheme > 2 || opts->physics < 0 ||
      opts->physics > 1 || opts->precision < 0 || opts->precision > 1 || opts->jv_mode < 0 || opts->jv_mode > 1 ||
      opts->solver < HGKS_SOLVER_GMRES || opts->solver > HGKS_SOLVER_LUSGS || opts->compact_subs < 0 ||
      opts->compact_subs > HGKS_SUBS_HEX_WENO ||
      (opts->physics == HGKS_NS && !(opts->mu > 0.0 && opts->prandtl > 0.0)) ||
      (opts->physics == HGKS_NS && opts->scheme == HGKS_KFVS1) || (!opts->dev_alloc != !opts->dev_free))
    return HGKS_EINVAL;
  hgks_ctx* ctx = new (std::nothrow) hgks_ctx;
  if (!ctx) return HGKS_ENOMEM;
  ctx->o = *opts;
  ctx->cfl_now = opts->cfl;
  ctx->A.ualloc = opts->dev_alloc;
  ctx->A.ufree = opts->dev_free;
  ctx->A.user = opts->alloc_user;
  for (int k = 0; k < 256; ++k) ctx->kind_of_tag[k] = HGKS_FARFIELD;
  if (opts->stream) {
    ctx->stream = (hipStream_t)opts->stream;
  } else {
    if (hipStreamCreate(&ctx->stream) != hipSuccess) {
      delete ctx;
      return HGKS_EDEVICE;
    }
    ctx->own_stream = true;
  }
  set_params(ctx);
  *out = ctx;
  return HGKS_OK;
}

// device upload and work allocation of a built host mesh
static hgks_status finish_load(hgks_ctx* ctx);

hgks_status hgks_load_mesh(hgks_ctx* ctx, int64_t n_nodes, const double* xyz, int64_t n_tets,
                           const int32_t* tet2node, int64_t n_bfaces, const int32_t* bface2node,
                           const int32_t* bface_tag) {
  if (!ctx) return HGKS_EINVAL;
  if (ctx->mesh) {
    ctx->err = "mesh already loaded";
    return HGKS_EINVAL;
  }
  if ((n_bfaces > 0 && (!bface2node || !bface_tag)) || n_bfaces < 0) {
    ctx->err = "invalid boundary arrays";
    return HGKS_EINVAL;
  }
  if (ctx->o.scheme == HGKS_HWENO && ctx->o.compact_subs == HGKS_SUBS_HEX_WENO) {
    ctx->err = "compact_subs = HGKS_SUBS_HEX_WENO needs a hexahedral mesh";
    return HGKS_EINVAL;
  }
  int rc = build_host_mesh(ctx->H, n_nodes, xyz, n_tets, tet2node, n_bfaces, bface2node, bface_tag, ctx->err);
  if (rc != 0) return rc == -3 ? HGKS_EMESH : HGKS_EINVAL;
  return finish_load(ctx);
}

hgks_status hgks_load_hex_mesh(hgks_ctx* ctx, int64_t n_nodes, const double* xyz, int64_t n_hex,
                               const int32_t* hex2node, int64_t n_bfaces, const int32_t* bface2node,
                               const int32_t* bface_tag) {
  if (!ctx) return HGKS_EINVAL;
  if (ctx->mesh) {
    ctx->err = "mesh already loaded";
    return HGKS_EINVAL;
  }
  if ((n_bfaces > 0 && (!bface2node || !bface_tag)) || n_bfaces < 0) {
    ctx->err = "invalid boundary arrays";
    return HGKS_EINVAL;
  }
  int rc = build_host_hex_mesh(ctx->H, n_nodes, xyz, n_hex, hex2node, n_bfaces, bface2node, bface_tag, ctx->err);
  if (rc != 0) return rc == -3 ? HGKS_EMESH : HGKS_EINVAL;
  return finish_load(ctx);
}

static hgks_status finish_load(hgks_ctx* ctx) {
  const HostMesh& H = ctx->H;
  DevMesh<double>& M = ctx->M;
  M.N = H.N;
  M.F = H.F;
  M.Nb = H.Nb;
  M.NX = H.N + H.Nb;
  M.nf = H.nf;
  M.ng = H.ng;
  M.nbig = H.nbig;
  TRY(upload(ctx, H.fL, M.fL));
  TRY(upload(ctx, H.fR, M.fR));
  TRY(upload(ctx, H.cface, M.cface));
  TRY(upload(ctx, H.gowner, M.gowner));
  TRY(upload(ctx, H.gface, M.gface));
  // face neighbours: the compact stencil, and the neighbour ids of the
  // Jacobi sweeps for every scheme
  TRY(upload(ctx, H.nbf, M.nbf));
  if (ctx->o.scheme == HGKS_WENO) {
    TRY(upload(ctx, H.stn, M.stn));
    TRY(upload(ctx, H.sstn, M.sstn));
    TRY(upload(ctx, H.smask, M.smask));
  } else if (ctx->P.csubs) {
    TRY(upload(ctx, H.sstn, M.sstn));
    TRY(upload(ctx, H.smask, M.smask));
  }
  if (ctx->o.solver == HGKS_SOLVER_LUSGS) {
    std::vector<int> col, order;
    colour_cells(H, col, order, ctx->cstart);
    TRY(upload(ctx, col, M.ccol));
    TRY(upload(ctx, order, M.cord));
  }
  ctx->d_fkind = ctx->A.get<int>(H.F);
  if (!ctx->d_fkind) return HGKS_ENOMEM;
  M.fkind = ctx->d_fkind;
  TRY(upload_mesh_fp<double>(ctx, M));
  TRY(alloc_work<double>(ctx, ctx->W64));
  size_t N = H.N, NX = H.N + H.Nb, n = 5 * N;
  int m = ctx->o.krylov_dim;
  ctx->Qc = ctx->A.get<double>(n);
  ctx->Qp64 = ctx->A.get<double>(5 * NX);
  ctx->Gc = ctx->o.scheme == HGKS_HWENO ? ctx->A.get<double>(15 * NX) : nullptr;
  ctx->dtc = ctx->A.get<double>(N);
  ctx->b = ctx->A.get<double>(n);
  ctx->b32 = ctx->A.get<double>(n);
  ctx->Gnew = ctx->A.get<double>(15 * N);
  ctx->lam = ctx->A.get<double>(H.F);
  ctx->D = ctx->A.get<double>(N);
  ctx->V = ctx->A.get<double>((size_t)(m + 1) * n);
  ctx->wv = ctx->A.get<double>(n);
  ctx->yv = ctx->A.get<double>(n);
  ctx->rv = ctx->A.get<double>(n);
  ctx->dQ = ctx->A.get<double>(n);
  ctx->t1 = ctx->A.get<double>(n);
  ctx->t2 = ctx->A.get<double>(n);
  ctx->part = ctx->A.get<double>(2 * REDUCE_PARTS);  // two halves: the Gram-Schmidt chain alternates
  ctx->sc = ctx->A.get<double>(64 + MAXM + 1);
  ctx->flags = ctx->A.get<int>(4);
  ctx->gm = ctx->A.get<double>((size_t)(m + 1) * m + 3 * m + 1);
  ctx->gst = ctx->A.get<int>(4);
  if (ctx->sc) {
    // device constant sc[4] = 1 (the unit coefficient of the update axpys),
    // set once so that no host copy sits between queued kernels; the other
    // scalars start at 0 (sc[41..42]: no FP32 rounding estimate yet)
    std::vector<double> init(64 + MAXM + 1, 0.0);
    init[4] = 1.0;
    HIPCHK(hipMemcpy(ctx->sc, init.data(), init.size() * sizeof(double), hipMemcpyHostToDevice));
  }
  if (!ctx->Qc || !ctx->dtc || !ctx->b || !ctx->V || !ctx->flags || !ctx->sc || !ctx->part || !ctx->gm || !ctx->gst) {
    ctx->err = "device allocation failed";
    return HGKS_ENOMEM;
  }
  ctx->mesh = true;
  ctx->kinds_dirty = true;
  return HGKS_OK;
}

hgks_status hgks_set_freestream(hgks_ctx* ctx, const double prim[5]) {
  if (!ctx || !prim) return HGKS_EINVAL;
  if (!(prim[0] > 0.0 && prim[4] > 0.0)) {
    ctx->err = "free stream must have rho > 0 and p > 0";
    return HGKS_EINVAL;
  }
  for (int k = 0; k < 5; ++k) ctx->prim_inf[k] = prim[k];
  set_params(ctx);
  return HGKS_OK;
}

hgks_status hgks_set_bc(hgks_ctx* ctx, int32_t tag, int32_t kind, const double* params) {
  (void)params;
  if (!ctx) return HGKS_EINVAL;
  if (tag < 0 || tag > 255 || kind < HGKS_FARFIELD || kind > HGKS_SUP_OUT) {
    ctx->err = "invalid boundary tag or kind";
    return HGKS_EINVAL;
  }
  ctx->kind_of_tag[tag] = kind;
  ctx->kinds_dirty = true;
  return HGKS_OK;
}

hgks_status hgks_set_state(hgks_ctx* ctx, const double* Q, const double* gradQ) {
  TRY(require(ctx, false));
  if (!Q) return HGKS_EINVAL;
  hipStream_t s = ctx->stream;
  HIPCHK(hipMemcpyAsync(ctx->Qc, Q, n5(ctx) * sizeof(double), hipMemcpyHostToDevice, s));
  if (ctx->o.scheme == HGKS_HWENO) {
    TRY(upload_gradients(ctx, gradQ, s));
    TRY(refresh_gradients(ctx, s));
  }
  ctx->have_state = true;
  ctx->res0 = -1.0;
  ctx->resumed = false;
  HIPCHK(hipStreamSynchronize(s));
  return HGKS_OK;
}

hgks_status hgks_get_state(hgks_ctx* ctx, double* Q, double* gradQ) {
  TRY(require(ctx, true));
  hipStream_t s = ctx->stream;
  if (Q) HIPCHK(hipMemcpyAsync(Q, ctx->Qc, n5(ctx) * sizeof(double), hipMemcpyDeviceToHost, s));
  if (gradQ) {
    const int N = ctx->H.N, NX = N + ctx->H.Nb;
    for (int k = 0; k < 15; ++k) {
      if (ctx->Gc)
        HIPCHK(hipMemcpyAsync(gradQ + (size_t)k * N, ctx->Gc + (size_t)k * NX, (size_t)N * sizeof(double),
                              hipMemcpyDeviceToHost, s));
      else
        std::memset(gradQ + (size_t)k * N, 0, (size_t)N * sizeof(double));
    }
  }
  HIPCHK(hipStreamSynchronize(s));
  return HGKS_OK;
}

hgks_status hgks_residual(hgks_ctx* ctx, const double* Q, const double* gradQ, double* R, double* gradQ_new) {
  TRY(require(ctx, Q == nullptr));
  if (!R) return HGKS_EINVAL;
  hipStream_t s = ctx->stream;
  if (Q) {
    HIPCHK(hipMemcpyAsync(ctx->Qc, Q, n5(ctx) * sizeof(double), hipMemcpyHostToDevice, s));
    ctx->have_state = true;
    ctx->res0 = -1.0;
    if (ctx->o.scheme == HGKS_HWENO) {
      TRY(upload_gradients(ctx, gradQ, s));
      TRY(refresh_gradients(ctx, s));
    }
  } else if (gradQ && ctx->o.scheme == HGKS_HWENO) {
    TRY(upload_gradients(ctx, gradQ, s));
    TRY(refresh_gradients(ctx, s));
  }
  bool want = gradQ_new && ctx->o.scheme == HGKS_HWENO;
  TRY(prepare_base(ctx, want, s));
  HIPCHK(hipMemcpyAsync(R, ctx->b, n5(ctx) * sizeof(double), hipMemcpyDeviceToHost, s));
  if (want) HIPCHK(hipMemcpyAsync(gradQ_new, ctx->Gnew, 15 * (size_t)ctx->H.N * sizeof(double), hipMemcpyDeviceToHost, s));
  else if (gradQ_new) std::memset(gradQ_new, 0, 15 * (size_t)ctx->H.N * sizeof(double));
  return check_state(ctx, s);
}

hgks_status hgks_time_step(hgks_ctx* ctx, const double* Q, double* dt) {
  TRY(require(ctx, Q == nullptr));
  if (!dt) return HGKS_EINVAL;
  hipStream_t s = ctx->stream;
  TRY(sync_kinds(ctx));
  if (Q) {
    HIPCHK(hipMemcpyAsync(ctx->Qc, Q, n5(ctx) * sizeof(double), hipMemcpyHostToDevice, s));
    ctx->have_state = true;
  }
  expand_state(ctx, ctx->Qc, s);
  launch_dt<double>(ctx->M, ctx->P, ctx->cfl_now, ctx->W64.Qx, ctx->W64.dt, s);
  HIPCHK(hipMemcpyAsync(dt, ctx->W64.dt, (size_t)ctx->H.N * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return HGKS_OK;
}

hgks_status hgks_jv(hgks_ctx* ctx, const double* v, double sigma, double* Av, double* sigma_used) {
  TRY(require(ctx, true));
  if (!v || !Av) return HGKS_EINVAL;
  hipStream_t s = ctx->stream;
  TRY(prepare_base(ctx, false, s));
  HIPCHK(hipMemcpyAsync(ctx->yv, v, n5(ctx) * sizeof(double), hipMemcpyHostToDevice, s));
  TRY(jv_device(ctx, ctx->yv, sigma, ctx->wv, s));
  HIPCHK(hipMemcpyAsync(Av, ctx->wv, n5(ctx) * sizeof(double), hipMemcpyDeviceToHost, s));
  double sg = 0.0;
  HIPCHK(hipMemcpyAsync(&sg, ctx->sc + 2, sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  if (sigma_used) *sigma_used = sg;
  return HGKS_OK;
}

hgks_status hgks_precond(hgks_ctx* ctx, const double* r, double* out) {
  TRY(require(ctx, true));
  if (!r || !out) return HGKS_EINVAL;
  hipStream_t s = ctx->stream;
  TRY(prepare_base(ctx, false, s));
  HIPCHK(hipMemcpyAsync(ctx->rv, r, n5(ctx) * sizeof(double), hipMemcpyHostToDevice, s));
  precond_device(ctx, ctx->rv, ctx->wv, s);
  HIPCHK(hipMemcpyAsync(out, ctx->wv, n5(ctx) * sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipStreamSynchronize(s));
  return HGKS_OK;
}

hgks_status hgks_implicit_step(hgks_ctx* ctx, hgks_step_info* info) {
  TRY(require(ctx, true));
  auto t0 = std::chrono::steady_clock::now();
  hipStream_t s = ctx->stream;
  const size_t n = n5(ctx);
  const int N = ctx->H.N;
  const bool hw = ctx->o.scheme == HGKS_HWENO;
  TRY(prepare_base(ctx, hw, s));
  const bool lusgs = ctx->o.solver == HGKS_SOLVER_LUSGS;
  const bool fd = !lusgs && ctx->o.jv_mode == HGKS_JV_FD;
  int64_t evals = (fd && ctx->o.precision == HGKS_FP32_INNER) ? 2 : 1;
  // residual norm of the base point (L1 density residual / total volume)
  launch_abssum(ctx->b, (size_t)N, ctx->part, ctx->sc + 3, s);
  double res_abs = 0.0;
  HIPCHK(hipMemcpyAsync(&res_abs, ctx->sc + 3, sizeof(double), hipMemcpyDeviceToHost, s));
  HIPCHK(hipMemsetAsync(ctx->dQ, 0, n * sizeof(double), s));
  // LU-SGS: one factorised solve of the approximate system, no GMRES cycles
  if (lusgs) {
    launch_lusgs<double>(ctx->M, ctx->P, ctx->W64.Qx, ctx->lam, ctx->D, ctx->cstart, ctx->b, ctx->yv, ctx->dQ, s);
    HIPCHK(hipStreamSynchronize(s));  // res_abs is read below
  }
  const int m = ctx->o.krylov_dim;
  double beta0 = -1.0, last = 0.0;
  bool nonfinite = false;  // a NaN/Inf in the residual or the preconditioned residual
  double* hc = ctx->sc + 8;  // device column of H (m+1 entries)
  double* yd = ctx->sc + 48;  // device solution of the cycle's least-squares problem (m entries)
  double* last_d = ctx->sc + 6;
  // The Arnoldi steps of a restart are queued without host round trips: the
  // Givens rotations run on the device (k_gmres_column), and a finished cycle
  // (happy breakdown, non-finite data) turns the remaining steps into no-ops
  // for the update.  One synchronisation per restart reads beta, the final
  // residual estimate and the cycle state.
  for (int rs = 0; rs < (lusgs ? 0 : ctx->o.restarts); ++rs) {
    if (rs == 0) {
      HIPCHK(hipMemcpyAsync(ctx->rv, ctx->b, n * sizeof(double), hipMemcpyDeviceToDevice, s));
    } else {
      TRY(jv_device(ctx, ctx->dQ, ctx->o.fd_sigma, ctx->yv, s, false));
      if (fd) ++evals;
      // r = b - A dQ (FP64 in both forms: the outer defect correction)
      HIPCHK(hipMemcpyAsync(ctx->rv, ctx->b, n * sizeof(double), hipMemcpyDeviceToDevice, s));
      launch_axpy_dev(ctx->yv, ctx->rv, n, ctx->sc + 4, -1.0, s);  // sc[4] = 1
    }
    precond_device(ctx, ctx->rv, ctx->wv, s);
    launch_dot(ctx->wv, ctx->wv, n, ctx->part, ctx->sc + 5, true, s);  // beta
    launch_gmres_start(ctx->sc + 5, ctx->gm, ctx->gst, m, s);
    launch_scale_inv(ctx->wv, ctx->V, n, ctx->sc + 5, s, ctx->gst);
    for (int j = 0; j < m; ++j) {
      double* vj = ctx->V + (size_t)j * n;
      TRY(jv_device(ctx, vj, ctx->o.fd_sigma, ctx->yv, s));
      if (fd) ++evals;
      precond_device(ctx, ctx->yv, ctx->wv, s);
      // modified Gram-Schmidt: partials of h_0 = (w, v_0); then per i one
      // pass that sums the partials of h_i (stored in hc[i]), forms
      // w -= h_i v_i and the partials of h_{i+1} = (w, v_{i+1}), the last
      // pass those of |w|^2; the two halves of part alternate
      launch_dot_part(ctx->wv, ctx->V, n, ctx->part, s);
      for (int i = 0; i <= j; ++i) {
        const double* vi = ctx->V + (size_t)i * n;
        const double* next = i < j ? ctx->V + (size_t)(i + 1) * n : nullptr;
        launch_axpy_dot_chain(ctx->part + (i & 1) * REDUCE_PARTS, hc + i, vi, ctx->wv, n, next,
                              ctx->part + ((i + 1) & 1) * REDUCE_PARTS, s);
      }
      launch_reduce_final(ctx->part + ((j + 1) & 1) * REDUCE_PARTS, hc + j + 1, true, s);
      launch_gmres_column(j, m, hc, ctx->gm, ctx->gst, s);
      if (j + 1 < m) launch_scale_inv(ctx->wv, ctx->V + (size_t)(j + 1) * n, n, hc + j + 1, s, ctx->gst);
    }
    launch_gmres_solve(m, ctx->gm, ctx->gst, yd, last_d, s);
    launch_combine(ctx->V, yd, m, n, ctx->dQ, ctx->dQ, s);
    double sc_h[2];
    int st_h[3];
    HIPCHK(hipMemcpyAsync(sc_h, ctx->sc + 5, 2 * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipMemcpyAsync(st_h, ctx->gst, sizeof(st_h), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    const double beta = sc_h[0];
    if (beta0 < 0) beta0 = beta;
    if (st_h[1]) {
      nonfinite = true;  // an FD product or the residual produced NaN/Inf: no update from this cycle
      break;
    }
    if (!(beta > 0.0)) break;
    last = sc_h[1];
  }
  // res_abs was read back before the first restart's synchronisation
  if (nonfinite || !std::isfinite(res_abs)) {
    if (info) {
      info->res = res_abs / ctx->H.total_volume;
      info->n_resid_evals = evals;
    }
    ctx->err = "non-finite residual (NaN or Inf in L(Q^n) or its GMRES solve); the state was not updated";
    return HGKS_ESTATE;
  }
  // Q^{n+1} = Q^n + dQ, with the optional per-cell update limit
  if (ctx->o.max_update > 0.0)
    launch_update_limited(ctx->Qc, ctx->dQ, N, ctx->o.max_update, ctx->o.gamma, ctx->flags + 2, s);
  else
    launch_axpy_dev(ctx->dQ, ctx->Qc, n, ctx->sc + 4, 1.0, s);  // sc[4] = 1
  if (hw) {
    const int NX = N + ctx->H.Nb;
    if (ctx->o.grad_relax < 1.0) {
      launch_relax_grad(ctx->Gc, ctx->Gnew, N, NX, ctx->o.grad_relax, s);  // G += omega (G_new - G)
    } else {
      for (int k = 0; k < 15; ++k)
        HIPCHK(hipMemcpyAsync(ctx->Gc + (size_t)k * NX, ctx->Gnew + (size_t)k * N, (size_t)N * sizeof(double),
                              hipMemcpyDeviceToDevice, s));
    }
    TRY(refresh_gradients(ctx, s));
  }
  int flags[3] = {0, 0, 0};
  HIPCHK(hipMemcpyAsync(flags, ctx->flags, sizeof(flags), hipMemcpyDeviceToHost, s));
  expand_state(ctx, ctx->Qc, s);
  HIPCHK(hipStreamSynchronize(s));
  double res = res_abs / ctx->H.total_volume;
  if (ctx->res0 < 0) ctx->res0 = res;
  if (info) {
    info->res = res;
    info->res_rel = ctx->res0 > 0 ? res / ctx->res0 : 0.0;
    info->gmres_rel = beta0 > 0 ? last / beta0 : 0.0;
    info->n_resid_evals = evals;
    info->n_fallbacks = flags[0];
    info->n_limited = flags[2];
    info->t_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  ctx->n_steps.fetch_add(1, std::memory_order_relaxed);
  return check_state(ctx, s);
}

hgks_status hgks_solve_steady(hgks_ctx* ctx, double drop, int32_t max_steps, hgks_solve_info* info) {
  TRY(require(ctx, true));
  auto t0 = std::chrono::steady_clock::now();
  hgks_solve_info si{};
  hgks_status st = HGKS_OK;
  // optional CFL ramp from an impulsive start; a solve resumed from a
  // checkpoint continues the ramp where it stood and measures the drop
  // against the reference residual of the interrupted solve
  const bool ramp = ctx->o.cfl_start > 0.0 && ctx->o.cfl_start < ctx->o.cfl;
  if (!ctx->resumed) {
    ctx->res0 = -1.0;
    ctx->cfl_now = ramp ? ctx->o.cfl_start : ctx->o.cfl;
  }
  ctx->resumed = false;
  set_params(ctx);
  for (int k = 0; k < max_steps; ++k) {
    hgks_step_info s{};
    st = hgks_implicit_step(ctx, &s);
    if (ramp && ctx->cfl_now < ctx->o.cfl) {
      ctx->cfl_now = std::min(ctx->o.cfl, ctx->cfl_now * std::max(1.0, ctx->o.cfl_growth));
      set_params(ctx);
    }
    si.steps = k + 1;
    si.n_resid_evals += s.n_resid_evals;
    if (k == 0) si.res0 = ctx->res0 > 0 ? ctx->res0 : s.res;
    si.res_final = s.res;
    if (st != HGKS_OK) break;
    if (s.res_rel <= drop) {
      si.converged = 1;
      break;
    }
  }
  si.drop = si.res0 > 0 ? si.res_final / si.res0 : 0.0;
  si.t_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (info) *info = si;
  if (st != HGKS_OK) return st;
  if (!si.converged) {
    ctx->err = "requested residual drop not reached";
    return HGKS_ENOCONV;
  }
  return HGKS_OK;
}

namespace {

// Checkpoint file: a fixed header, the state [5][N], the gradients [15][N]
// (compact scheme only), then an FNV-1a 64-bit hash of everything before it.
struct CkptHeader {
  char magic[8];     // "HGKSCKP1"
  int32_t version;   // 2
  int32_t scheme;    // HGKS_WENO | HGKS_HWENO
  int64_t n_cells;
  int64_t n_bfaces;
  double res0;       // residual the relative residual is measured against (< 0: none yet)
  double gamma;
  double cfl_now;    // CFL number the next step runs at (the solve_steady ramp)
};
constexpr int32_t CKPT_VERSION = 2;

uint64_t fnv1a(uint64_t h, const void* p, size_t n) {
  const unsigned char* b = (const unsigned char*)p;
  for (size_t k = 0; k < n; ++k) {
    h ^= b[k];
    h *= 1099511628211ull;
  }
  return h;
}

constexpr uint64_t FNV_OFFSET = 14695981039346656037ull;

}  // namespace

hgks_status hgks_checkpoint(hgks_ctx* ctx, const char* path) {
  TRY(require(ctx, true));
  if (!path) return HGKS_EINVAL;
  const int64_t N = ctx->H.N;
  const bool hw = ctx->o.scheme == HGKS_HWENO;
  std::vector<double> Q((size_t)5 * N), G(hw ? (size_t)15 * N : 0);
  TRY(hgks_get_state(ctx, Q.data(), hw ? G.data() : nullptr));
  CkptHeader h{};
  std::memcpy(h.magic, "HGKSCKP1", 8);
  h.version = CKPT_VERSION;
  h.scheme = ctx->o.scheme;
  h.n_cells = N;
  h.n_bfaces = ctx->H.Nb;
  h.res0 = ctx->res0;
  h.gamma = ctx->o.gamma;
  h.cfl_now = ctx->cfl_now;
  uint64_t hash = fnv1a(FNV_OFFSET, &h, sizeof(h));
  hash = fnv1a(hash, Q.data(), Q.size() * sizeof(double));
  if (hw) hash = fnv1a(hash, G.data(), G.size() * sizeof(double));
  // write to a temporary name and rename, so a crash never leaves a torn file
  std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "wb");
  if (!f) {
    ctx->err = "cannot open checkpoint file for writing";
    return HGKS_EINVAL;
  }
  bool ok = std::fwrite(&h, sizeof(h), 1, f) == 1 && std::fwrite(Q.data(), sizeof(double), Q.size(), f) == Q.size() &&
            (!hw || std::fwrite(G.data(), sizeof(double), G.size(), f) == G.size()) &&
            std::fwrite(&hash, sizeof(hash), 1, f) == 1;
  ok = (std::fclose(f) == 0) && ok;
  if (!ok || std::rename(tmp.c_str(), path) != 0) {
    std::remove(tmp.c_str());
    ctx->err = "writing the checkpoint file failed";
    return HGKS_EINVAL;
  }
  return HGKS_OK;
}

hgks_status hgks_restore(hgks_ctx* ctx, const char* path) {
  TRY(require(ctx, false));
  if (!path) return HGKS_EINVAL;
  FILE* f = std::fopen(path, "rb");
  if (!f) {
    ctx->err = "cannot open checkpoint file";
    return HGKS_EINVAL;
  }
  auto fail = [&](const char* msg) {
    std::fclose(f);
    ctx->err = msg;
    return HGKS_EINVAL;
  };
  CkptHeader h{};
  if (std::fread(&h, sizeof(h), 1, f) != 1 || std::memcmp(h.magic, "HGKSCKP1", 8) != 0 || h.version != CKPT_VERSION)
    return fail("not an HGKS checkpoint file (bad magic or version)");
  const int64_t N = ctx->H.N;
  if (h.n_cells != N || h.n_bfaces != ctx->H.Nb) return fail("checkpoint was written for a different mesh");
  if (h.scheme != ctx->o.scheme) return fail("checkpoint was written for a different reconstruction scheme");
  const bool hw = h.scheme == HGKS_HWENO;
  std::vector<double> Q((size_t)5 * N), G(hw ? (size_t)15 * N : 0);
  uint64_t stored = 0;
  if (std::fread(Q.data(), sizeof(double), Q.size(), f) != Q.size() ||
      (hw && std::fread(G.data(), sizeof(double), G.size(), f) != G.size()) ||
      std::fread(&stored, sizeof(stored), 1, f) != 1)
    return fail("checkpoint file is truncated");
  char extra;
  if (std::fread(&extra, 1, 1, f) != 0) return fail("checkpoint file has trailing bytes");
  std::fclose(f);
  uint64_t hash = fnv1a(FNV_OFFSET, &h, sizeof(h));
  hash = fnv1a(hash, Q.data(), Q.size() * sizeof(double));
  if (hw) hash = fnv1a(hash, G.data(), G.size() * sizeof(double));
  if (hash != stored) {
    ctx->err = "checkpoint file is corrupt (hash mismatch)";
    return HGKS_EINVAL;
  }
  if (!(h.cfl_now > 0.0)) {
    ctx->err = "checkpoint holds no valid CFL number";
    return HGKS_EINVAL;
  }
  TRY(hgks_set_state(ctx, Q.data(), hw ? G.data() : nullptr));
  ctx->res0 = h.res0;
  ctx->cfl_now = h.cfl_now;
  ctx->resumed = true;
  set_params(ctx);
  return HGKS_OK;
}

hgks_status hgks_residual_dev(hgks_ctx* ctx, const void* Q_dev, void* R_dev, void* stream) {
  TRY(require(ctx, false));
  if (!Q_dev || !R_dev) return HGKS_EINVAL;
  hipStream_t s = stream ? (hipStream_t)stream : ctx->stream;
  TRY(sync_kinds(ctx));
  expand_state(ctx, (const double*)Q_dev, s);
  launch_ghost<double>(ctx->M, ctx->P, ctx->W64.Qx, (double*)nullptr, s);
  launch_dt<double>(ctx->M, ctx->P, ctx->cfl_now, ctx->W64.Qx, ctx->W64.dt, s);
  residual_pipeline<double, double>(ctx, ctx->M, ctx->W64, ctx->W64.Qx, ctx->W64.dt, 0, (double*)R_dev,
                                    (const double*)nullptr, (const double*)nullptr, (const double*)nullptr,
                                    (double*)nullptr, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    ctx->err = hipGetErrorString(e);
    return HGKS_EDEVICE;
  }
  return HGKS_OK;
}

// Bytes of the residual work space of a mesh (extended state, time steps,
// reconstruction coefficients, side values, face fluxes and face point
// values), each part starting on a 256-byte boundary; offsets in off[6].
static size_t residual_work_layout(const hgks_ctx* ctx, size_t off[6]) {
  const HostMesh& H = ctx->H;
  const size_t N = H.N, F = H.F, NX = H.N + H.Nb;
  const bool ho = ctx->o.scheme != HGKS_KFVS1;
  const size_t nsub = H.nf == 4 ? 4 : (ctx->o.scheme == HGKS_HWENO && !ctx->P.csubs ? 6 : 8);
  const size_t len[6] = {5 * NX, N, ho ? 5 * (9 + 3 * nsub) * N : 0, ho ? (size_t)20 * H.ng * 2 * F : 0, 5 * F, 5 * F};
  size_t at = 0;
  for (int k = 0; k < 6; ++k) {
    off[k] = at;
    at += (len[k] * sizeof(double) + 255) / 256 * 256;
  }
  return at;
}

hgks_status hgks_residual_dev_static(hgks_ctx* ctx, const void* Q_dev, void* R_dev, void* stream) {
  TRY(require(ctx, false));
  if (!Q_dev || !R_dev) return HGKS_EINVAL;
  size_t off[6];
  const size_t need = residual_work_layout(ctx, off);
  if (need > STATIC_SCRATCH_BYTES) {
    ctx->err = "mesh needs " + std::to_string(need) + " bytes of residual work space, more than the " +
               std::to_string(STATIC_SCRATCH_BYTES) + " bytes of the static device buffer";
    return HGKS_EINVAL;
  }
  void* base = nullptr;
  HIPCHK(static_scratch_ptr(&base));
  hipStream_t s = stream ? (hipStream_t)stream : ctx->stream;
  TRY(sync_kinds(ctx));
  // every part of the work space is written before it is read: nothing to clear
  unsigned char* b = (unsigned char*)base;
  const bool ho = ctx->o.scheme != HGKS_KFVS1;
  Work<double> w;
  w.Qx = (double*)(b + off[0]);
  w.dt = (double*)(b + off[1]);
  w.coef = ho ? (double*)(b + off[2]) : nullptr;
  w.sv = ho ? (double*)(b + off[3]) : nullptr;
  w.ff = (double*)(b + off[4]);
  w.fq = (double*)(b + off[5]);
  w.Gx = ctx->W64.Gx;  // the context's frozen gradients (compact scheme), read only
  launch_perturb<double>((const double*)Q_dev, nullptr, nullptr, ctx->H.N, ctx->H.N + ctx->H.Nb, w.Qx, s);
  launch_ghost<double>(ctx->M, ctx->P, w.Qx, (double*)nullptr, s);
  launch_dt<double>(ctx->M, ctx->P, ctx->cfl_now, w.Qx, w.dt, s);
  residual_pipeline<double, double>(ctx, ctx->M, w, w.Qx, w.dt, 0, (double*)R_dev, (const double*)nullptr,
                                    (const double*)nullptr, (const double*)nullptr, (double*)nullptr, s);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    ctx->err = hipGetErrorString(e);
    return HGKS_EDEVICE;
  }
  return HGKS_OK;
}

size_t hgks_residual_static_bytes(const hgks_ctx* ctx) {
  if (!ctx || !ctx->mesh) return 0;
  size_t off[6];
  return residual_work_layout(ctx, off);
}

hgks_status hgks_jv_dev(hgks_ctx* ctx, const void* v_dev, double sigma, void* Av_dev, void* stream) {
  TRY(require(ctx, true));
  if (!v_dev || !Av_dev) return HGKS_EINVAL;
  hipStream_t s = stream ? (hipStream_t)stream : ctx->stream;
  TRY(prepare_base(ctx, false, s));
  TRY(jv_device(ctx, (const double*)v_dev, sigma, (double*)Av_dev, s));
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) {
    ctx->err = hipGetErrorString(e);
    return HGKS_EDEVICE;
  }
  return HGKS_OK;
}

int64_t hgks_n_cells(const hgks_ctx* ctx) { return ctx && ctx->mesh ? ctx->H.N : 0; }
int64_t hgks_steps_done(const hgks_ctx* ctx) { return ctx ? ctx->n_steps.load(std::memory_order_relaxed) : 0; }
int64_t hgks_n_faces(const hgks_ctx* ctx) { return ctx && ctx->mesh ? ctx->H.F : 0; }

hgks_status hgks_kernel_times(hgks_ctx* ctx, const char** names, double* ms, int32_t* n, int32_t cap) {
  if (!ctx || !n) return HGKS_EINVAL;
  if (!ctx->prof) {
    ctx->evpool.resize(6 * EVSETS);
    for (auto& e : ctx->evpool)
      if (hipEventCreate(&e) != hipSuccess) return HGKS_EDEVICE;
    ctx->prof = true;  // timing starts with the next evaluation
  }
  drain_events(ctx);
  int c = std::min(cap, 6);
  for (int k = 0; k < c; ++k) {
    if (names) names[k] = k < 5 ? KNAMES[k] : "evaluations";
    if (ms) ms[k] = k < 5 ? (ctx->kcount ? ctx->ksum[k] / ctx->kcount : 0.0) : (double)ctx->kcount;
  }
  *n = c;
  for (int k = 0; k < 5; ++k) ctx->ksum[k] = 0.0;
  ctx->kcount = 0;
  return HGKS_OK;
}

const char* hgks_last_error(const hgks_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

void hgks_destroy(hgks_ctx* ctx) {
  if (!ctx) return;
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  ctx->A.free_all();
  for (auto& e : ctx->evpool) (void)hipEventDestroy(e);
  if (ctx->own_stream) (void)hipStreamDestroy(ctx->stream);
  delete ctx;
}

}  // extern "C"
