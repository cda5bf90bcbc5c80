// Host-side launchers of the HGKS kernels (defined in hgks_kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <vector>

#include "hgks_device.h"

namespace hgks {

template <typename T> void launch_ghost(const DevMesh<T>&, const Params&, T* Qx, T* Gx, hipStream_t);
template <typename T>
void launch_recon(const DevMesh<T>&, const Params&, const T* Qx, const T* Gx, T* coef, hipStream_t);
template <typename T>
void launch_side(const DevMesh<T>&, const Params&, const T* Qx, const T* coef, T* sv, int* nfall, hipStream_t);
template <typename T>
void launch_flux(const DevMesh<T>&, const Params&, const T* sv, const T* dt, T* ff, T* fq, bool qg, hipStream_t);
template <typename T>
void launch_flux_kfvs(const DevMesh<T>&, const Params&, const T* Qx, T* ff, hipStream_t);
template <typename T, typename TO>
void launch_gather(const DevMesh<T>&, int mode, const T* ff, const T* fq, TO* out, const TO* v, const TO* b,
                   const T* dt, const double* sigma, TO* gout, hipStream_t);
template <typename T> void launch_dt(const DevMesh<T>&, const Params&, double cfl, const T* Qx, T* dt, hipStream_t);
template <typename T>
void launch_lambda_diag(const DevMesh<T>&, const Params&, const T* Qx, const T* dt, T* lam, T* D, hipStream_t);
// xo == nullptr: xn = D^{-1} r; xo == r: one sweep from x0 = D^{-1} r (the first
// two sweeps fused); otherwise one sweep from xo
template <typename T>
void launch_jacobi(const DevMesh<T>&, const Params&, const T* Qx, const T* lam, const T* D, const double* r,
                   const double* xo, double* xn, hipStream_t);
template <typename T>
void launch_amatvec(const DevMesh<T>&, const Params&, const T* Qx, const T* lam, const T* D, const double* x,
                    double* out, hipStream_t);
// LU-SGS: forward sweep over the colour classes start[c]..start[c+1] of
// M.cord ((D + L) y = r), then backward (D + U) x = D y
template <typename T>
void launch_lusgs(const DevMesh<T>&, const Params&, const T* Qx, const T* lam, const T* D,
                  const std::vector<int>& start, const double* r, double* y, double* x, hipStream_t);
template <typename T>
void launch_perturb(const double* Q, const double* v, const double* sigma, int N, int NX, T* Qp, hipStream_t);
template <typename T> void launch_check(const T* Qx, int N, int NX, double gamma, int* bad, hipStream_t);

void launch_dot(const double* x, const double* y, size_t n, double* part, double* out, bool sqrt_out, hipStream_t);
void launch_abssum(const double* x, size_t n, double* part, double* out, hipStream_t);
// block partials of x.y into part[REDUCE_PARTS]; their fixed-order sum
// (sqrt of it if sq) into out[0]
void launch_dot_part(const double* x, const double* y, size_t n, double* part, hipStream_t);
void launch_reduce_final(const double* part, double* out, bool sq, hipStream_t);
// h = the fixed-order sum of pin (stored in hout[0]); w -= h v; pout = block
// partials of w.z, or of w.w if z is null (pin and pout distinct)
void launch_axpy_dot_chain(const double* pin, double* hout, const double* v, double* w, size_t n, const double* z,
                           double* pout, hipStream_t);
void launch_axpy_dev(const double* x, double* y, size_t n, const double* a, double sgn, hipStream_t);
void launch_scale_inv(const double* x, double* y, size_t n, const double* a, hipStream_t, const int* skip = nullptr);
// Q += alpha_i dQ with the per-cell update limit th (counted in nlim[0])
void launch_update_limited(double* Q, const double* dQ, int N, double th, double gamma, int* nlim, hipStream_t);
// GMRES cycle bookkeeping on the device: G [(m+1) m + 2 m + m + 1] holds H,
// the Givens rotations and g; st [3]: finished, non-finite, columns done
void launch_gmres_start(const double* beta, double* G, int* st, int m, hipStream_t);
void launch_gmres_column(int j, int m, const double* hc, double* G, int* st, hipStream_t);
void launch_gmres_solve(int m, const double* G, const int* st, double* y, double* out, hipStream_t);
void launch_combine(const double* V, const double* c, int nv, size_t n, const double* x, double* y, hipStream_t);
void launch_convert(const double* src, float* dst, size_t n, hipStream_t);
// FD step of the Jv product from the block partials of |v|^2 (vpart) and the
// reduced |Q|^2 (qq[0]) into sigma[0]; with rpart (block maxima of
// launch_ratio_part) the step is also capped at eta / max ratio
// vnorm (if set) receives |v|; noise (if set) = {rounding of one inner-precision
// residual evaluation, |A u| / |u| of the last inner product} caps the step
// where it balances rounding against truncation
void launch_sigma(const double* vpart, const double* qq, double n, double eps, double fixed, double* sigma,
                  hipStream_t, const double* rpart = nullptr, double eta = 0.0, const double* noise = nullptr,
                  double* vnorm = nullptr);
// out[0] = |x - y| (fixed-order sum)
void launch_diff_norm(const double* x, const double* y, size_t n, double* part, double* out, hipStream_t);
// out[0] = |x| / den[0] (0 if den[0] is 0)
void launch_norm_ratio(const double* x, size_t n, const double* den, double* part, double* out, hipStream_t);
// G[k][i] += w (Gnew[k][i] - G[k][i]) for the 15 gradient rows (G: leading dimension NX, Gnew: N)
void launch_relax_grad(double* G, const double* Gnew, int N, int NX, double w, hipStream_t);
// block maxima of max(|v_rho| / rho, |v_m| / sqrt(rho E), |v_E| / E) over the cells into part[REDUCE_PARTS]
void launch_ratio_part(const double* Q, const double* v, int N, double* part, hipStream_t);

constexpr int REDUCE_PARTS = 1024;  // partials of a reduction

// Device work space of the allocation-free residual (64 MiB per GPU); its
// device address on the current device (looked up on first use per device)
constexpr size_t STATIC_SCRATCH_BYTES = size_t(64) << 20;
constexpr int MAX_DEVICES = 64;
hipError_t static_scratch_ptr(void** out);

}  // namespace hgks
