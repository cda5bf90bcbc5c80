// Host instantiation of the device flux function, for CPU tests only.
//
// gks_flux.h is written as __host__ __device__ templates; this file builds the
// double and float instantiations into a small test library
// (libhgks_hostcheck.so) so the tests can compare the exact arithmetic of the
// GPU flux with the oracle on the CPU.  The product library does not contain
// or call it.
#include <cstdint>

#include "gks_flux.h"

extern "C" {

void hgks_hostcheck_flux(const double* Wl, const double* dWl, const double* Wr, const double* dWr, double dt,
                         const double* params /* gamma, K, tau_eps, tau_C, mu, prandtl */, int32_t physics,
                         int32_t want_qg, double* F, double* QG) {
  hgks::FluxParams<double> P;
  P.gamma = params[0];
  P.K = params[1];
  P.tau_eps = params[2];
  P.tau_C = params[3];
  P.mu = params[4];
  P.prandtl = params[5];
  P.physics = physics;
  double l[5], r[5], dl[3][5], dr[3][5], q[5];
  for (int k = 0; k < 5; ++k) {
    l[k] = Wl[k];
    r[k] = Wr[k];
    for (int d = 0; d < 3; ++d) {
      dl[d][k] = dWl[d * 5 + k];
      dr[d][k] = dWr[d * 5 + k];
    }
  }
  if (want_qg)
    hgks::gks_flux<double, true>(l, dl, r, dr, dt, P, F, q);
  else
    hgks::gks_flux<double, false>(l, dl, r, dr, dt, P, F, q);
  if (QG)
    for (int k = 0; k < 5; ++k) QG[k] = want_qg ? q[k] : 0.0;
}

void hgks_hostcheck_flux_f32(const double* Wl, const double* dWl, const double* Wr, const double* dWr, double dt,
                             const double* params, int32_t physics, double* F) {
  hgks::FluxParams<float> P;
  P.gamma = (float)params[0];
  P.K = (float)params[1];
  P.tau_eps = (float)params[2];
  P.tau_C = (float)params[3];
  P.mu = (float)params[4];
  P.prandtl = (float)params[5];
  P.physics = physics;
  float l[5], r[5], dl[3][5], dr[3][5], f[5], q[5];
  for (int k = 0; k < 5; ++k) {
    l[k] = (float)Wl[k];
    r[k] = (float)Wr[k];
    for (int d = 0; d < 3; ++d) {
      dl[d][k] = (float)dWl[d * 5 + k];
      dr[d][k] = (float)dWr[d * 5 + k];
    }
  }
  hgks::gks_flux<float, false>(l, dl, r, dr, (float)dt, P, f, q);
  for (int k = 0; k < 5; ++k) F[k] = f[k];
}

void hgks_hostcheck_kfvs(const double* Wl, const double* Wr, double gamma, double K, double* F) {
  double l[5], r[5];
  for (int k = 0; k < 5; ++k) {
    l[k] = Wl[k];
    r[k] = Wr[k];
  }
  hgks::kfvs_flux(l, r, gamma, K, F);
}

void hgks_hostcheck_slope(const double* b, double U, double V, double W, double lam, double K, double* a) {
  double bb[5] = {b[0], b[1], b[2], b[3], b[4]};
  hgks::micro_slope(bb, U, V, W, lam, 0.5 / lam, K, 1.0 / (K + 3.0), a);
}
}
