// Gas-kinetic (BGK) flux at one Gauss point in the local face frame
// (paper Sec. 2 Eq. (flux) and the moment systems below it; time average of
// Sec. 4.1; collision time of Sec. 5; Prandtl correction of the heat flux).
//
// Velocity moments of a Maxwellian are tabulated per side once; every moment
// the flux needs is then a compile-time indexed product, so the compiler emits
// straight-line VALU code.  T is double (plain path) or float (inner path of
// the mixed-precision form).
#pragma once
#include <hip/hip_runtime.h>

namespace hgks {

template <typename T>
struct Mxw {
  T u[8];  // <u^k>, half or full space
  T v[6];  // <v^k>
  T w[6];  // <w^k>
  T x2, x4;  // <xi^2>, <xi^4>
};

template <typename T>
__host__ __device__ __forceinline__ void mxw_vw(Mxw<T>& M, T V, T W, T lam, T K) {
  T r = T(0.5) / lam;
  M.v[0] = T(1); M.v[1] = V;
  M.w[0] = T(1); M.w[1] = W;
#pragma unroll
  for (int k = 2; k < 6; ++k) {
    M.v[k] = V * M.v[k - 1] + T(k - 1) * r * M.v[k - 2];
    M.w[k] = W * M.w[k - 1] + T(k - 1) * r * M.w[k - 2];
  }
  M.x2 = K * r;
  M.x4 = K * (K + T(2)) * r * r;
}

// u-moments; sgn = 0 full space, +1 half space u > 0, -1 half space u < 0
template <typename T>
__host__ __device__ __forceinline__ void mxw_u(Mxw<T>& M, T U, T lam, int sgn) {
  T r = T(0.5) / lam;
  if (sgn == 0) {
    M.u[0] = T(1);
    M.u[1] = U;
  } else {
    T sl = sqrt(lam);
    T e = exp(-lam * U * U) / sqrt(T(M_PI) * lam);
    if (sgn > 0) {
      M.u[0] = T(0.5) * erfc(-sl * U);
      M.u[1] = U * M.u[0] + T(0.5) * e;
    } else {
      M.u[0] = T(0.5) * erfc(sl * U);
      M.u[1] = U * M.u[0] - T(0.5) * e;
    }
  }
#pragma unroll
  for (int k = 2; k < 8; ++k) M.u[k] = U * M.u[k - 1] + T(k - 1) * r * M.u[k - 2];
}

template <int a, int b, int c, int d, typename T>
__host__ __device__ __forceinline__ T mm(const Mxw<T>& M) {
  T x = M.u[a] * M.v[b] * M.w[c];
  if (d == 1) x *= M.x2;
  if (d == 2) x *= M.x4;
  return x;
}

// out += s <u^a v^b w^c xi^(2d) psi>
template <int a, int b, int c, int d, typename T>
__host__ __device__ __forceinline__ void psi5(const Mxw<T>& M, T s, T out[5]) {
  out[0] += s * mm<a, b, c, d>(M);
  out[1] += s * mm<a + 1, b, c, d>(M);
  out[2] += s * mm<a, b + 1, c, d>(M);
  out[3] += s * mm<a, b, c + 1, d>(M);
  out[4] += s * T(0.5) * (mm<a + 2, b, c, d>(M) + mm<a, b + 2, c, d>(M) + mm<a, b, c + 2, d>(M) +
                          mm<a, b, c, d + 1>(M));
}

// out += s <(co . psi) u^a v^b w^c psi>
template <int a, int b, int c, typename T>
__host__ __device__ __forceinline__ void apsi(const Mxw<T>& M, const T co[5], T s, T out[5]) {
  psi5<a, b, c, 0>(M, s * co[0], out);
  psi5<a + 1, b, c, 0>(M, s * co[1], out);
  psi5<a, b + 1, c, 0>(M, s * co[2], out);
  psi5<a, b, c + 1, 0>(M, s * co[3], out);
  T hh = T(0.5) * s * co[4];
  psi5<a + 2, b, c, 0>(M, hh, out);
  psi5<a, b + 2, c, 0>(M, hh, out);
  psi5<a, b, c + 2, 0>(M, hh, out);
  psi5<a, b, c, 1>(M, hh, out);
}

// Closed-form solution of <a psi> = b (normalised moments of the full-space
// Maxwellian with velocity (U,V,W), lam = rho/(2p), K internal dof): solved
// in the peculiar-velocity basis where the moment matrix is block diagonal.
template <typename T>
__host__ __device__ __forceinline__ void micro_slope(const T b[5], T U, T V, T W, T lam, T K, T a[5]) {
  T q2 = U * U + V * V + W * W;
  T d1 = b[0];
  T d2 = b[1] - U * b[0];
  T d3 = b[2] - V * b[0];
  T d4 = b[3] - W * b[0];
  T d5 = b[4] - U * b[1] - V * b[2] - W * b[3] + T(0.5) * q2 * b[0];
  T a5 = T(4) * lam * lam / (K + T(3)) * (T(2) * d5 - (K + T(3)) / (T(2) * lam) * d1);
  T al0 = d1 - (K + T(3)) / (T(4) * lam) * a5;
  a[4] = a5;
  a[1] = T(2) * lam * d2 - U * a5;
  a[2] = T(2) * lam * d3 - V * a5;
  a[3] = T(2) * lam * d4 - W * a5;
  a[0] = al0 - U * a[1] - V * a[2] - W * a[3] - T(0.5) * q2 * a5;
}

// time derivative coefficients from <a_n u + a_t1 v + a_t2 w + A> = 0
template <typename T>
__host__ __device__ __forceinline__ void time_slope(const Mxw<T>& M, const T an[5], const T at1[5],
                                           const T at2[5], T U, T V, T W, T lam, T K, T A[5]) {
  T s[5] = {0, 0, 0, 0, 0};
  apsi<1, 0, 0>(M, an, T(-1), s);
  apsi<0, 1, 0>(M, at1, T(-1), s);
  apsi<0, 0, 1>(M, at2, T(-1), s);
  micro_slope(s, U, V, W, lam, K, A);
}

// Moments of one distribution term with an extra u^k weight:
// out += rho [c0 <u^k psi> + c1 (<u^(k+1) a_n psi> + <u^k v a_t1 psi> + <u^k w a_t2 psi>) + c2 <u^k A psi>]
template <int k, typename T>
__host__ __device__ __forceinline__ void term_moments(const Mxw<T>& M, T rho, T c0, T c1, T c2,
                                             const T an[5], const T at1[5], const T at2[5],
                                             const T A[5], T out[5]) {
  psi5<k, 0, 0, 0>(M, rho * c0, out);
  apsi<k + 1, 0, 0>(M, an, rho * c1, out);
  apsi<k, 1, 0>(M, at1, rho * c1, out);
  apsi<k, 0, 1>(M, at2, rho * c1, out);
  apsi<k, 0, 0>(M, A, rho * c2, out);
}

template <typename T>
struct FluxParams {
  T gamma, K, tau_eps, tau_C, mu, prandtl;
  int physics;
};

// Time-averaged flux over [0, dt] (local frame) and, if want_qg, the point
// value Q(x_G, t = dt) of Eq. (point).  W*: conserved local-frame states,
// d*[3][5]: their derivatives along (n, t1, t2).
template <typename T, bool want_qg>
__host__ __device__ __forceinline__ void gks_flux(const T Wl[5], const T dWl[3][5], const T Wr[5],
                                         const T dWr[3][5], T dt, const FluxParams<T>& P, T F[5],
                                         T QG[5]) {
  const T g = P.gamma, K = P.K;
  // primitive variables of both sides
  T rl = Wl[0], Ul = Wl[1] / rl, Vl = Wl[2] / rl, Wwl = Wl[3] / rl;
  T pl = (g - T(1)) * (Wl[4] - T(0.5) * rl * (Ul * Ul + Vl * Vl + Wwl * Wwl));
  T ll = rl / (T(2) * pl);
  T rr = Wr[0], Ur = Wr[1] / rr, Vr = Wr[2] / rr, Wwr = Wr[3] / rr;
  T pr = (g - T(1)) * (Wr[4] - T(0.5) * rr * (Ur * Ur + Vr * Vr + Wwr * Wwr));
  T lr = rr / (T(2) * pr);

  Mxw<T> Ml, Mr;  // half-space moments u>0 (left) and u<0 (right)
  mxw_vw(Ml, Vl, Wwl, ll, K);
  mxw_u(Ml, Ul, ll, +1);
  mxw_vw(Mr, Vr, Wwr, lr, K);
  mxw_u(Mr, Ur, lr, -1);

  // interface equilibrium Q0 from the compatibility condition
  T Q0[5] = {0, 0, 0, 0, 0};
  psi5<0, 0, 0, 0>(Ml, rl, Q0);
  psi5<0, 0, 0, 0>(Mr, rr, Q0);
  T r0 = Q0[0], U0 = Q0[1] / r0, V0 = Q0[2] / r0, W0 = Q0[3] / r0;
  T p0 = (g - T(1)) * (Q0[4] - T(0.5) * r0 * (U0 * U0 + V0 * V0 + W0 * W0));
  T l0 = r0 / (T(2) * p0);

  // slopes of the initial distributions and kinetic-weighted equilibrium slopes
  T al[3][5], ar[3][5], ab[3][5];
  {
    T il = T(1) / rl, ir = T(1) / rr, i0 = T(1) / r0;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      T bl[5], br[5];
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        bl[k] = dWl[d][k] * il;
        br[k] = dWr[d][k] * ir;
      }
      micro_slope(bl, Ul, Vl, Wwl, ll, K, al[d]);
      micro_slope(br, Ur, Vr, Wwr, lr, K, ar[d]);
      T dq0[5] = {0, 0, 0, 0, 0};
      apsi<0, 0, 0>(Ml, al[d], rl, dq0);
      apsi<0, 0, 0>(Mr, ar[d], rr, dq0);
#pragma unroll
      for (int k = 0; k < 5; ++k) dq0[k] *= i0;
      micro_slope(dq0, U0, V0, W0, l0, K, ab[d]);
    }
  }
  // time derivatives (full-space moments of each Maxwellian)
  Mxw<T> M0;
  mxw_vw(M0, V0, W0, l0, K);
  mxw_u(M0, U0, l0, 0);
  T Ab[5], Al[5], Ar[5];
  time_slope(M0, ab[0], ab[1], ab[2], U0, V0, W0, l0, K, Ab);
  {
    Mxw<T> Mf;
    mxw_vw(Mf, Vl, Wwl, ll, K);
    mxw_u(Mf, Ul, ll, 0);
    time_slope(Mf, al[0], al[1], al[2], Ul, Vl, Wwl, ll, K, Al);
    mxw_vw(Mf, Vr, Wwr, lr, K);
    mxw_u(Mf, Ur, lr, 0);
    time_slope(Mf, ar[0], ar[1], ar[2], Ur, Vr, Wwr, lr, K, Ar);
  }
  // collision time (Sec. 5)
  T jump = fabs((pl - pr) / (pl + pr));
  T tau = P.physics ? P.mu / p0 + P.tau_C * jump * dt : (P.tau_eps + P.tau_C * jump) * dt;
  // time integrals of the coefficients of Eq. (flux), divided by dt
  T x = dt / tau;
  T e = exp(-x);
  T em1 = -expm1(-x);
  T idt = T(1) / dt;
  T c1 = (dt - tau * em1) * idt;
  T c2 = (-tau * dt + T(2) * tau * tau * em1 - tau * dt * e) * idt;
  T c3 = (T(0.5) * dt * dt - tau * dt + tau * tau * em1) * idt;
  T c4 = tau * em1 * idt;
  T c5 = (-T(2) * tau * tau * em1 + tau * dt * e) * idt;
  T c6 = (-tau * tau * em1) * idt;
#pragma unroll
  for (int k = 0; k < 5; ++k) F[k] = T(0);
  term_moments<1>(M0, r0, c1, c2, c3, ab[0], ab[1], ab[2], Ab, F);
  term_moments<1>(Ml, rl, c4, c5, c6, al[0], al[1], al[2], Al, F);
  term_moments<1>(Mr, rr, c4, c5, c6, ar[0], ar[1], ar[2], Ar, F);
  if (P.physics) {
    // heat flux relative to U0 carried by the time-averaged f, rescaled to Pr
    T Ph[5] = {0, 0, 0, 0, 0};
    term_moments<0>(M0, r0, c1, c2, c3, ab[0], ab[1], ab[2], Ab, Ph);
    term_moments<0>(Ml, rl, c4, c5, c6, al[0], al[1], al[2], Al, Ph);
    term_moments<0>(Mr, rr, c4, c5, c6, ar[0], ar[1], ar[2], Ar, Ph);
    T u2 = U0 * U0 + V0 * V0 + W0 * W0;
    T q = F[4] - (F[1] * U0 + F[2] * V0 + F[3] * W0) + T(0.5) * u2 * F[0] -
          U0 * (Ph[4] - (Ph[1] * U0 + Ph[2] * V0 + Ph[3] * W0) + T(0.5) * u2 * Ph[0]);
    F[4] += (T(1) / P.prandtl - T(1)) * q;
  }
  if (want_qg) {
    T t = dt;
    T d1 = em1, d2 = (t + tau) * e - tau, d3 = t - tau + tau * e;
    T d4 = e, d5 = -(tau + t) * e, d6 = -tau * e;
#pragma unroll
    for (int k = 0; k < 5; ++k) QG[k] = T(0);
    term_moments<0>(M0, r0, d1, d2, d3, ab[0], ab[1], ab[2], Ab, QG);
    term_moments<0>(Ml, rl, d4, d5, d6, al[0], al[1], al[2], Al, QG);
    term_moments<0>(Mr, rr, d4, d5, d6, ar[0], ar[1], ar[2], Ar, QG);
  }
}

}  // namespace hgks
