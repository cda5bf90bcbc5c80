// Gas-kinetic (BGK) flux at one Gauss point in the local face frame
// (paper Sec. 2 Eq. (flux) and the moment systems below it; time average of
// Sec. 4.1; collision time of Sec. 5; Prandtl correction of the heat flux).
//
// Every velocity moment the scheme needs has the form <u^k psi_j W>, with W a
// polynomial in (u, v, w, xi^2) of degree <= 3 built from the expansion
// coefficients (a . psi, u a_n.psi + v a_t1.psi + w a_t2.psi, A . psi).  W is
// held in a fixed 23-monomial basis.  Because the Maxwellian factorises over
// u, v, w and xi, the (v, w, xi) part of each monomial is summed once into 16
// "G-sums" (grouped by the power of u); the moments for any u-table (half or
// full space, k = 0 or 1) are then 4-term dot products.  T is double (plain
// path) or float (inner operator of the mixed-precision form).
#pragma once
#include <hip/hip_runtime.h>

namespace hgks {

#define HGKS_HD __host__ __device__ __forceinline__

// moments of v, w (full space) and xi of one Maxwellian
template <typename T>
struct VWX {
  T v[6], w[6], x2, x4;
};

// r = 1/(2 lam), computed once per Maxwellian by the caller
template <typename T>
HGKS_HD void vwx_table(VWX<T>& M, T V, T W, T r, T K) {
  M.v[0] = T(1);
  M.v[1] = V;
  M.w[0] = T(1);
  M.w[1] = W;
#pragma unroll
  for (int k = 2; k < 6; ++k) {
    M.v[k] = V * M.v[k - 1] + T(k - 1) * r * M.v[k - 2];
    M.w[k] = W * M.w[k - 1] + T(k - 1) * r * M.w[k - 2];
  }
  M.x2 = K * r;
  M.x4 = K * (K + T(2)) * r * r;
}

// u-moments <u^k>, k < 8, from <u^0> and <u^1> (recurrence valid for the
// full space and both half spaces)
template <typename T>
HGKS_HD void u_table(T u[8], T U, T r, T u0, T u1) {
  u[0] = u0;
  u[1] = u1;
#pragma unroll
  for (int k = 2; k < 8; ++k) u[k] = U * u[k - 1] + T(k - 1) * r * u[k - 2];
}

// <u^0>, <u^1> over u > 0 (sgn > 0) or u < 0 (sgn < 0)
template <typename T>
HGKS_HD void half_base(T U, T lam, int sgn, T& u0, T& u1) {
  T sl = sqrt(lam);
  T e = exp(-lam * U * U) / sqrt(T(M_PI) * lam);
  if (sgn > 0) {
    u0 = T(0.5) * erfc(-sl * U);
    u1 = U * u0 + T(0.5) * e;
  } else {
    u0 = T(0.5) * erfc(sl * U);
    u1 = U * u0 - T(0.5) * e;
  }
}

// Monomial basis u^i v^j w^l xi^(2q), 23 entries, grouped by i:
//  i=0: 1 v w v2 w2 vw xi2 v3 vw2 vxi2 v2w w3 wxi2   i=1: u uv uw uv2 uw2 uxi2
//  i=2: u2 u2v u2w                                    i=3: u3
HGKS_HD constexpr int mono_i(int m) { return m < 13 ? 0 : (m < 19 ? 1 : (m < 22 ? 2 : 3)); }
HGKS_HD constexpr int mono_j(int m) {
  return m == 1 || m == 5 || m == 8 || m == 9 || m == 14 || m == 20 ? 1
         : m == 3 || m == 10 || m == 16                            ? 2
         : m == 7                                                  ? 3
                                                                   : 0;
}
HGKS_HD constexpr int mono_l(int m) {
  return m == 2 || m == 5 || m == 10 || m == 12 || m == 15 || m == 21 ? 1
         : m == 4 || m == 8 || m == 17                              ? 2
         : m == 11                                                  ? 3
                                                                    : 0;
}
HGKS_HD constexpr int mono_q(int m) { return m == 6 || m == 9 || m == 12 || m == 18 ? 1 : 0; }

// c += s (a . psi), psi = (1, u, v, w, (u^2+v^2+w^2+xi^2)/2)
template <typename T>
HGKS_HD void add_apsi(T c[23], const T a[5], T s) {
  c[0] += s * a[0];
  c[13] += s * a[1];
  c[1] += s * a[2];
  c[2] += s * a[3];
  T h = T(0.5) * s * a[4];
  c[19] += h;
  c[3] += h;
  c[4] += h;
  c[6] += h;
}

// c += s (u a_n.psi + v a_t1.psi + w a_t2.psi)
template <typename T>
HGKS_HD void add_slopes(T c[23], const T an[5], const T at1[5], const T at2[5], T s) {
  T hn = T(0.5) * s * an[4], h1 = T(0.5) * s * at1[4], h2 = T(0.5) * s * at2[4];
  c[13] += s * an[0];
  c[19] += s * an[1];
  c[14] += s * (an[2] + at1[1]);
  c[15] += s * (an[3] + at2[1]);
  c[22] += hn;
  c[16] += hn;
  c[17] += hn;
  c[18] += hn;
  c[1] += s * at1[0];
  c[3] += s * at1[2];
  c[5] += s * (at1[3] + at2[2]);
  c[20] += h1;
  c[7] += h1;
  c[8] += h1;
  c[9] += h1;
  c[2] += s * at2[0];
  c[4] += s * at2[3];
  c[21] += h2;
  c[10] += h2;
  c[11] += h2;
  c[12] += h2;
}

template <typename T>
struct GSum {
  T g0[4], gv[4], gw[4], g4[4];
};

template <typename T>
HGKS_HD T xi_mom(const VWX<T>& M, int q) {
  return q == 0 ? T(1) : (q == 1 ? M.x2 : M.x4);
}

// G-sums of a weight polynomial: for each power i of u,
//   g0 = sum c <v^j w^l xi^2q>,  gv: one more v,  gw: one more w,
//   g4 = sum c (<v^(j+2) w^l xi^2q> + <v^j w^(l+2) xi^2q> + <v^j w^l xi^(2q+2)>)
template <typename T>
HGKS_HD void gsum(const T c[23], const VWX<T>& M, GSum<T>& G) {
#pragma unroll
  for (int i = 0; i < 4; ++i) G.g0[i] = G.gv[i] = G.gw[i] = G.g4[i] = T(0);
#pragma unroll
  for (int m = 0; m < 23; ++m) {
    const int i = mono_i(m), j = mono_j(m), l = mono_l(m), q = mono_q(m);
    T x0 = xi_mom(M, q), x1 = xi_mom(M, q + 1);
    T vw = M.v[j] * M.w[l];
    G.g0[i] += c[m] * (vw * x0);
    G.gv[i] += c[m] * (M.v[j + 1] * M.w[l] * x0);
    G.gw[i] += c[m] * (M.v[j] * M.w[l + 1] * x0);
    G.g4[i] += c[m] * ((M.v[j + 2] * M.w[l] + M.v[j] * M.w[l + 2]) * x0 + vw * x1);
  }
}

template <typename T>
HGKS_HD void gaxpy(GSum<T>& Y, T s, const GSum<T>& X) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    Y.g0[i] += s * X.g0[i];
    Y.gv[i] += s * X.gv[i];
    Y.gw[i] += s * X.gw[i];
    Y.g4[i] += s * X.g4[i];
  }
}

// out += s <u^k psi W> for the u-table u[] and the G-sums of W
template <int k, typename T>
HGKS_HD void gmom(const T u[8], const GSum<T>& G, T s, T out[5]) {
  T o0 = T(0), o1 = T(0), o2 = T(0), o3 = T(0), o4 = T(0);
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    o0 += u[k + i] * G.g0[i];
    o1 += u[k + i + 1] * G.g0[i];
    o2 += u[k + i] * G.gv[i];
    o3 += u[k + i] * G.gw[i];
    o4 += u[k + i + 2] * G.g0[i] + u[k + i] * G.g4[i];
  }
  out[0] += s * o0;
  out[1] += s * o1;
  out[2] += s * o2;
  out[3] += s * o3;
  out[4] += s * T(0.5) * o4;
}

// Closed-form solution of <a psi> = b (normalised moments of the full-space
// Maxwellian with velocity (U,V,W), lam = rho/(2p), K internal dof): solved
// in the peculiar-velocity basis where the moment matrix is block diagonal.
// (r = 1/(2 lam) and ik3 = 1/(K + 3) are passed in: no division here)
template <typename T>
HGKS_HD void micro_slope(const T b[5], T U, T V, T W, T lam, T r, T K, T ik3, T a[5]) {
  T q2 = U * U + V * V + W * W;
  T d1 = b[0];
  T d2 = b[1] - U * b[0];
  T d3 = b[2] - V * b[0];
  T d4 = b[3] - W * b[0];
  T d5 = b[4] - U * b[1] - V * b[2] - W * b[3] + T(0.5) * q2 * b[0];
  T a5 = T(4) * lam * lam * ik3 * (T(2) * d5 - (K + T(3)) * r * d1);
  T al0 = d1 - T(0.5) * (K + T(3)) * r * a5;
  a[4] = a5;
  a[1] = T(2) * lam * d2 - U * a5;
  a[2] = T(2) * lam * d3 - V * a5;
  a[3] = T(2) * lam * d4 - W * a5;
  a[0] = al0 - U * a[1] - V * a[2] - W * a[3] - T(0.5) * q2 * a5;
}

template <typename T>
struct FluxParams {
  T gamma, K, tau_eps, tau_C, mu, prandtl;
  int physics;
};

// One distribution term of Eq. (flux): a Maxwellian (vw-table, u-table uh for
// the flux moments, u-table uf of its full space for the time derivative)
// times [c_e + c_s (u a_n.psi + v a_t1.psi + w a_t2.psi) + c_A A.psi], where
// A solves <a_n u + a_t1 v + a_t2 w + A> = 0.  Accumulates rho x the
// flux moments (k = 1) into F and the point-value moments with the second
// coefficient set into QG.
template <typename T, bool QG>
HGKS_HD void term(const VWX<T>& M, const T uh[8], const T uf[8], T rho, T U, T V, T W, T lam, T r, T K, T ik3,
                  const T an[5], const T at1[5], const T at2[5], T ce, T cs, T cA, T de, T ds, T dA, T F[5],
                  T Qg[5]) {
  GSum<T> Ga;
  {
    T c[23];
#pragma unroll
    for (int m = 0; m < 23; ++m) c[m] = T(0);
    add_slopes(c, an, at1, at2, T(1));
    gsum(c, M, Ga);
  }
  T A[5];
  {
    T rhs[5] = {0, 0, 0, 0, 0};
    gmom<0>(uf, Ga, T(-1), rhs);
    micro_slope(rhs, U, V, W, lam, r, K, ik3, A);
  }
  if (QG) {
    T c[23];
#pragma unroll
    for (int m = 0; m < 23; ++m) c[m] = T(0);
    c[0] = de;
    add_apsi(c, A, dA);
    GSum<T> Gq;
    gsum(c, M, Gq);
    gaxpy(Gq, ds, Ga);
    gmom<0>(uh, Gq, rho, Qg);
  }
  GSum<T> Gt;
  {
    T c[23];
#pragma unroll
    for (int m = 0; m < 23; ++m) c[m] = T(0);
    c[0] = ce;
    add_apsi(c, A, cA);
    gsum(c, M, Gt);
  }
  gaxpy(Gt, cs, Ga);
  gmom<1>(uh, Gt, rho, F);
}

// <psi a.psi> over a u-table: the moment of a single expansion (k = 0)
template <typename T>
HGKS_HD void apsi_mom(const VWX<T>& M, const T u[8], const T a[5], T s, T out[5]) {
  T c[23];
#pragma unroll
  for (int m = 0; m < 23; ++m) c[m] = T(0);
  add_apsi(c, a, T(1));
  GSum<T> G;
  gsum(c, M, G);
  gmom<0>(u, G, s, out);
}

// Time-averaged flux over [0, dt] (local frame) and, if want_qg, the point
// value Q(x_G, t = dt) of Eq. (point).  W*: conserved local-frame states,
// d*[3][5]: their derivatives along (n, t1, t2).  sl: storage for the 45
// slope values (left, right, equilibrium); the device passes a slot of LDS,
// so that the slopes need not stay in registers between their formation and
// the terms that use them.
template <typename T, bool want_qg>
HGKS_HD void gks_flux(const T Wl[5], const T dWl[3][5], const T Wr[5], const T dWr[3][5], T dt,
                      const FluxParams<T>& P, T F[5], T QG[5], T* sl) {
  const T g = P.gamma, K = P.K;
  const T ik3 = T(1) / (K + T(3));
  // primitive variables of both sides; per Maxwellian the factor 1/(2 lam)
  // of the moment recurrences is formed once
  T rl = Wl[0], il = T(1) / rl, Ul = Wl[1] * il, Vl = Wl[2] * il, Wwl = Wl[3] * il;
  T pl = (g - T(1)) * (Wl[4] - T(0.5) * rl * (Ul * Ul + Vl * Vl + Wwl * Wwl));
  T ll = rl / (T(2) * pl), hl = pl * il;  // lam and 1/(2 lam) = p/rho
  T rr = Wr[0], ir = T(1) / rr, Ur = Wr[1] * ir, Vr = Wr[2] * ir, Wwr = Wr[3] * ir;
  T pr = (g - T(1)) * (Wr[4] - T(0.5) * rr * (Ur * Ur + Vr * Vr + Wwr * Wwr));
  T lr = rr / (T(2) * pr), hr = pr * ir;
  T ul0, ul1, ur0, ur1;  // half-space base moments: u > 0 left, u < 0 right
  half_base(Ul, ll, +1, ul0, ul1);
  half_base(Ur, lr, -1, ur0, ur1);

  // interface equilibrium Q0 from the compatibility condition
  T Q0[5] = {0, 0, 0, 0, 0};
  {
    VWX<T> M;
    T u[8];
    vwx_table(M, Vl, Wwl, hl, K);
    u_table(u, Ul, hl, ul0, ul1);
    Q0[0] += rl * u[0];
    Q0[1] += rl * u[1];
    Q0[2] += rl * u[0] * M.v[1];
    Q0[3] += rl * u[0] * M.w[1];
    Q0[4] += rl * T(0.5) * (u[2] + u[0] * (M.v[2] + M.w[2] + M.x2));
    vwx_table(M, Vr, Wwr, hr, K);
    u_table(u, Ur, hr, ur0, ur1);
    Q0[0] += rr * u[0];
    Q0[1] += rr * u[1];
    Q0[2] += rr * u[0] * M.v[1];
    Q0[3] += rr * u[0] * M.w[1];
    Q0[4] += rr * T(0.5) * (u[2] + u[0] * (M.v[2] + M.w[2] + M.x2));
  }
  // Two receding half-space tails that carry less than 2^-40 of the
  // adjacent densities meet at this point: the interface is vacuum and
  // transports nothing.  (Below that fraction the interface temperature,
  // 1/rho0 and, for Navier-Stokes, tau = mu/p0 are dominated by rounding or
  // overflow, while the exact flux is of that relative size.)
  if (!(Q0[0] > T(1.0 / 1099511627776.0) * (rl + rr))) {
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      F[k] = T(0);
      if (want_qg) QG[k] = T(0);
    }
    return;
  }
  T r0 = Q0[0], i0 = T(1) / r0, U0 = Q0[1] * i0, V0 = Q0[2] * i0, W0 = Q0[3] * i0;
  T p0 = (g - T(1)) * (Q0[4] - T(0.5) * r0 * (U0 * U0 + V0 * V0 + W0 * W0));
  T l0 = r0 / (T(2) * p0), h0 = p0 * i0;

  // collision time (Sec. 5) and the time coefficients of Eq. (flux),
  // integrated over [0, dt] and divided by dt
  T jump = fabs((pl - pr) / (pl + pr));
  T tau = P.physics ? P.mu / p0 + P.tau_C * jump * dt : (P.tau_eps + P.tau_C * jump) * dt;
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
  // coefficients of Eq. (flux) at t^n (local t = 0) for the point value of
  // the gradient update (Sec. 4.2): the equilibrium terms vanish there
  T d1 = T(0), d2 = T(0), d3 = T(0);
  T d4 = T(1), d5 = -tau, d6 = -tau;

  // slopes of the initial distributions in the directions (n, t1, t2) and
  // the kinetic-weighted derivatives of Q0
  T(*al)[5] = reinterpret_cast<T(*)[5]>(sl);
  T(*ar)[5] = reinterpret_cast<T(*)[5]>(sl + 15);
  T(*ab)[5] = reinterpret_cast<T(*)[5]>(sl + 30);
  {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      T bl[5], br[5];
#pragma unroll
      for (int k = 0; k < 5; ++k) {
        bl[k] = dWl[d][k] * il;
        br[k] = dWr[d][k] * ir;
      }
      micro_slope(bl, Ul, Vl, Wwl, ll, hl, K, ik3, al[d]);
      micro_slope(br, Ur, Vr, Wwr, lr, hr, K, ik3, ar[d]);
    }
  }
  {
    T dq[3][5];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
      for (int k = 0; k < 5; ++k) dq[d][k] = T(0);
    VWX<T> M;
    T u[8];
    vwx_table(M, Vl, Wwl, hl, K);
    u_table(u, Ul, hl, ul0, ul1);
#pragma unroll
    for (int d = 0; d < 3; ++d) apsi_mom(M, u, al[d], rl, dq[d]);
    vwx_table(M, Vr, Wwr, hr, K);
    u_table(u, Ur, hr, ur0, ur1);
#pragma unroll
    for (int d = 0; d < 3; ++d) apsi_mom(M, u, ar[d], rr, dq[d]);
#pragma unroll
    for (int d = 0; d < 3; ++d) {
#pragma unroll
      for (int k = 0; k < 5; ++k) dq[d][k] *= i0;
      micro_slope(dq[d], U0, V0, W0, l0, h0, K, ik3, ab[d]);
    }
  }
#pragma unroll
  for (int k = 0; k < 5; ++k) F[k] = T(0);
  T Qg[5] = {0, 0, 0, 0, 0};
  // initial-distribution terms: half-space moments of g_l (u > 0), g_r (u < 0)
  // (first, so that their slopes are dead before the equilibrium term)
  {
    VWX<T> M;
    T uh[8], uf[8];
    vwx_table(M, Vl, Wwl, hl, K);
    u_table(uh, Ul, hl, ul0, ul1);
    u_table(uf, Ul, hl, T(1), Ul);
    if (P.physics)
      term<T, want_qg>(M, uh, uf, rl, Ul, Vl, Wwl, ll, hl, K, ik3, al[0], al[1], al[2], c4, c5, c6, d4, d5, d6, F, Qg);
    else
      term<T, want_qg>(M, uh, uf, rl, Ul, Vl, Wwl, ll, hl, K, ik3, al[0], al[1], al[2], c4, c5, c6, d4, d5, d6, F, Qg);
  }
  {
    VWX<T> M;
    T uh[8], uf[8];
    vwx_table(M, Vr, Wwr, hr, K);
    u_table(uh, Ur, hr, ur0, ur1);
    u_table(uf, Ur, hr, T(1), Ur);
    if (P.physics)
      term<T, want_qg>(M, uh, uf, rr, Ur, Vr, Wwr, lr, hr, K, ik3, ar[0], ar[1], ar[2], c4, c5, c6, d4, d5, d6, F, Qg);
    else
      term<T, want_qg>(M, uh, uf, rr, Ur, Vr, Wwr, lr, hr, K, ik3, ar[0], ar[1], ar[2], c4, c5, c6, d4, d5, d6, F, Qg);
  }
  // equilibrium term: full-space moments of g0
  {
    VWX<T> M;
    T u[8];
    vwx_table(M, V0, W0, h0, K);
    u_table(u, U0, h0, T(1), U0);
    // (no point-value contribution: its coefficients d1..d3 vanish at t^n)
    if (P.physics)
      term<T, false>(M, u, u, r0, U0, V0, W0, l0, h0, K, ik3, ab[0], ab[1], ab[2], c1, c2, c3, d1, d2, d3, F, Qg);
    else
      term<T, false>(M, u, u, r0, U0, V0, W0, l0, h0, K, ik3, ab[0], ab[1], ab[2], c1, c2, c3, d1, d2, d3, F, Qg);
  }
  if (P.physics) {
    // Prandtl correction: the BGK flux carries the heat flux of Pr = 1,
    // -mu c_p dT/dn; the energy flux gets (1/Pr - 1) times that.  T = 1/(2
    // lam), and the normal slope of the interface Maxwellian has the
    // coefficient -2 dlam/dn on (u^2+v^2+w^2+xi^2)/2: dT/dn = ab[0][4] / (4 lam0^2)
    F[4] += (T(1) / P.prandtl - T(1)) * (-P.mu * g / (g - T(1)) * ab[0][4] / (T(4) * l0 * l0));
  }
  if (want_qg)
#pragma unroll
    for (int k = 0; k < 5; ++k) QG[k] = Qg[k];
}

// the same with the slopes in a local array (host builds)
template <typename T, bool want_qg>
HGKS_HD void gks_flux(const T Wl[5], const T dWl[3][5], const T Wr[5], const T dWr[3][5], T dt,
                      const FluxParams<T>& P, T F[5], T QG[5]) {
  T sl[45];
  gks_flux<T, want_qg>(Wl, dWl, Wr, dWr, dt, P, F, QG, sl);
}

// First-order kinetic flux vector splitting (the Mach 3 retest of Sec. 5):
// the free transport of the two half-space Maxwellians of the side states,
// F = rho_l <u psi>_{u>0} + rho_r <u psi>_{u<0}, with no collision term and
// no slopes.  Per side, with h = 1/(2 lam):
//   <v^2 + w^2 + xi^2> = V^2 + W^2 + (K + 2) h,  <u^2> and <u^3> from the
//   recurrence of u_table.
template <typename T>
HGKS_HD void kfvs_flux(const T Wl[5], const T Wr[5], T g, T K, T F[5]) {
#pragma unroll
  for (int k = 0; k < 5; ++k) F[k] = T(0);
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const T* W = s ? Wr : Wl;
    T rho = W[0], irho = T(1) / rho, U = W[1] * irho, V = W[2] * irho, Ww = W[3] * irho;
    T p = (g - T(1)) * (W[4] - T(0.5) * rho * (U * U + V * V + Ww * Ww));
    T lam = rho / (T(2) * p), h = p * irho;
    T u0, u1;
    half_base(U, lam, s ? -1 : +1, u0, u1);
    T u2 = U * u1 + h * u0;
    T u3 = U * u2 + T(2) * h * u1;
    T e = V * V + Ww * Ww + (K + T(2)) * h;
    F[0] += rho * u1;
    F[1] += rho * u2;
    F[2] += rho * u1 * V;
    F[3] += rho * u1 * Ww;
    F[4] += rho * T(0.5) * (u3 + u1 * e);
  }
}

#undef HGKS_HD

}  // namespace hgks
