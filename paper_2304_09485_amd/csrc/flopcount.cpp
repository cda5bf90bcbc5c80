// Algorithmic operation count of the gas-kinetic flux at one Gauss point.
//
// The flux function of gks_flux.h is instantiated on the host with a scalar
// type that counts every arithmetic operation it performs; the counts are the
// algorithmic work per Gauss point used for the flux kernel's roofline.
// Convention: +, -, *, / and sqrt count one FP64 operation each (an FMA is two);
// exp, expm1 and erfc are reported separately as transcendental calls.
// Output: a JSON object on stdout.
#include <cmath>
#include <cstdio>

#include "gks_flux.h"

namespace {
long n_add = 0, n_mul = 0, n_div = 0, n_sqrt = 0, n_trans = 0;

// A value constructed from a literal 0 or 1 is a structural constant: the
// compiler folds x * 0, x + 0 and x * 1, so those are not counted.
struct C {
  double v;
  bool z, one;
  C() : v(0), z(true), one(false) {}
  C(double x) : v(x), z(x == 0.0), one(x == 1.0) {}
  explicit C(int x) : v(x), z(x == 0), one(x == 1) {}
  static C val(double x) {
    C c(x);
    c.z = c.one = false;
    return c;
  }
};
inline C operator+(C a, C b) {
  if (a.z) return b;
  if (b.z) return a;
  ++n_add;
  return C::val(a.v + b.v);
}
inline C operator-(C a) {
  C r = C::val(-a.v);
  r.z = a.z;
  return r;
}
inline C operator-(C a, C b) { return a + (-b); }
inline C operator*(C a, C b) {
  if (a.z || b.z) return C();
  if (a.one) return b;
  if (b.one) return a;
  ++n_mul;
  return C::val(a.v * b.v);
}
inline C operator/(C a, C b) {
  if (a.z) return C();
  if (b.one) return a;
  ++n_div;
  return C::val(a.v / b.v);
}
inline bool operator>(C a, C b) { return a.v > b.v; }  // a comparison, not counted
inline C& operator+=(C& a, C b) { a = a + b; return a; }
inline C& operator-=(C& a, C b) { a = a - b; return a; }
inline C& operator*=(C& a, C b) { a = a * b; return a; }
inline C sqrt(C a) { ++n_sqrt; return C(std::sqrt(a.v)); }
inline C exp(C a) { ++n_trans; return C(std::exp(a.v)); }
inline C expm1(C a) { ++n_trans; return C(std::expm1(a.v)); }
inline C erfc(C a) { ++n_trans; return C(std::erfc(a.v)); }
inline C fabs(C a) { return C(std::fabs(a.v)); }

void reset() { n_add = n_mul = n_div = n_sqrt = n_trans = 0; }

template <bool QG>
void count(int physics, const char* name, bool last) {
  reset();
  C Wl[5] = {1.1, 0.3, 0.05, -0.02, 2.0}, Wr[5] = {0.9, 0.25, 0.01, 0.03, 1.7};
  C dWl[3][5], dWr[3][5];
  for (int d = 0; d < 3; ++d)
    for (int k = 0; k < 5; ++k) {
      dWl[d][k] = C(0.01 * (d + 1) * (k + 1));
      dWr[d][k] = C(-0.02 * (d + 1) + 0.003 * k);
    }
  hgks::FluxParams<C> P;
  P.gamma = C(1.4);
  P.K = C(2.0);
  P.tau_eps = C(0.1);
  P.tau_C = C(1.0);
  P.mu = C(1e-3);
  P.prandtl = C(0.72);
  P.physics = physics;
  C F[5], Q[5];
  hgks::gks_flux<C, QG>(Wl, dWl, Wr, dWr, C(0.01), P, F, Q);
  long flops = n_add + n_mul + n_div + n_sqrt;
  std::printf("  \"%s\": %ld,\n  \"%s_detail\": {\"add\": %ld, \"mul\": %ld, \"div\": %ld, \"sqrt\": %ld, "
              "\"transcendental\": %ld}%s\n",
              name, flops, name, n_add, n_mul, n_div, n_sqrt, n_trans, last ? "" : ",");
}
}  // namespace

int main() {
  std::printf("{\n");
  count<false>(0, "euler", false);
  count<true>(0, "euler_qg", false);
  count<false>(1, "ns", true);
  std::printf("}\n");
  return 0;
}
