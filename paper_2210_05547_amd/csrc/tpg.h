// Thermally perfect single-species air (Sec. 2.2.2): one harmonic vibrational mode with
// Theta = 3055 K in the specific heat (Eq. 23), Keyes' conductivity (Eq. 25), Sutherland's
// viscosity (Eq. 24) and the perfect-gas equation of state (Eq. 22).
//
// Nondimensional form (scales of Sec. 2.1: T_ref = (gamma_inf - 1) T_inf, energies by
// c_inf^2 = c_p,inf T_ref): with a = (gamma_inf - 1)/gamma_inf, k0 = c_p0 / c_p,inf
// (c_p0 fixed by c_p(T_inf) = c_p,inf) and th = Theta / T_ref,
//   e(T)   = k0 T + k0 a th / (e^(th/T) - 1) - a T,
//   c_v(T) = k0 (1 + a f(th/T)) - a,   f(x) = x^2 e^x / (e^x - 1)^2,
// the enthalpy being the integral of Eq. (23) read with the oscillator's squared
// denominator, zero at 0 K.  The gas constant is that of dry air.
#pragma once
#include "air5.h"

namespace hrx {

constexpr double TPG_THETA = 3055.0;                 // K
constexpr double KEYES_C2 = 2.646e-3;                // W m^-1 K^-3/2
constexpr double KEYES_C3 = 245.4;                   // K
constexpr double KEYES_C4 = 12.0;                    // K
constexpr double TPG_R = RU / 28.9647e-3;            // J/(kg K), dry air
constexpr double LN10 = 2.302585092994045684;

// Keyes' law [W/(m K)] at T [K]
HRX_HD double keyes(double T) {
  return KEYES_C2 * sqrt(T) / (1.0 + (KEYES_C3 / T) * exp(-(KEYES_C4 * LN10) / T));
}

// x^2 e^-x / (1 - e^-x)^2 (= f(x)); vanishes for large x instead of overflowing
HRX_HD double tpg_vib(double x) {
  const double em = expm1(-x);
  return x * x * (1.0 + em) / (em * em);
}

HRX_HD double tpg_energy(double T, double k0, double th, double a) {
  return k0 * T + k0 * a * th / expm1(th / T) - a * T;
}

// s + err = a + b exactly (Knuth)
HRX_HD void two_sum(double a, double b, double& s, double& err) {
  s = a + b;
  const double bb = s - a;
  err = (a - (s - bb)) + (b - bb);
}

// Newton on e(T) = e from T0 > 0 (the previous stage's T), else from the frozen-vibration
// bound e / (k0 - a), which lies above the root (e(T) is increasing and convex, so the
// iterates fall monotonically onto it; from below, the first step lands above it);
// status 1 when |dT| <= rtol T is not reached in max_iter steps.  A last step takes the
// residual with its products split by fma and its sums by two_sum, so that T ends within
// about one unit in the last place of the root (only the vibrational term keeps its own
// rounding): the right-hand side amplifies differences of a few units in T near a wall.
HRX_HD double tpg_temperature(double e, double k0, double th, double a, double rtol,
                              int max_iter, int* status, double T0 = 0.0) {
  double T = T0 > 0.0 ? T0 : e / (k0 - a);
  *status = 1;
  for (int it = 0; it < max_iter; ++it) {
    const double x = th / T;
    const double em1 = expm1(x);
    const double g = k0 * T + k0 * a * th / em1 - a * T - e;
    const double cv = k0 * (1.0 + a * tpg_vib(x)) - a;
    const double dT = g / cv;
    T -= dT;
    if (fabs(dT) <= rtol * fabs(T)) { *status = 0; break; }
  }
  const double p1 = k0 * T, q1 = fma(k0, T, -p1);
  const double p2 = -a * T, q2 = fma(-a, T, -p2);
  const double x = th / T;
  const double v = k0 * a * th / expm1(x);
  double r, t, err = q1 + q2;
  two_sum(p1, p2, r, t);
  err += t;
  two_sum(r, v, r, t);
  err += t;
  two_sum(r, -e, r, t);
  err += t;
  const double cv = k0 * (1.0 + a * tpg_vib(x)) - a;
  return T - (r + err) / cv;
}

}  // namespace hrx
