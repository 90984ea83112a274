// Pointwise thermochemistry of 5-species air (N2, O2, NO, N, O) and of a calorically
// perfect gas, written for gfx950 device code and usable on the host.
//
// Paper: Sec. 2.2.1 (mixture sums, Eq. 12; finite-rate chemistry, Eqs. 13-15;
// Ramshaw diffusion with the averaged coefficient, Eqs. 18-19; frozen conductivity
// in the heat flux), Sec. 2.2.2 (CPG, Eq. 22; Sutherland, Eq. 24) and Sec. 3.4 (every
// state evaluation needs the iterative solution of a nonlinear equation: here the
// Newton inversion of e(T)).  The paper delegates species data and mixture rules to
// a thermochemical library without printing them; the model used here is
//  * rigid-rotor/harmonic-oscillator species with the ground electronic multiplet
//    lumped into a degeneracy and 0 K formation enthalpies,
//  * first Chapman-Enskog transport with Lennard-Jones 12-6 collision integrals
//    (Neufeld-Janzen-Aziz fits), Eucken conductivities and Wilke mixing,
//  * Park's 5-species air mechanism in third-body form with equilibrium constants
//    from the species Gibbs energies.
// Every function is templated on the floating type R of the transport and rate
// arithmetic (double for the FP64 path, float where the mixed form allows it);
// the energy inversion is always double.
#pragma once
#include <hip/hip_runtime.h>
#include <math.h>

#define HRX_HD __host__ __device__ __forceinline__

namespace hrx {

constexpr int NS = 5;

// SI 2019 exact constants
constexpr double KB = 1.380649e-23;
constexpr double HPL = 6.62607015e-34;
constexpr double NAV = 6.02214076e23;
constexpr double RU = KB * NAV;
constexpr double P0 = 1.0e5;          // standard-state pressure of the Gibbs energies
constexpr double PI = 3.14159265358979323846;

// species order N2, O2, NO, N, O
HRX_HD double molar_mass(int s) {
  constexpr double m[NS] = {28.0134e-3, 31.9988e-3, 30.0061e-3, 14.0067e-3, 15.9994e-3};
  return m[s];
}
HRX_HD double theta_vib(int s) {
  constexpr double t[NS] = {3393.5, 2273.6, 2739.7, 0.0, 0.0};
  return t[s];
}
HRX_HD double theta_rot(int s) {
  constexpr double t[NS] = {2.875, 2.080, 2.406, 1.0, 1.0};
  return t[s];
}
HRX_HD double sym_number(int s) {
  constexpr double t[NS] = {2.0, 2.0, 1.0, 1.0, 1.0};
  return t[s];
}
HRX_HD double g_elec(int s) {
  constexpr double t[NS] = {1.0, 3.0, 4.0, 4.0, 9.0};
  return t[s];
}
HRX_HD double hf0_molar(int s) {   // J/mol at 0 K
  constexpr double t[NS] = {0.0, 0.0, 89.775e3, 470.82e3, 246.79e3};
  return t[s];
}
HRX_HD bool is_diatomic(int s) { return s < 3; }
HRX_HD double lj_sigma(int s) {    // m
  constexpr double t[NS] = {3.798e-10, 3.467e-10, 3.492e-10, 3.298e-10, 3.050e-10};
  return t[s];
}
HRX_HD double lj_eps(int s) {      // K
  constexpr double t[NS] = {71.4, 106.7, 116.7, 71.4, 106.7};
  return t[s];
}
HRX_HD double gas_const(int s) { return RU / molar_mass(s); }

// ----------------------------------------------------------------- thermodynamics
// Species energy and heat capacity per unit mass at one temperature:
//   e_s = R_s [(3/2 + r_s) T + r_s theta_s / (exp(theta_s/T) - 1)] + h_f,s(0 K)/M_s
// with r_s = 1 for the diatomics (one rotational and one vibrational mode), 0 for atoms.
// em1[s] = exp(theta_s/T) - 1 of the three diatomics is kept for reuse (Gibbs energies).
struct SpeciesThermo {
  double e[NS];    // J/kg
  double cv[NS];   // J/(kg K)
  double em1[3];
};

HRX_HD void species_e_cv(double T, SpeciesThermo& st) {
  const double iT = 1.0 / T;
  // the three molecules (species 0..2): e^x - 1 and its reciprocal, one division for
  // the three (prefix products)
  double x[3], em1[3];
#pragma unroll
  for (int s = 0; s < 3; ++s) {
    x[s] = theta_vib(s) * iT;
    em1[s] = expm1(x[s]);
  }
  const double p01 = em1[0] * em1[1];
  const double inv = 1.0 / (p01 * em1[2]);
  double iem[3];
  iem[2] = inv * p01;
  const double inv01 = inv * em1[2];
  iem[1] = inv01 * em1[0];
  iem[0] = inv01 * em1[1];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const double Rs = gas_const(s);
    const double hf = hf0_molar(s) / molar_mass(s);
    if (is_diatomic(s)) {
      const double ex = em1[s] + 1.0;
      st.em1[s] = em1[s];
      st.e[s] = Rs * (2.5 * T + theta_vib(s) * iem[s]) + hf;
      st.cv[s] = Rs * (2.5 + x[s] * x[s] * ex * (iem[s] * iem[s]));
    } else {
      st.e[s] = Rs * (1.5 * T) + hf;
      st.cv[s] = Rs * 1.5;
    }
  }
}

HRX_HD void species_h(double T, double* h) {
  const double iT = 1.0 / T;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const double Rs = gas_const(s);
    const double hf = hf0_molar(s) / molar_mass(s);
    if (is_diatomic(s)) {
      const double em1 = expm1(theta_vib(s) * iT);
      h[s] = Rs * (2.5 * T + theta_vib(s) / em1) + hf + Rs * T;
    } else {
      h[s] = Rs * (1.5 * T) + hf + Rs * T;
    }
  }
}

HRX_HD double mixture_e(double T, const double* Y) {
  SpeciesThermo st;
  species_e_cv(T, st);
  double e = 0.0;
#pragma unroll
  for (int s = 0; s < NS; ++s) e += Y[s] * st.e[s];
  return e;
}

HRX_HD double mixture_R(const double* Y) {
  double r = 0.0;
#pragma unroll
  for (int s = 0; s < NS; ++s) r += Y[s] * gas_const(s);
  return r;
}

constexpr double T_MIN = 50.0;
constexpr double T_GUESS_MAX = 1.0e5;

// Newton inversion of e = sum_s Y_s e_s(T) (Sec. 3.4).  e(T) is increasing and
// convex (c_v rises with T), so Newton's method converges from any start: from below
// the root the first step lands above it, and from above the iterates decrease
// monotonically.  Cold start: the temperature that solves the energy equation with
// fully excited vibration (a lower bound of the root).  Warm start: a previous
// temperature T_guess in (T_MIN, T_GUESS_MAX), which the caller may pass to save
// iterations; the root is the same.  Stops when |dT| <= rtol T.  status: 0 converged,
// 1 no convergence in max_iter, 2 energy below e(T_MIN).  When st_last is given and the
// iteration converged, it receives the species state at the last iterate, which lies
// within rtol T of the returned root (callers reuse it instead of a fresh evaluation).
HRX_HD double temperature_from_energy(double e, const double* Y, double rtol, int max_iter,
                                      int* status, int* iters, double T_guess = 0.0,
                                      SpeciesThermo* st_last = nullptr) {
  double ef = 0.0, cfull = 0.0, emin = 0.0;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const double Rs = gas_const(s);
    ef += Y[s] * (hf0_molar(s) / molar_mass(s));
    cfull += Y[s] * Rs * (is_diatomic(s) ? 3.5 : 1.5);
    // e_s(T_MIN): at 50 K the vibrational energy theta/(exp(theta/T) - 1) is below
    // 1e-18 of the translational-rotational part for every species, so it vanishes in
    // double precision and is left out
    emin += Y[s] * (Rs * ((is_diatomic(s) ? 2.5 : 1.5) * T_MIN) + hf0_molar(s) / molar_mass(s));
  }
  *iters = 0;
  if (!(e >= emin)) {
    *status = 2;
    return T_MIN;
  }
  double T = (T_guess > T_MIN && T_guess < T_GUESS_MAX) ? T_guess : (e - ef) / cfull;
  if (T < T_MIN) T = T_MIN;
  SpeciesThermo st;
  for (int it = 0; it < max_iter; ++it) {
    species_e_cv(T, st);
    double f = 0.0, cv = 0.0;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
      f += Y[s] * st.e[s];
      cv += Y[s] * st.cv[s];
    }
    f -= e;
    const double dT = f / cv;
    T = T - dT;
    *iters = it + 1;
    if (fabs(dT) <= rtol * T) {
      *status = 0;
      if (st_last) *st_last = st;
      return T;
    }
  }
  *status = 1;
  return T;
}

// ----------------------------------------------------------------- transport
constexpr double X_CLIP = 1e-12;

// Reciprocals of NS nonzero values with one division (prefix products, then the
// inverse of the full product walked back): r_s = 1/x_s to a few ulp.
template <class R>
HRX_HD void reciprocals(const R* x, R* r) {
  R pre[NS];
  pre[0] = x[0];
#pragma unroll
  for (int s = 1; s < NS; ++s) pre[s] = pre[s - 1] * x[s];
  R inv = R(1) / pre[NS - 1];
#pragma unroll
  for (int s = NS - 1; s > 0; --s) {
    r[s] = inv * pre[s - 1];
    inv = inv * x[s];
  }
  r[0] = inv;
}

template <class R>
struct Transport {
  R mu, kappa;     // Pa s, W/(m K)
  R D[NS];         // m^2/s, averaged coefficients of Eq. (19)
  R iD[10];        // s/m^2, reciprocal binary coefficients 1/D_sr of the pairs s < r in
                   // the order (0,1), (0,2), .., (3,4) (the Stefan-Maxwell system)
};

// Mixture viscosity, frozen conductivity (Wilke/Eucken) and averaged diffusion
// coefficients at (T, p, X).  cv[s] is the species c_v at T (J/(kg K)).
//   mu_s  = (5/16) sqrt(pi m_s k T) / (pi sigma_s^2 Omega22*(T/eps_s))
//   D_sr  = (3/16) sqrt(2 pi k^3 T^3 / m_sr) / (p pi sigma_sr^2 Omega11*(T/eps_sr))
//   Omega22*(x) = 1.16145 x^-0.14874 + 0.52487 e^-0.77320x + 2.16178 e^-2.43787x
//   Omega11*(x) = 1.06036 x^-0.15610 + 0.19300 e^-0.47635x + 1.03587 e^-1.52996x
//                 + 1.76474 e^-3.89411x                        (Neufeld et al. 1972)
//   kappa_s = mu_s (15/4 R_s + c_v,int,s)   (Eucken; c_v,int = c_v - 3/2 R_s)
//   phi_sr = [1 + sqrt(mu_s/mu_r) (M_r/M_s)^(1/4)]^2 / sqrt(8 (1 + M_s/M_r))
//   mu = sum_s X_s mu_s / sum_r X_r phi_sr, kappa likewise;
//   D_s = (1 - X_s) / sum_{r != s} X_r / D_sr (Eq. 19) with 1 - X_s formed as
//   sum_{r != s} X_r and every X_r clipped below at 1e-12 in this formula only.
// The molecular constants are folded in double precision so that the float
// instantiation sees only well-scaled numbers; powers x^a are exp(a (ln T - ln eps)).
template <class R>
HRX_HD void mixture_transport(double T, double p, const double* X, const double* cv,
                              Transport<R>& out) {
  R mu_s[NS], k_s[NS], smu[NS], ismu[NS], om[NS], iom[NS];
  const R Tr = R(T);
  const R sqT = sqrt(Tr);
  const R lnT = log(Tr);
  // (T/eps)^a = T^a eps^-a: one power of T per fit, shared by all species or pairs
  const R T22 = exp(R(-0.14874) * lnT);
  const R T11 = exp(R(-0.15610) * lnT);
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const R Ts = Tr * R(1.0 / lj_eps(s));
    om[s] = R(1.16145 * pow(lj_eps(s), 0.14874)) * T22 +
            R(0.52487) * exp(R(-0.77320) * Ts) + R(2.16178) * exp(R(-2.43787) * Ts);
  }
  reciprocals(om, iom);
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const double m = molar_mass(s) / NAV;
    const double sig = lj_sigma(s);
    const R A = R((5.0 / 16.0) * sqrt(PI * m * KB) / (PI * sig * sig));
    mu_s[s] = A * sqT * iom[s];
    const R Rs = R(gas_const(s));
    const R cv_int = R(cv[s]) - R(1.5) * Rs;
    k_s[s] = mu_s[s] * (R(3.75) * Rs + cv_int);
    smu[s] = sqrt(mu_s[s]);
  }
  reciprocals(smu, ismu);
  R mu = R(0), kap = R(0);
  R wden[NS], iwden[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    R den = R(0);
#pragma unroll
    for (int r = 0; r < NS; ++r) {
      R phi;
      if (r == s) {
        phi = R(1);
      } else {
        const R a = R(1) + smu[s] * ismu[r] * R(pow(molar_mass(r) / molar_mass(s), 0.25));
        phi = a * a * R(1.0 / sqrt(8.0 * (1.0 + molar_mass(s) / molar_mass(r))));
      }
      den += R(X[r]) * phi;
    }
    wden[s] = den;
  }
  reciprocals(wden, iwden);
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const R xd = R(X[s]) * iwden[s];
    mu += xd * mu_s[s];
    kap += xd * k_s[s];
  }
  out.mu = mu;
  out.kappa = kap;
  // reciprocal binary coefficients 1/D_sr = p Omega11 / (B_sr T^(3/2)), each pair
  // accumulated straight into the two sums of Eq. (19) that use it (the pairs are
  // visited so that every sum still runs over r in increasing order)
  R Xc[NS], den[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    Xc[s] = R(X[s] > X_CLIP ? X[s] : X_CLIP);
    den[s] = R(0);
  }
  const R pr_iT15 = R(p) / (Tr * sqT);
  int q = 0;
#pragma unroll
  for (int s = 0; s < NS; ++s) {
#pragma unroll
    for (int r = s + 1; r < NS; ++r, ++q) {
      const double ms = molar_mass(s) / NAV, mr = molar_mass(r) / NAV;
      const double msr = ms * mr / (ms + mr);
      const double sig = 0.5 * (lj_sigma(s) + lj_sigma(r));
      const double eps = sqrt(lj_eps(s) * lj_eps(r));
      const R iB = R((PI * sig * sig) / ((3.0 / 16.0) * sqrt(2.0 * PI * KB * KB * KB / msr)));
      const R Ts = Tr * R(1.0 / eps);
      const R om = R(1.06036 * pow(eps, 0.15610)) * T11 +
                   R(0.19300) * exp(R(-0.47635) * Ts) + R(1.03587) * exp(R(-1.52996) * Ts) +
                   R(1.76474) * exp(R(-3.89411) * Ts);
      const R v = pr_iT15 * om * iB;
      out.iD[q] = v;
      den[s] += Xc[r] * v;
      den[r] += Xc[s] * v;
    }
  }
  R iden[NS];
  reciprocals(den, iden);
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    R num = R(0);
#pragma unroll
    for (int r = 0; r < NS; ++r)
      if (r != s) num += Xc[r];
    out.D[s] = num * iden[s];
  }
}

// Sutherland's law, Eq. (24): C1 = 1.458e-6 kg/(m s K^1/2), T_S = 110.4 K.
template <class R>
HRX_HD R sutherland(R T) {
  return R(1.458e-6) * T * sqrt(T) / (T + R(110.4));
}

// ----------------------------------------------------------------- chemistry
// Standard-state molar Gibbs energy g_s/(R_u T) at p0 (statistical mechanics):
//   g_s/(R_u T) = h_f,s/(R_u T) - ln[(2 pi m_s k T/h^2)^(3/2) k T/p0] - ln g_el,s
//                 - r_s ln(T/(sigma_s theta_r,s)) + r_s ln(1 - exp(-theta_s/T))
// em1[s] = exp(theta_s/T) - 1 of the diatomics (1 - exp(-x) = em1/(em1 + 1)).
HRX_HD void gibbs_over_RT(double iT, double lnT, const double* em1, double* g) {
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    const double m = molar_mass(s) / NAV;
    const double ltr = 1.5 * log(2.0 * PI * m * KB / (HPL * HPL)) + 2.5 * lnT + log(KB / P0);
    double gs = (hf0_molar(s) / RU) * iT - ltr - log(g_elec(s));
    if (is_diatomic(s)) {
      gs -= lnT - log(sym_number(s) * theta_rot(s));
      gs += log(em1[s] / (em1[s] + 1.0));
    }
    g[s] = gs;
  }
}

struct Reaction {
  double C;          // cm^3 / (mol s)
  double n;
  double theta;      // K
};

// Park-type mechanism, third-body form (Eq. 13-14):
//   0: N2 + M = 2N + M      1: O2 + M = 2O + M     2: NO + M = N + O + M
//   3: N2 + O = NO + N      4: NO + O = O2 + N
HRX_HD Reaction reaction(int r) {
  constexpr Reaction t[5] = {{7.0e21, -1.6, 113200.0}, {2.0e21, -1.5, 59500.0},
                             {5.0e15, 0.0, 75500.0},   {6.4e17, -1.0, 38400.0},
                             {8.4e12, 0.0, 19450.0}};
  return t[r];
}
// third-body efficiencies (relative to the reference partner)
HRX_HD double tb_eff(int r, int s) {
  constexpr double z[3][NS] = {{1.0, 1.0, 1.0, 30.0 / 7.0, 30.0 / 7.0},
                               {1.0, 1.0, 1.0, 5.0, 5.0},
                               {1.0, 1.0, 22.0, 22.0, 22.0}};
  return z[r][s];
}

// exp in the precision of the rate arithmetic: FP64 for R = double, and for R = float
// FP64 at and above T_hi (where the rates matter), FP32 below with the argument
// clamped to the float range.  The argument itself is always formed in FP64.
template <class R>
HRX_HD R rate_exp(double x, bool hi) {
  if (sizeof(R) == sizeof(double) || hi) return R(exp(x));
  const float xf = (float)(x < -87.0 ? -87.0 : (x > 88.0 ? 88.0 : x));
  return R(expf(xf));
}

// Net mass production rates wdot_s [kg/(m^3 s)] from partial densities [kg/m^3] and T.
// Rates of progress R_r = (k_f prod c^nu' - k_b prod c^nu'') * (sum Z c) (Eq. 14),
// k_f = C T^n exp(-theta/T) (the printed exponent read with a minus sign), k_b = k_f/K_c,
// K_c = (p0/(R_u T))^dnu exp(-sum dnu g/(R_u T)); wdot_s = M_s sum_r (nu'' - nu') R_r (Eq. 15).
// Both k_f and k_b are formed as one exponential of a log-sum (C T^n exp(-theta/T)
// = C exp(n ln T - theta/T)); em1 as for gibbs_over_RT.
template <class R>
HRX_HD void production_rates(const double* rho_s, double T, const double* em1, R* wdot,
                             double T_hi = 0.0) {
  const double lnT = log(T);
  const double iT = 1.0 / T;
  double g[NS];
  gibbs_over_RT(iT, lnT, em1, g);
  R c[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) c[s] = R(rho_s[s] * (1.0 / molar_mass(s)));
  const double ln_c0 = log(P0 / RU) - lnT;     // ln(p0/(R_u T))
  const double dG[5] = {2.0 * g[3] - g[0], 2.0 * g[4] - g[1], g[3] + g[4] - g[2],
                        g[2] + g[3] - g[0] - g[4], g[1] + g[3] - g[2] - g[4]};
  const double dnu[5] = {1.0, 1.0, 1.0, 0.0, 0.0};
  const R fwdp[5] = {c[0], c[1], c[2], c[0] * c[4], c[2] * c[4]};
  const R bwdp[5] = {c[3] * c[3], c[4] * c[4], c[3] * c[4], c[2] * c[3], c[1] * c[3]};
  const bool hi = T >= T_hi;
  R Rr[5];
#pragma unroll
  for (int r = 0; r < 5; ++r) {
    const Reaction re = reaction(r);
    const double lkf = log(re.C * 1e-6) + re.n * lnT - re.theta * iT;
    const R kf = rate_exp<R>(lkf, hi);
    const R kb = rate_exp<R>(lkf + dG[r] - dnu[r] * ln_c0, hi);
    R tb = R(1);
    if (r < 3) {
      tb = R(0);
#pragma unroll
      for (int s = 0; s < NS; ++s) tb += R(tb_eff(r, s)) * c[s];
    }
    Rr[r] = (kf * fwdp[r] - kb * bwdp[r]) * tb;
  }
  wdot[0] = R(molar_mass(0)) * (-Rr[0] - Rr[3]);
  wdot[1] = R(molar_mass(1)) * (-Rr[1] + Rr[4]);
  wdot[2] = R(molar_mass(2)) * (-Rr[2] + Rr[3] - Rr[4]);
  wdot[3] = R(molar_mass(3)) * (R(2) * Rr[0] + Rr[2] + Rr[3] + Rr[4]);
  wdot[4] = R(molar_mass(4)) * (R(2) * Rr[1] + Rr[2] - Rr[3] - Rr[4]);
}

HRX_HD void vib_em1(double T, double* em1) {
#pragma unroll
  for (int s = 0; s < 3; ++s) em1[s] = expm1(theta_vib(s) / T);
}

// ----------------------------------------------------------------- equilibrium (LTE)
// Composition of local thermodynamic equilibrium (Sec. 2.2.1, frozen and equilibrium
// flow): at density rho [kg/m^3] and temperature T [K], the minimum of the mixture's free
// energy over the compositions whose element-N mass fraction is xiN.  At that minimum
// every species sits at c_s = (p0/(R_u T)) exp(-g_s/(R_u T) + sum_e a_es lambda_e): the
// atoms carry the element potentials, u = ln c_N and w = ln c_O, and the molecules follow
// from the dissociation equilibria, c_N2 = c_N^2 / K_1, c_O2 = c_O^2 / K_2,
// c_NO = c_N c_O / K_3 (K_c from the Gibbs energies, as the chemistry uses them).
// Newton's method on the two element balances in (u, w), each step limited to 1 in
// either logarithm, from the smaller of the atom-rich and the molecule-rich limits;
// stops after the step that is below rtol (a relative change of the concentrations).
// One element alone has the closed form c = 2 n / (1 + sqrt(1 + 8 n / K)).
// status: 0 converged, 1 not converged in max_iter, 3 invalid input (Y = NaN).
HRX_HD void equilibrium_composition(double rho, double T, double xiN, double rtol, int max_iter,
                                    double* Y, int* status) {
  if (!(rho > 0.0) || !(T > 0.0) || !(xiN >= 0.0) || !(xiN <= 1.0) || !isfinite(rho) ||
      !isfinite(T)) {
    for (int s = 0; s < NS; ++s) Y[s] = __builtin_nan("");
    *status = 3;
    return;
  }
  const double lnT = log(T), iT = 1.0 / T;
  double em1[3], g[NS];
  vib_em1(T, em1);
  gibbs_over_RT(iT, lnT, em1, g);
  const double lnc0 = log(P0 / RU) - lnT;                 // ln(p0/(R_u T))
  const double lK1 = lnc0 - (2.0 * g[3] - g[0]);          // N2 = 2N
  const double lK2 = lnc0 - (2.0 * g[4] - g[1]);          // O2 = 2O
  const double lK3 = lnc0 - (g[3] + g[4] - g[2]);         // NO = N + O
  const double nN = rho * xiN / molar_mass(3);
  const double nO = rho * (1.0 - xiN) / molar_mass(4);
  const double irho = 1.0 / rho;
  *status = 0;
  if (nN == 0.0 || nO == 0.0) {
    // one element: atoms c and molecules c^2/K with 2 c^2 / K + c = n
    const bool n_only = nO == 0.0;
    const double ne = n_only ? nN : nO, lK = n_only ? lK1 : lK2;
    // (the molecule from its own equilibrium c^2 / K: as 1 - Y_atom it would lose its
    // digits where it is a trace species)
    const double c = 2.0 * ne / (1.0 + sqrt(1.0 + 8.0 * exp(log(ne) - lK)));
    for (int s = 0; s < NS; ++s) Y[s] = 0.0;
    Y[n_only ? 3 : 4] = c * (n_only ? molar_mass(3) : molar_mass(4)) * irho;
    Y[n_only ? 0 : 1] = exp(2.0 * log(c) - lK) * (n_only ? molar_mass(0) : molar_mass(1)) * irho;
    return;
  }
  double u = fmin(log(nN), 0.5 * (lK1 + log(0.5 * nN)));
  double w = fmin(log(nO), 0.5 * (lK2 + log(0.5 * nO)));
  const double inN = 1.0 / nN, inO = 1.0 / nO;
  bool conv = false;
  for (int it = 0; it < max_iter; ++it) {
    const double cN = exp(u), cO = exp(w);
    const double cN2 = exp(2.0 * u - lK1), cO2 = exp(2.0 * w - lK2), cNO = exp(u + w - lK3);
    const double F1 = (2.0 * cN2 + cNO + cN) * inN - 1.0;
    const double F2 = (2.0 * cO2 + cNO + cO) * inO - 1.0;
    const double a = (4.0 * cN2 + cNO + cN) * inN, b = cNO * inN;
    const double c = cNO * inO, d = (4.0 * cO2 + cNO + cO) * inO;
    const double idet = 1.0 / (a * d - b * c);
    double du = -(d * F1 - b * F2) * idet, dw = -(a * F2 - c * F1) * idet;
    const double step = fmax(fabs(du), fabs(dw));
    if (step > 1.0) {
      du /= step;
      dw /= step;
    }
    u += du;
    w += dw;
    if (step <= rtol) {
      conv = true;
      break;
    }
  }
  if (!conv) *status = 1;
  Y[0] = exp(2.0 * u - lK1) * molar_mass(0) * irho;
  Y[1] = exp(2.0 * w - lK2) * molar_mass(1) * irho;
  Y[2] = exp(u + w - lK3) * molar_mass(2) * irho;
  Y[3] = exp(u) * molar_mass(3) * irho;
  Y[4] = exp(w) * molar_mass(4) * irho;
}

}  // namespace hrx
