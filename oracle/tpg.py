"""Thermally perfect gas, Sec. 2.2.2 (oracle; test infrastructure only).

Single-species air whose specific heat follows one harmonic vibrational mode (Eq. 23):
  c_p(T) = c_p0 [1 + (gamma_inf - 1)/gamma_inf (Theta/T)^2 e^(Theta/T)/(e^(Theta/T) - 1)^2]
with Theta = 3055 K and c_p0 chosen so that c_p(T_inf) = c_p,inf; Sutherland's viscosity
(Eq. 24) and Keyes' conductivity (Eq. 25),
  kappa(T) = C2 T^(1/2) / (1 + (C3/T) 10^(-C4/T)),  C2 = 2.646e-3, C3 = 245.4 K, C4 = 12 K;
and the perfect-gas equation of state of the calorically perfect case (Eq. 22).

Readings (where the paper is silent or garbled):
* Eq. (23) prints the denominator e^(Theta/T) - 1 unsquared; the harmonic oscillator's
  specific heat, which the cited thermally perfect models use, has it squared, and only
  that form has the closed-form enthalpy below.  Read squared.
* The gas constant is that of dry air, R = R_u / 28.9647 g/mol; c_p,inf = gamma_inf R /
  (gamma_inf - 1) with the configured gamma_inf, and Pr_inf = mu_inf c_p,inf / kappa_inf
  follows from the two laws at T_inf (the configured Pr is not used).
* Enthalpy and energy are zero at 0 K: integrating Eq. (23),
  h(T) = c_p0 [T + (gamma_inf - 1)/gamma_inf Theta / (e^(Theta/T) - 1)],  e = h - R T.
* Nondimensional form with the scales of Sec. 2.1 (T_ref = (gamma_inf - 1) T_inf,
  energies by c_inf^2 = c_p,inf T_ref, Ec = 1): with k0 = c_p0/c_p,inf, g = gamma_inf and
  th = Theta/T_ref,
  e(T) = k0 T + k0 (g - 1)/g th/(e^(th/T) - 1) - (g - 1)/g T,
  c_v(T) = k0 [1 + (g - 1)/g f(th/T)] - (g - 1)/g,  f(x) = x^2 e^x / (e^x - 1)^2.
* Energy inversion: Newton from the frozen-vibration bound T0 = e / (k0 - (g - 1)/g),
  which lies above the root (e(T) is convex and increasing), stopped at
  |dT| <= 1e-13 T or after 50 iterations, as for 5-species air; then one Newton step
  whose residual is evaluated in extended precision, so that the returned T is the root
  rounded to double (the right-hand side amplifies differences of a few units in the
  last place of T near the wall).
"""
import numpy as np

from . import species as sp

THETA = 3055.0          # K, Eq. (23)
KEYES_C2 = 2.646e-3     # W m^-1 K^-3/2, Eq. (25)
KEYES_C3 = 245.4        # K
KEYES_C4 = 12.0         # K
M_AIR = 28.9647e-3      # kg/mol (reading: dry air)
R_AIR = sp.R_U / M_AIR  # J/(kg K)


def keyes(T):
    """Dimensional equilibrium conductivity of air [W/(m K)], Eq. (25)."""
    T = np.asarray(T, dtype=np.float64)
    return KEYES_C2 * np.sqrt(T) / (1.0 + (KEYES_C3 / T) * 10.0 ** (-KEYES_C4 / T))


def vib_factor(x):
    """f(x) = x^2 e^x / (e^x - 1)^2, the harmonic oscillator's c_v / R at x = Theta/T,
    written with e^-x (= x^2 e^-x / (1 - e^-x)^2) so that large x gives 0, not inf/inf."""
    x = np.asarray(x, dtype=np.float64)
    em = np.expm1(-x)
    return x * x * (1.0 + em) / (em * em)


def cp_dimensional(T, gamma, T_inf):
    """c_p(T) [J/(kg K)] of Eq. (23) with c_p(T_inf) = c_p,inf."""
    cp_inf = gamma * R_AIR / (gamma - 1.0)
    a = (gamma - 1.0) / gamma
    cp0 = cp_inf / (1.0 + a * vib_factor(THETA / T_inf))
    return cp0 * (1.0 + a * vib_factor(THETA / np.asarray(T, dtype=np.float64)))


def constants(gamma, T_inf):
    """Nondimensional constants k0 = c_p0 / c_p,inf and th = Theta / T_ref."""
    a = (gamma - 1.0) / gamma
    k0 = 1.0 / (1.0 + a * vib_factor(THETA / T_inf))
    return dict(k0=float(k0), th=THETA / ((gamma - 1.0) * T_inf))


def energy(T, k0, th, gamma):
    """Nondimensional internal energy e(T) (module doc)."""
    T = np.asarray(T, dtype=np.float64)
    a = (gamma - 1.0) / gamma
    return k0 * T + k0 * a * th / np.expm1(th / T) - a * T


def cv(T, k0, th, gamma):
    """Nondimensional d e / d T."""
    a = (gamma - 1.0) / gamma
    return k0 * (1.0 + a * vib_factor(th / np.asarray(T, dtype=np.float64))) - a


def temperature(e, k0, th, gamma, rtol=1e-13, max_iter=50):
    """Newton inversion of e(T) (module doc); returns (T, iterations, converged)."""
    e = np.asarray(e, dtype=np.float64)
    a = (gamma - 1.0) / gamma
    T = e / (k0 - a)
    done = np.zeros(e.shape, dtype=bool)
    it = np.zeros(e.shape, dtype=np.int64)
    for _ in range(max_iter):
        dT = (energy(T, k0, th, gamma) - e) / cv(T, k0, th, gamma)
        T = np.where(done, T, T - dT)
        it = it + (~done)
        done = done | (np.abs(dT) <= rtol * np.abs(T))
        if done.all():
            break
    # refinement: residual e(T) - e in extended precision (80-bit long double)
    L = np.longdouble
    TL = T.astype(L)
    aL = L((gamma - 1.0) / gamma)
    res = L(k0) * TL + L(k0) * aL * L(th) / np.expm1(L(th) / TL) - aL * TL - e.astype(L)
    T = (TL - res / cv(T, k0, th, gamma).astype(L)).astype(np.float64)
    return T, it, done
