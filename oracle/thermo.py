"""Species and mixture thermodynamics (oracle; test infrastructure only).

Single-temperature rigid-rotor / harmonic-oscillator (RRHO) model for 5-species air.
The paper states that species properties come from statistical mechanics
(Sec. 2.2.1) and that each state evaluation involves the iterative solution of
nonlinear equations (Sec. 3.4); it prints neither.  Reading taken here:

    e_s(T) = R_s [(3/2 + r_s) T + v_s theta_s / (exp(theta_s/T) - 1)] + h0_s / M_s
    h_s    = e_s + R_s T
    g_s/(R_u T) = h0_s/(R_u T) - ln[(2 pi m_s k T / h^2)^(3/2) k T / p0]
                  - r_s ln(T / (sigma_s theta_r,s)) + v_s ln(1 - exp(-theta_s/T)) - ln g_el,s

with r_s = v_s = 1 for the diatomics and 0 for the atoms.  Mixture sums follow
Eq. (12); the energy -> temperature inversion is Newton's method from the lower
bound obtained with fully excited vibration.
"""
import numpy as np

from . import species as sp


def R_s():
    """Specific gas constants R_u / M_s [J/(kg K)]."""
    return sp.R_U / sp.M


def e_species(T):
    """Species internal energy per unit mass e_s(T) [J/kg], shape (5,)+T.shape."""
    T = np.asarray(T, dtype=np.float64)
    Rs = R_s()[:, None]
    th = sp.THETA_V[:, None]
    r = sp.DIATOMIC[:, None]
    Tf = T.reshape(1, -1)
    with np.errstate(over="ignore", divide="ignore", invalid="ignore"):
        evib = np.where(th > 0, th / np.expm1(th / Tf), 0.0)
    e = Rs * ((1.5 + r) * Tf + r * evib) + (sp.HF0 / sp.M)[:, None]
    return e.reshape((5,) + T.shape)


def h_species(T):
    """Species enthalpy per unit mass h_s = e_s + R_s T [J/kg]."""
    T = np.asarray(T, dtype=np.float64)
    return e_species(T) + R_s().reshape((5,) + (1,) * T.ndim) * T


def cv_species(T):
    """Species heat capacity at constant volume de_s/dT [J/(kg K)]."""
    T = np.asarray(T, dtype=np.float64)
    Rs = R_s()[:, None]
    th = sp.THETA_V[:, None]
    r = sp.DIATOMIC[:, None]
    Tf = T.reshape(1, -1)
    with np.errstate(over="ignore", divide="ignore", invalid="ignore"):
        x = th / Tf
        ex = np.exp(x)
        cvib = np.where(th > 0, x * x * ex / (ex - 1.0) ** 2, 0.0)
        cvib = np.where(np.isfinite(cvib), cvib, 0.0)
    cv = Rs * (1.5 + r + r * cvib)
    return cv.reshape((5,) + T.shape)


def gibbs_molar_over_RT(T):
    """Standard-state molar Gibbs energy g_s/(R_u T) at p0 = 1e5 Pa, shape (5,)+T.shape."""
    T = np.asarray(T, dtype=np.float64)
    Tf = T.reshape(1, -1)
    m = (sp.M / sp.N_A)[:, None]
    qtr = (2.0 * np.pi * m * sp.K_B * Tf / sp.H_PLANCK ** 2) ** 1.5 * sp.K_B * Tf / sp.P_STD
    g = sp.HF0[:, None] / (sp.R_U * Tf) - np.log(qtr) - np.log(sp.G_EL)[:, None]
    r = sp.DIATOMIC[:, None]
    with np.errstate(divide="ignore", invalid="ignore"):
        rot = np.where(r > 0, np.log(Tf / (sp.SIGMA_SYM[:, None] * np.where(r > 0, sp.THETA_R[:, None], 1.0))), 0.0)
        vib = np.where(r > 0, np.log(-np.expm1(-sp.THETA_V[:, None] / Tf)), 0.0)
    g = g - r * rot + r * vib
    return g.reshape((5,) + T.shape)


def mixture_e(T, Y):
    """Mixture internal energy e = sum_s Y_s e_s(T), Eq. (12)."""
    return np.sum(np.asarray(Y) * e_species(T), axis=0)


def mixture_cv(T, Y):
    """Frozen mixture c_v = sum_s Y_s c_v,s(T)."""
    return np.sum(np.asarray(Y) * cv_species(T), axis=0)


def mixture_R(Y):
    """Mixture gas constant sum_s Y_s R_s."""
    Y = np.asarray(Y)
    return np.sum(Y * R_s().reshape((5,) + (1,) * (Y.ndim - 1)), axis=0)


def temperature_from_energy(e, Y, T_min=50.0, rtol=1e-13, max_iter=50):
    """Invert e = sum_s Y_s e_s(T) for T [K] (Sec. 3.4: iterative solution per point).

    Start: the temperature at which the energy with fully excited vibration (an upper
    bound of e_s(T), since e_vib <= R_s T) equals e; that start is a lower bound of
    the root.  e(T) is increasing and convex (c_v rises with T), so Newton's method
    T <- T - (e(T) - e)/c_v(T) converges monotonically after its first step.
    Stops when |dT| <= rtol*T.  Returns (T, iterations, status) with status
    0 = converged, 1 = not converged in max_iter, 2 = e below e(T_min).
    """
    e = np.asarray(e, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    shp = e.shape
    e1 = e.reshape(-1)
    Y1 = Y.reshape(5, -1)
    Rs = R_s()[:, None]
    ef = np.sum(Y1 * (sp.HF0 / sp.M)[:, None], axis=0)
    cfull = np.sum(Y1 * Rs * (1.5 + 2.0 * sp.DIATOMIC[:, None]), axis=0)
    T = (e1 - ef) / cfull
    emin = np.sum(Y1 * e_species(np.full(e1.shape, T_min)), axis=0)
    status = np.where(e1 < emin, 2, 0)
    T = np.where(T < T_min, T_min, T)
    T = np.where(status == 2, T_min, T)
    iters = np.zeros(e1.shape, dtype=np.int64)
    active = status == 0
    for _ in range(max_iter):
        if not active.any():
            break
        Ta = T[active]
        Ya = Y1[:, active]
        f = np.sum(Ya * e_species(Ta), axis=0) - e1[active]
        cv = np.sum(Ya * cv_species(Ta), axis=0)
        dT = f / cv
        Tn = Ta - dT
        T[active] = Tn
        iters[active] += 1
        done = np.abs(dT) <= rtol * Tn
        idx = np.flatnonzero(active)
        active[idx[done]] = False
    status = np.where(active, 1, status)
    return T.reshape(shp), iters.reshape(shp), status.reshape(shp)


def frozen_gamma(T, Y):
    """Frozen ratio of specific heats (c_v + R_mix)/c_v."""
    cv = mixture_cv(T, Y)
    return (cv + mixture_R(Y)) / cv


# ---------------------------------------------------------------- calorically perfect gas
def cpg_temperature(e_nd, gamma):
    """Nondimensional CPG temperature from nondimensional internal energy: gamma e = T (Sec. 2.2.2)."""
    return gamma * np.asarray(e_nd)


def cpg_pressure(rho, T, gamma, Ec=1.0):
    """Nondimensional equation of state p = rho (gamma-1) T / (gamma Ec), Eq. (22)."""
    return rho * (gamma - 1.0) * T / (gamma * Ec)
