"""Finite-rate chemistry (oracle; test infrastructure only), Sec. 2.2.1, Eqs. (13)-(15).

    k_f,r = C_r T^n_r exp(-theta_r / T)
    k_b,r = k_f,r / K_c,r(T)
    R_r   = [k_f,r prod_s c_s^nu'_rs - k_b,r prod_s c_s^nu''_rs] * sum_s Z_rs c_s
    wdot_s = M_s sum_r (nu''_rs - nu'_rs) R_r,          c_s = rho_s / M_s

Readings: the exponent of the printed Arrhenius law carries no minus sign; it is read
as exp(-theta/T) with theta > 0 (an activation temperature).  The backward product is
read over species s.  The third-body sum multiplies only reactions that have a third
body (for the others the factor is 1).  K_c comes from the standard-state Gibbs
energies of the thermodynamic model:
    K_c = (p0 / (R_u T))^dnu exp(-sum_s (nu'' - nu')_s g_s / (R_u T)).
"""
import numpy as np

from . import species as sp
from . import thermo


def _nu(r):
    return np.array(r["nu_f"], float), np.array(r["nu_b"], float)


def equilibrium_constant(T, nu_f, nu_b):
    """K_c in (mol/m^3)^dnu."""
    g = thermo.gibbs_molar_over_RT(T)
    dnu = np.asarray(nu_b, float) - np.asarray(nu_f, float)
    dG = np.tensordot(dnu, g, axes=(0, 0))
    return (sp.P_STD / (sp.R_U * np.asarray(T))) ** dnu.sum() * np.exp(-dG)


def rates_of_progress(rho_s, T):
    """R_r [mol/(m^3 s)] for the 5 reactions of the third-body mechanism, shape (5,)+T.shape."""
    rho_s = np.asarray(rho_s, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    c = rho_s / sp.M.reshape((5,) + (1,) * T.ndim)
    out = []
    for r in sp.REACTIONS:
        nf, nb = _nu(r)
        kf = r["C"] * 1e-6 * T ** r["n"] * np.exp(-r["theta"] / T)
        kb = kf / equilibrium_constant(T, nf, nb)
        fwd = kf * np.prod([c[s] ** nf[s] for s in range(5)], axis=0)
        bwd = kb * np.prod([c[s] ** nb[s] for s in range(5)], axis=0)
        tb = 1.0
        if r["Z"] is not None:
            tb = np.sum([r["Z"][s] * c[s] for s in range(5)], axis=0)
        out.append((fwd - bwd) * tb)
    return np.array(out)


def production_rates(rho_s, T):
    """Net mass production wdot_s [kg/(m^3 s)], Eq. (15)."""
    R = rates_of_progress(rho_s, T)
    w = np.zeros_like(np.asarray(rho_s, dtype=np.float64))
    for ir, r in enumerate(sp.REACTIONS):
        nf, nb = _nu(r)
        for s in range(5):
            d = nb[s] - nf[s]
            if d != 0.0:
                w[s] = w[s] + sp.M[s] * d * R[ir]
    return w


def production_rates_explicit17(rho_s, T):
    """Same production rates summed over the 17 partner-explicit reactions (pin only)."""
    rho_s = np.asarray(rho_s, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    c = rho_s / sp.M.reshape((5,) + (1,) * T.ndim)
    w = np.zeros_like(rho_s)
    for nf, nb, C, n, th in sp.EXPLICIT_17:
        nf = np.array(nf, float); nb = np.array(nb, float)
        kf = C * 1e-6 * T ** n * np.exp(-th / T)
        # the partner appears on both sides: K_c of the reaction without it
        kb = kf / equilibrium_constant(T, nf, nb)
        R = kf * np.prod([c[s] ** nf[s] for s in range(5)], axis=0) - kb * np.prod(
            [c[s] ** nb[s] for s in range(5)], axis=0)
        for s in range(5):
            if nb[s] != nf[s]:
                w[s] = w[s] + sp.M[s] * (nb[s] - nf[s]) * R
    return w


def gross_magnitude(rho_s, T):
    """M_max * sum_r (|forward term| + |backward term|) * |third-body factor|: the
    gross rate scale against which cancellation in wdot is judged."""
    rho_s = np.asarray(rho_s, dtype=np.float64)
    T = np.asarray(T, dtype=np.float64)
    c = rho_s / sp.M.reshape((5,) + (1,) * T.ndim)
    tot = np.zeros(T.shape)
    for r in sp.REACTIONS:
        nf, nb = _nu(r)
        kf = r["C"] * 1e-6 * T ** r["n"] * np.exp(-r["theta"] / T)
        kb = kf / equilibrium_constant(T, nf, nb)
        fwd = kf * np.prod([c[s] ** nf[s] for s in range(5)], axis=0)
        bwd = kb * np.prod([c[s] ** nb[s] for s in range(5)], axis=0)
        tb = 1.0
        if r["Z"] is not None:
            tb = np.sum([r["Z"][s] * c[s] for s in range(5)], axis=0)
        tot = tot + (np.abs(fwd) + np.abs(bwd)) * np.abs(tb) * np.max(sp.M)
    return tot
