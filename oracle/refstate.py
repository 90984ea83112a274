"""Reference state and nondimensional numbers (oracle; test infrastructure only).

Sec. 2.1, Eqs. (7) and (11): density, velocity, pressure, energies scale with the
free-stream rho_inf and c_inf; temperature with T_ref = (gamma_inf - 1) T_inf;
viscosity and conductivity with their free-stream values; the production rate with
rho_inf c_inf / L_ref; Re = rho c L / mu, Pr = mu c_p / kappa, Ec = c^2/(c_p T_ref),
all at the free stream.  Ec = 1 by construction; this oracle uses Ec = 1 in the
equations and keeps the computed value only for a pin.

For 5-species air the free-stream gamma and c_p are the frozen values of the RRHO
model at (T_inf, Y_inf) and c_inf is the frozen sound speed.  The reference length
is either given or follows from a given Re.  Diffusion coefficients are scaled by
c_inf L_ref (reading: consistent with V_s / c_inf of Eq. 7).
"""
import math

import numpy as np

from . import species as sp
from . import thermo
from . import transport


def reference_cpg(gamma, Pr, mach, T_inf, Re):
    """Calorically perfect gas (Sec. 2.2.2): nondimensional constants only."""
    T_ref = (gamma - 1.0) * T_inf
    return dict(gas="cpg", gamma=gamma, Pr=Pr, Re=Re, Ec=1.0, mach=mach,
                T_inf=T_inf, T_ref=T_ref, T_inf_nd=1.0 / (gamma - 1.0),
                mu_inf=float(transport.sutherland(T_inf)))


def reference_tpg(gamma, mach, T_inf, Re):
    """Thermally perfect gas (Sec. 2.2.2, module tpg): nondimensional constants, with
    Pr = mu_inf c_p,inf / kappa_inf from Sutherland's and Keyes' laws at T_inf."""
    from . import tpg
    T_ref = (gamma - 1.0) * T_inf
    mu = float(transport.sutherland(T_inf))
    kap = float(tpg.keyes(T_inf))
    cp = gamma * tpg.R_AIR / (gamma - 1.0)
    out = dict(gas="tpg", gamma=gamma, Pr=mu * cp / kap, Re=Re, Ec=1.0, mach=mach,
               T_inf=T_inf, T_ref=T_ref, T_inf_nd=1.0 / (gamma - 1.0), mu_inf=mu,
               kappa_inf=kap, cp_inf=cp)
    out.update(tpg.constants(gamma, T_inf))
    return out


def reference_air5(p_inf, T_inf, Y_inf, mach, Re=None, L_ref=None):
    """5-species air free stream and scales; exactly one of Re, L_ref (> 0) is used."""
    Y = np.asarray(Y_inf, dtype=np.float64).reshape(5, 1)
    T = np.array([T_inf], dtype=np.float64)
    R = float(thermo.mixture_R(Y)[0])
    cv = float(thermo.mixture_cv(T, Y)[0])
    cp = cv + R
    gam = cp / cv
    rho = p_inf / (R * T_inf)
    c = math.sqrt(gam * R * T_inf)
    T_ref = (gam - 1.0) * T_inf
    mu, kap = transport.mixture_viscosity_conductivity(T, Y)
    mu = float(mu[0]); kap = float(kap[0])
    if L_ref is not None and L_ref > 0.0:
        Re = rho * c * L_ref / mu
    else:
        L_ref = Re * mu / (rho * c)
    Pr = mu * cp / kap
    Ec = c * c / (cp * T_ref)
    return dict(gas="air5", p_inf=p_inf, T_inf=T_inf, Y_inf=Y[:, 0].copy(), R_inf=R,
                cv_inf=cv, cp_inf=cp, gamma=gam, rho_inf=rho, c_inf=c, T_ref=T_ref,
                mu_inf=mu, kappa_inf=kap, Re=Re, L_ref=L_ref, Pr=Pr, Ec_computed=Ec, Ec=1.0,
                mach=mach, T_inf_nd=1.0 / (gam - 1.0))


def reference_from_config(cfg):
    """Reference state for a workload configuration (fields.FlowConfig)."""
    if cfg.gas == 0:
        return reference_cpg(cfg.gamma, cfg.Pr, cfg.mach, cfg.T_inf, cfg.Re)
    if cfg.gas == 2:
        return reference_tpg(cfg.gamma, cfg.mach, cfg.T_inf, cfg.Re)
    if cfg.L_ref > 0.0:
        return reference_air5(cfg.p_inf, cfg.T_inf, cfg.Y_inf, cfg.mach, L_ref=cfg.L_ref)
    return reference_air5(cfg.p_inf, cfg.T_inf, cfg.Y_inf, cfg.mach, Re=cfg.Re)
