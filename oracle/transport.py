"""Transport properties (oracle; test infrastructure only).

Calorically/thermally perfect gas: Sutherland's law, Eq. (24), with the printed
C1 = 1.458e-6 kg/(m s K^1/2) and T_S = 110.4 K.

5-species air: the paper takes mixture viscosity, frozen conductivity and diffusion
coefficients from its thermochemical library (Sec. 2.2.1) without formulas.  Reading
taken here: first Chapman-Enskog approximation with Lennard-Jones 12-6 collision
integrals in the Neufeld-Janzen-Aziz (1972) fits, Eucken conductivities, Wilke's
mixing rule for viscosity and conductivity, and the averaged diffusion coefficient
of Eq. (19) built from the binary coefficients.
"""
import numpy as np

from . import species as sp
from . import thermo


def sutherland(T):
    """Dimensional viscosity mu(T) = C1 T^(3/2)/(T + T_S) [Pa s], Eq. (24)."""
    T = np.asarray(T, dtype=np.float64)
    return sp.SUTH_C1 * T ** 1.5 / (T + sp.SUTH_TS)


def omega11(Ts):
    """Reduced collision integral Omega^(1,1)* (Neufeld et al. 1972)."""
    return (1.06036 / Ts ** 0.15610 + 0.19300 / np.exp(0.47635 * Ts)
            + 1.03587 / np.exp(1.52996 * Ts) + 1.76474 / np.exp(3.89411 * Ts))


def omega22(Ts):
    """Reduced collision integral Omega^(2,2)* (Neufeld et al. 1972)."""
    return (1.16145 / Ts ** 0.14874 + 0.52487 / np.exp(0.77320 * Ts)
            + 2.16178 / np.exp(2.43787 * Ts))


def species_viscosity(T):
    """mu_s = (5/16) sqrt(pi m_s k T) / (pi sigma_s^2 Omega22*(T/eps_s)) [Pa s], shape (5,)+T.shape."""
    T = np.asarray(T, dtype=np.float64)
    sh = (5,) + (1,) * T.ndim
    m = (sp.M / sp.N_A).reshape(sh)
    sig = sp.LJ_SIGMA.reshape(sh)
    eps = sp.LJ_EPS.reshape(sh)
    return (5.0 / 16.0) * np.sqrt(np.pi * m * sp.K_B * T) / (np.pi * sig ** 2 * omega22(T / eps))


def binary_diffusion(T, p):
    """Binary coefficients D_sr(T, p) [m^2/s], shape (5,5)+T.shape.

    D_sr = (3/16) sqrt(2 pi k^3 T^3 / m_sr) / (p pi sigma_sr^2 Omega11*(T/eps_sr)),
    m_sr reduced mass, sigma_sr = (sigma_s+sigma_r)/2, eps_sr = sqrt(eps_s eps_r).
    """
    T = np.asarray(T, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64)
    out = np.empty((5, 5) + T.shape)
    m = sp.M / sp.N_A
    for s in range(5):
        for r in range(5):
            msr = m[s] * m[r] / (m[s] + m[r])
            sig = 0.5 * (sp.LJ_SIGMA[s] + sp.LJ_SIGMA[r])
            eps = np.sqrt(sp.LJ_EPS[s] * sp.LJ_EPS[r])
            out[s, r] = (3.0 / 16.0) * np.sqrt(2.0 * np.pi * sp.K_B ** 3 * T ** 3 / msr) / (
                p * np.pi * sig ** 2 * omega11(T / eps))
    return out


def species_conductivity(T):
    """Eucken: kappa_s = mu_s (15/4 R_s + c_v,int,s) with c_v,int = rotational + vibrational."""
    T = np.asarray(T, dtype=np.float64)
    sh = (5,) + (1,) * T.ndim
    Rs = thermo.R_s().reshape(sh)
    cv = thermo.cv_species(T)
    cv_int = cv - 1.5 * Rs
    return species_viscosity(T) * (3.75 * Rs + cv_int)


def mole_fractions(Y):
    """X_s = (Y_s/M_s) / sum_r (Y_r/M_r)."""
    Y = np.asarray(Y, dtype=np.float64)
    sh = (5,) + (1,) * (Y.ndim - 1)
    n = Y / sp.M.reshape(sh)
    return n / np.sum(n, axis=0)


def wilke_phi(mu_s):
    """Wilke interaction factors phi_sr = [1 + sqrt(mu_s/mu_r)(M_r/M_s)^(1/4)]^2 / sqrt(8 (1 + M_s/M_r))."""
    out = np.empty((5, 5) + mu_s.shape[1:])
    for s in range(5):
        for r in range(5):
            out[s, r] = (1.0 + np.sqrt(mu_s[s] / mu_s[r]) * (sp.M[r] / sp.M[s]) ** 0.25) ** 2 / np.sqrt(
                8.0 * (1.0 + sp.M[s] / sp.M[r]))
    return out


def mixture_viscosity_conductivity(T, Y):
    """Wilke mixture viscosity and frozen conductivity (the conductivity of Sec. 2.2.1's heat flux)."""
    X = mole_fractions(Y)
    mu_s = species_viscosity(T)
    k_s = species_conductivity(T)
    phi = wilke_phi(mu_s)
    den = np.einsum("r...,sr...->s...", X, phi)
    mu = np.sum(X * mu_s / den, axis=0)
    kap = np.sum(X * k_s / den, axis=0)
    return mu, kap


X_CLIP = 1e-12


def averaged_diffusion(T, p, Y):
    """Averaged coefficients D_s = (1 - X_s) / sum_{r != s} X_r / D_sr, Eq. (19).

    Reading: 1 - X_s is formed as sum_{r != s} X_r (equal when sum X = 1), and in this
    formula only every X_r is clipped below at 1e-12 so that a pure species gets the
    finite limit instead of 0/0.
    """
    X = np.maximum(mole_fractions(Y), X_CLIP)
    Dsr = binary_diffusion(T, p)
    out = np.empty_like(X)
    for s in range(5):
        num = 0.0
        den = 0.0
        for r in range(5):
            if r == s:
                continue
            num = num + X[r]
            den = den + X[r] / Dsr[s, r]
        out[s] = num / den
    return out


def air5_properties(rho, T, Y):
    """SI transport state at (rho, T, Y): returns p, mu, kappa, D_s."""
    p = rho * thermo.mixture_R(Y) * T
    mu, kap = mixture_viscosity_conductivity(T, Y)
    D = averaged_diffusion(T, p, Y)
    return p, mu, kap, D


def stefan_maxwell_fluxes(rho, Y, gradX, Dsr):
    """Stefan-Maxwell diffusion mass fluxes J_s (Eq. 17 with the driving forces of Eq. 16,
    closed by the mass constraint of Eq. 20), in any consistent units: rho, Y [5][...],
    gradX [5][nd][...], Dsr [5][5][...] (e.g. binary_diffusion(T, p)) -> J [5][nd][...].

    The relations grad X_s = sum_{i != s} (X_s X_i / D_si) (V_i - V_s) are written for the
    molar fluxes j_s = J_s / M_s = rho Y_s V_s / M_s (so that X_i V_i = (Mbar / rho) j_i):
        sum_{i != s} (X_s j_i - X_i j_s) / D_si = (rho / Mbar) grad X_s,
    i.e. C j = (rho / Mbar) grad X with C_si = X_s / D_si (i != s) and
    C_ss = -sum_{i != s} X_i / D_si.  Every column of C sums to zero, so the five
    relations hold four independent conditions; the mass constraint sum_s M_s j_s = 0
    (Eq. 20) is the fifth.  It is added to every row, (C + alpha 1 m^T) j = (rho/Mbar)
    grad X with m_s = M_s / Mbar and alpha the mean |C_ss|: the added term vanishes on
    the solution, and the matrix is regular whenever C has rank four (summing its rows
    gives 5 alpha m.j = sum_s (rho/Mbar) grad X_s, which is zero when sum_s X_s = 1).
    The mole fractions enter as they are: no entry holds 1/X_s; the row of an absent
    species (X_s = 0) reduces to j_s = -(rho / Mbar) grad X_s / sum_{i != s} X_i / D_si;
    negative values (undershoots of a discrete field) are used unchanged.  Solved per point with LAPACK (partial pivoting).
    """
    Y = np.asarray(Y, dtype=np.float64)
    X = mole_fractions(Y)
    sh = (5,) + (1,) * (Y.ndim - 1)
    Mbar = 1.0 / np.sum(Y / sp.M.reshape(sh), axis=0)
    rest = Y.shape[1:]
    n = int(np.prod(rest)) if rest else 1
    Xf = X.reshape(5, n)
    Df = np.asarray(Dsr, dtype=np.float64).reshape(5, 5, n)
    nd = gradX.shape[1]
    C = np.zeros((n, 5, 5))
    for s in range(5):
        for i in range(5):
            if i == s:
                continue
            C[:, s, i] = Xf[s] / Df[s, i]
            C[:, s, s] -= Xf[i] / Df[s, i]
    m = (sp.M.reshape(5, 1) / Mbar.reshape(1, n)).T          # [n][5]
    alpha = np.mean(np.abs(np.diagonal(C, axis1=1, axis2=2)), axis=1)
    A = C + alpha[:, None, None] * m[:, None, :]              # + alpha 1 m^T
    b = (np.asarray(rho, dtype=np.float64).reshape(n) / Mbar.reshape(n))[:, None, None] * \
        np.moveaxis(np.asarray(gradX, dtype=np.float64).reshape(5, nd, n), 2, 0)
    j = np.linalg.solve(A, b)                                 # [n][5][nd]
    J = sp.M.reshape(1, 5, 1) * j
    return np.moveaxis(J, 0, 2).reshape((5, nd) + rest)
