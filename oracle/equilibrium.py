"""Chemical equilibrium of 5-species air in mpmath (oracle; test infrastructure only).

At fixed T and element densities, chemical equilibrium holds when every
independent reaction balances: for N2 = 2N, O2 = 2O and NO = N + O,
prod c^(nu'' - nu') = K_c(T), with K_c from the standard-state Gibbs energies
(Sec. 2.2.1, finite-rate chemistry paragraph; the backward rate is k_f / K_c).  This
module evaluates those Gibbs energies in 50-digit arithmetic from the species data
and solves the three balances plus the two element balances by Newton's method in
log-concentrations.  Any composition it returns must give zero net production
through the five-reaction mechanism (detailed balance), which pins the FP64
chemistry code to an independent evaluation.

Local thermodynamic equilibrium (Sec. 2.2.1, frozen and equilibrium flow): the
composition at a given temperature and density is the one that minimises the free
energy over all compositions with the mixture's elements.  At fixed T and volume the
function minimised is, per unit volume and in units of R_u T,
    f(c) = sum_s c_s [g_s/(R_u T) + ln(c_s R_u T / p0) - 1]
(ideal-gas species at their partial pressures; the minimum over the same elements at
fixed T and p gives the same state).  Its stationary point under the element balances
sum_s a_es c_s = n_e is c_s = (p0/(R_u T)) exp(-g_s/(R_u T) + sum_e a_es lambda_e) with
the element potentials lambda_e: for the atoms c_N = c0 e^{lambda_N - g_N}, and every
molecule follows from them, c_N2 = c_N^2 / K_1 and so on -- exactly the balances
solve() takes, with the element potentials carried as ln c_N, ln c_O.
"""
import mpmath as mp

from . import species as sp

mp.mp.dps = 50


def g_over_RT(T):
    T = mp.mpf(T)
    kB, h, NA = mp.mpf(sp.K_B), mp.mpf(sp.H_PLANCK), mp.mpf(sp.N_A)
    RU = kB * NA
    out = []
    for s in range(5):
        m = mp.mpf(sp.M[s]) / NA
        qt = (2 * mp.pi * m * kB * T / h ** 2) ** mp.mpf(1.5) * kB * T / mp.mpf(sp.P_STD)
        g = mp.mpf(sp.HF0[s]) / (RU * T) - mp.log(qt) - mp.log(mp.mpf(sp.G_EL[s]))
        if sp.DIATOMIC[s] > 0:
            g -= mp.log(T / (mp.mpf(sp.SIGMA_SYM[s]) * mp.mpf(sp.THETA_R[s])))
            g += mp.log(1 - mp.exp(-mp.mpf(sp.THETA_V[s]) / T))
        out.append(g)
    return out


def Kc(T, dnu):
    g = g_over_RT(T)
    RU = mp.mpf(sp.K_B) * mp.mpf(sp.N_A)
    dG = sum(mp.mpf(d) * gi for d, gi in zip(dnu, g))
    return (mp.mpf(sp.P_STD) / (RU * mp.mpf(T))) ** sum(dnu) * mp.exp(-dG)


def solve(T, nN, nO):
    """Equilibrium concentrations [mol/m^3] (N2, O2, NO, N, O) for element moles nN, nO per m^3."""
    K1 = Kc(T, [-1, 0, 0, 2, 0])
    K2 = Kc(T, [0, -1, 0, 0, 2])
    K3 = Kc(T, [0, 0, -1, 1, 1])
    nN, nO = mp.mpf(nN), mp.mpf(nO)

    def conc(lN, lO):
        cN, cO = mp.exp(lN), mp.exp(lO)
        return [cN * cN / K1, cO * cO / K2, cN * cO / K3, cN, cO]

    def F(lN, lO):
        c = conc(lN, lO)
        return [(2 * c[0] + c[2] + c[3]) / nN - 1, (2 * c[1] + c[2] + c[4]) / nO - 1]

    # start from the atom-rich or molecule-rich limit, whichever is closer
    x0 = [mp.log(min(nN, mp.sqrt(K1 * nN / 2))), mp.log(min(nO, mp.sqrt(K2 * nO / 2)))]
    sol = mp.findroot(F, x0, tol=mp.mpf(10) ** -40, maxsteps=200)
    return conc(sol[0], sol[1])


M_N_ATOM = sp.M[3]
M_O_ATOM = sp.M[4]


def free_energy(T, c):
    """f(c) of the module doc (per unit volume, units of R_u T), mpmath."""
    g = g_over_RT(T)
    RU = mp.mpf(sp.K_B) * mp.mpf(sp.N_A)
    out = mp.mpf(0)
    for s, cs in enumerate(c):
        cs = mp.mpf(cs)
        if cs > 0:
            out += cs * (g[s] + mp.log(cs * RU * mp.mpf(T) / mp.mpf(sp.P_STD)) - 1)
    return out


def _single_element(T, n, dnu_molecule):
    """One element only: atoms c and molecules c^2/K with 2 c^2/K + c = n."""
    K = Kc(T, dnu_molecule)
    c = 2 * n / (1 + mp.sqrt(1 + 8 * n / K))
    return c, c * c / K


def composition(rho, T, xiN):
    """LTE mass fractions Y [5][n] and status [n] at densities rho [kg/m^3], temperatures
    T [K] and element-N mass fractions xiN (arrays of n points, mpmath per point).
    Status 0, or 3 where an input is not finite, rho <= 0, T <= 0 or xiN is outside
    [0, 1] (then Y is NaN)."""
    import numpy as np
    rho = np.atleast_1d(np.asarray(rho, dtype=np.float64))
    T = np.atleast_1d(np.asarray(T, dtype=np.float64))
    xiN = np.atleast_1d(np.asarray(xiN, dtype=np.float64))
    n = len(rho)
    Y = np.full((5, n), np.nan)
    st = np.zeros(n, dtype=np.int64)
    for p in range(n):
        r, t, x = rho[p], T[p], xiN[p]
        if not (np.isfinite(r) and np.isfinite(t) and np.isfinite(x) and r > 0 and t > 0
                and 0.0 <= x <= 1.0):
            st[p] = 3
            continue
        nN = mp.mpf(r) * mp.mpf(x) / mp.mpf(M_N_ATOM)
        nO = mp.mpf(r) * (1 - mp.mpf(x)) / mp.mpf(M_O_ATOM)
        if nO == 0:
            cN, cN2 = _single_element(t, nN, [-1, 0, 0, 2, 0])
            c = [cN2, 0, 0, cN, 0]
        elif nN == 0:
            cO, cO2 = _single_element(t, nO, [0, -1, 0, 0, 2])
            c = [0, cO2, 0, 0, cO]
        else:
            c = solve(t, nN, nO)
        for s in range(5):
            Y[s, p] = float(c[s] * mp.mpf(sp.M[s]) / mp.mpf(r))
    return Y, st
