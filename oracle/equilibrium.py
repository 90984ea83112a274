"""Law-of-mass-action equilibrium of 5-species air in mpmath (oracle pin only).

At fixed T and element densities, chemical equilibrium holds when every
independent reaction balances: for N2 = 2N, O2 = 2O and NO = N + O,
prod c^(nu'' - nu') = K_c(T), with K_c from the standard-state Gibbs energies
(Sec. 2.2.1, finite-rate chemistry paragraph; the backward rate is k_f / K_c).  This
module evaluates those Gibbs energies in 50-digit arithmetic from the species data
and solves the three balances plus the two element balances by Newton's method in
log-concentrations.  Any composition it returns must give zero net production
through the five-reaction mechanism (detailed balance), which pins the FP64
chemistry code to an independent evaluation.
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
