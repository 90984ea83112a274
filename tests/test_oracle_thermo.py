"""Pins of the oracle's thermodynamics, transport and chemistry (Sec. 2.2).

Printed values: Sutherland constants (Eq. 24), the CPG relations (Sec. 2.2.2,
Eq. 22), Ec = 1 (Sec. 2.1).  Mathematical identities: Gibbs-Helmholtz linking the
Gibbs energies (used by K_c) to the enthalpies (used by the energy equation),
c_v = de/dT and its classical limits, Newton round trips against 50-digit
bisection, pure-species and binary limits of the mixing rules, sum of production
rates, element conservation, the partner-explicit 17-reaction sum, and zero net
production at an independently computed (mpmath) equilibrium composition.
"""
import mpmath as mp
import numpy as np
import pytest

from oracle import chemistry as ch
from oracle import equilibrium as eqm
from oracle import refstate as rs
from oracle import species as sp
from oracle import thermo as th
from oracle import transport as tr


def test_sutherland_printed_constants():
    # Eq. (24) with C1 = 1.458e-6, T_S = 110.4 K
    for T, mu in [(220.0, 1.458e-6 * 220.0 ** 1.5 / 330.4), (350.0, 1.458e-6 * 350.0 ** 1.5 / 460.4)]:
        assert abs(tr.sutherland(T) - mu) <= 1e-15 * mu
    assert abs(tr.sutherland(220.0) - 1.4399637e-5) < 1e-11
    assert abs(tr.sutherland(350.0) - 2.0735966e-5) < 1e-11


def test_cpg_relations_and_ec():
    ref = rs.reference_cpg(1.4, 0.72, 6.0, 220.0, 1e5)
    e = np.linspace(0.5, 5.0, 7)
    T = th.cpg_temperature(e, 1.4)
    assert np.all(T == 1.4 * e)
    p = th.cpg_pressure(2.0, T, 1.4)
    assert np.allclose(p, 2.0 * 0.4 * T / 1.4, rtol=1e-15, atol=0)
    # free stream: T_inf = 1/(gamma - 1), p_inf = 1/gamma (rho = 1)
    assert abs(th.cpg_pressure(1.0, ref["T_inf_nd"], 1.4) - 1 / 1.4) < 1e-15
    for p_inf, T_inf in [(3596.0, 350.0), (60967.0, 1110.5), (49800.0, 947.0)]:
        r = rs.reference_air5(p_inf, T_inf, [0.767082, 0.232918, 0, 0, 0], 8.0, Re=1e5)
        assert abs(r["Ec_computed"] - 1.0) <= 4 * np.finfo(float).eps
        assert abs(r["rho_inf"] * r["c_inf"] * r["L_ref"] / r["mu_inf"] - 1e5) < 1e-9 * 1e5


def test_gibbs_helmholtz_links_gibbs_and_enthalpy():
    """H = -T^2 d(G/T)/dT: molar h_s M_s = -R_u T^2 d(g_s/(R_u T))/dT (finite difference)."""
    for T in [300.0, 1000.0, 3000.0, 8000.0, 15000.0]:
        dT = 1e-3 * T
        gp = th.gibbs_molar_over_RT(np.array([T + dT]))[:, 0]
        gm = th.gibbs_molar_over_RT(np.array([T - dT]))[:, 0]
        dg = (gp - gm) / (2 * dT)
        h_from_g = -sp.R_U * T * T * dg
        h = th.h_species(np.array([T]))[:, 0] * sp.M
        assert np.allclose(h_from_g, h, rtol=2e-6, atol=1e-3 * sp.R_U * T), (T, h_from_g, h)


def test_cv_is_derivative_and_limits():
    for T in [250.0, 2000.0, 9000.0]:
        dT = 1e-4 * T
        num = (th.e_species(np.array([T + dT])) - th.e_species(np.array([T - dT])))[:, 0] / (2 * dT)
        assert np.allclose(num, th.cv_species(np.array([T]))[:, 0], rtol=1e-8)
    Rs = th.R_s()
    lo = th.cv_species(np.array([30.0]))[:, 0] / Rs
    hi = th.cv_species(np.array([1e6]))[:, 0] / Rs
    assert np.allclose(lo, [2.5, 2.5, 2.5, 1.5, 1.5], atol=1e-12)
    assert np.allclose(hi, [3.5, 3.5, 3.5, 1.5, 1.5], atol=1e-6)


def test_newton_round_trip_and_bisection():
    rng = np.random.default_rng(3)
    T = rng.uniform(200.0, 20000.0, 4000)
    Y = rng.dirichlet(np.ones(5), 4000).T
    e = th.mixture_e(T, Y)
    T2, it, status = th.temperature_from_energy(e, Y)
    assert np.all(status == 0)
    assert np.max(np.abs(T2 - T) / T) <= 1e-13
    assert it.max() <= 12
    # 50-digit bisection of the same energy equation on a few states
    mp.mp.dps = 50
    for k in range(5):
        Yk = [mp.mpf(float(v)) for v in Y[:, k]]
        ek = mp.mpf(float(e[k]))

        def emix(Tm):
            acc = mp.mpf(0)
            for s in range(5):
                Rs = mp.mpf(sp.R_U) / mp.mpf(sp.M[s])
                es = Rs * (mp.mpf(1.5) + sp.DIATOMIC[s]) * Tm + mp.mpf(sp.HF0[s]) / mp.mpf(sp.M[s])
                if sp.DIATOMIC[s]:
                    tv = mp.mpf(sp.THETA_V[s])
                    es += Rs * tv / (mp.exp(tv / Tm) - 1)
                acc += Yk[s] * es
            return acc
        a, b = mp.mpf(50), mp.mpf(50000)
        for _ in range(200):
            mid = (a + b) / 2
            if emix(mid) < ek:
                a = mid
            else:
                b = mid
        assert abs(float(a) - T2[k]) <= 2e-15 * T2[k] * 10
    # below the energy at T_min the status says so
    Tl, _, st_ = th.temperature_from_energy(th.mixture_e(np.array([40.0]), Y[:, :1]), Y[:, :1])
    assert st_[0] == 2


def test_transport_limits():
    T = np.array([300.0, 1500.0, 6000.0])
    mu_s = tr.species_viscosity(T)
    for s in range(5):
        Y = np.zeros((5, 3)); Y[s] = 1.0
        mu, kap = tr.mixture_viscosity_conductivity(T, Y)
        assert np.allclose(mu, mu_s[s], rtol=1e-14)
        assert np.allclose(kap, tr.species_conductivity(T)[s], rtol=1e-14)
    # binary mixture: averaged coefficient of Eq. (19) equals the binary one
    Y = np.zeros((5, 3)); Y[0] = 0.6; Y[4] = 0.4
    Y2 = Y.copy()
    D = tr.averaged_diffusion(T, 1e4, Y2)
    Dsr = tr.binary_diffusion(T, 1e4)
    assert np.allclose(D[0], Dsr[0, 4], rtol=1e-9)
    assert np.allclose(D[4], Dsr[4, 0], rtol=1e-9)
    # collision-integral fits against the Lennard-Jones tables at T* = 1 (Hirschfelder et al.)
    assert abs(tr.omega11(1.0) - 1.439) < 0.005
    assert abs(tr.omega22(1.0) - 1.587) < 0.008
    # plausibility of the model against handbook nitrogen viscosity near 300 K (1.78e-5 Pa s)
    assert abs(mu_s[0, 0] - 1.78e-5) / 1.78e-5 < 0.02


def _states(n=500, seed=5):
    rng = np.random.default_rng(seed)
    T = rng.uniform(1500.0, 9000.0, n)
    rho = 10 ** rng.uniform(-3, 0, n)
    Y = rng.dirichlet(np.ones(5), n).T
    return rho[None] * Y, T


def test_production_invariants():
    rhos, T = _states()
    w = ch.production_rates(rhos, T)
    scale = ch.gross_magnitude(rhos, T)
    assert np.max(np.abs(w.sum(axis=0)) / scale) < 1e-13
    elem = (w / sp.M[:, None]).T @ sp.ELEMENTS
    assert np.max(np.abs(elem) / (scale / sp.M.min())[:, None]) < 1e-13
    w17 = ch.production_rates_explicit17(rhos, T)
    assert np.max(np.abs(w17 - w) / scale) < 1e-12
    # Arrhenius read with exp(-theta/T): dissociation speeds up with temperature
    r1 = ch.rates_of_progress(np.array([[0.1], [0.0], [0.0], [0.0], [0.0]]), np.array([3000.0]))
    r2 = ch.rates_of_progress(np.array([[0.1], [0.0], [0.0], [0.0], [0.0]]), np.array([6000.0]))
    assert 0 < r1[0, 0] < r2[0, 0]


@pytest.mark.parametrize("T", [2500.0, 4500.0, 7000.0])
def test_zero_production_at_equilibrium(T):
    rho = 0.02
    nN = rho * 0.767082 / sp.M[0] * 2
    nO = rho * 0.232918 / sp.M[1] * 2
    c = eqm.solve(T, nN, nO)
    rhos = np.array([float(v) for v in c]) * sp.M
    w = ch.production_rates(rhos[:, None], np.array([T]))[:, 0]
    scale = ch.gross_magnitude(rhos[:, None], np.array([T]))[0]
    assert np.max(np.abs(w)) / scale < 1e-12
    # and a perturbed composition is not in equilibrium
    w2 = ch.production_rates((rhos * [1.1, 0.9, 1, 1, 1])[:, None], np.array([T]))[:, 0]
    assert np.max(np.abs(w2)) / scale > 1e-6
