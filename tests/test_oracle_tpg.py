"""Pins of the thermally perfect gas oracle (Sec. 2.2.2, module oracle/tpg).

Keyes' law against tabulated conductivities of air; the normalisation c_p(T_inf) =
c_p,inf; the low- and high-temperature limits of the harmonic-oscillator specific heat
(7/2 R with vibration frozen, 9/2 R with it fully excited); the closed-form energy
against a numerical integral of c_v from 0 K; the calorically perfect limit; the energy
inversion round trip; the free-stream Prandtl number of air; uniform flow preserved.
"""
import dataclasses

import numpy as np
from scipy import integrate

from oracle import refstate as rs
from oracle import rhs as R
from oracle import tpg
from paper_2210_05547_amd import fields as f

G = 1.4


def test_keyes_matches_tabulated_air_conductivity():
    # thermal conductivity of air at 1 atm [W/(m K)], standard heat-transfer tables
    table = {300.0: 26.3e-3, 600.0: 46.9e-3, 1000.0: 66.7e-3}
    for T, k in table.items():
        assert abs(float(tpg.keyes(T)) / k - 1.0) < 0.02, T


def test_cp_normalised_at_free_stream():
    for T_inf in (220.0, 350.0, 947.0):
        cp_inf = G * tpg.R_AIR / (G - 1.0)
        assert abs(float(tpg.cp_dimensional(T_inf, G, T_inf)) / cp_inf - 1.0) < 1e-14


def test_cp_limits_frozen_and_fully_excited_vibration():
    T_inf = 220.0
    # vibration frozen far below Theta: 7/2 R (up to the tiny excitation at T_inf)
    assert abs(float(tpg.cp_dimensional(30.0, G, T_inf)) / tpg.R_AIR - 3.5) < 1e-3
    # fully excited far above Theta: 7/2 R + R
    assert abs(float(tpg.cp_dimensional(3.0e6, G, T_inf)) / tpg.R_AIR - 4.5) < 1e-3
    # monotone in between
    T = np.linspace(50.0, 20000.0, 400)
    assert np.all(np.diff(tpg.cp_dimensional(T, G, T_inf)) > 0.0)


def test_energy_is_the_integral_of_cv():
    c = tpg.constants(G, 220.0)
    k0, th = c["k0"], c["th"]
    for T in (0.5, 2.5, 10.0, 40.0, 120.0):
        num, err = integrate.quad(lambda t: float(tpg.cv(t, k0, th, G)), 0.0, T,
                                  epsabs=0.0, epsrel=1e-13, limit=400)
        assert abs(num - float(tpg.energy(T, k0, th, G))) <= 1e-11 * num, T


def test_calorically_perfect_limit():
    T = np.linspace(0.1, 50.0, 200)
    e = tpg.energy(T, 1.0, 1.0e6, G)          # Theta -> infinity, c_p0 = c_p,inf
    assert np.max(np.abs(G * e / T - 1.0)) < 1e-15


def test_energy_inversion_round_trip():
    c = tpg.constants(G, 220.0)
    T = np.linspace(50.0, 6000.0, 1000) / ((G - 1.0) * 220.0)
    e = tpg.energy(T, c["k0"], c["th"], G)
    Tn, it, ok = tpg.temperature(e, c["k0"], c["th"], G)
    assert ok.all() and it.max() <= 12
    assert np.max(np.abs(Tn / T - 1.0)) < 1e-13


def test_free_stream_prandtl_number_of_air():
    ref = rs.reference_tpg(G, 6.0, 220.0, 1.0e5)
    assert 0.70 < ref["Pr"] < 0.76
    assert ref["Ec"] == 1.0 and abs(ref["k0"] - 1.0) < 1e-4


def test_uniform_flow_tpg():
    cfg = dataclasses.replace(f.get_config("c1t"), nx=24, ny=16, sponge_out=0, sponge_top=0)
    x, y, z = f.grid(cfg)
    case = R.Case(cfg, x, y, z)
    sh = (1, cfg.ny, cfg.nx)
    rho, u, v, T = 1.3, 5.0, 0.7, 9.0
    ref = case.ref
    e = float(tpg.energy(T, ref["k0"], ref["th"], ref["gamma"]))
    Q = np.stack([np.full(sh, rho), np.full(sh, rho * u), np.full(sh, rho * v),
                  np.full(sh, rho * (e + 0.5 * (u * u + v * v)))])
    P = R.primitives(Q, case)
    assert np.max(np.abs(P["T"] / T - 1.0)) < 1e-13
    Rr = R.rhs(Q, Q.copy(), case)
    assert np.max(np.abs(Rr)) < 1e-10
