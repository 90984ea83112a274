"""Closed-form pins of oracle functions that the flow-level pins leave open.

* Artificial diffusivity (Sec. 3.3 reading, oracle/ad.py::coefficients): on a uniform
  grid a quartic field has the constant fourth difference 24 h^4 (ends copy the nearest
  interior value, so also constant there), and the Gaussian filter maps a constant to
  itself.  Each coefficient is then a closed form that fixes its power of the spacing,
  its prefactor (rho, rho f_sw, rho c / T, c) and the overshoot term with the
  geometric-mean spacing.
* Wall-row update (Sec. 3.2, oracle/rhs.py::apply_bc): interior rows whose mass
  fractions and temperature are even polynomials plus a cubic in the wall distance
  (zero slope at the wall) extrapolate exactly to the wall value; the wall row then
  holds the evolved density, zero momentum and the energy of (T_w or the extrapolated
  T, the extrapolated Y), and the inflow column and held points keep their state.
* Thermally perfect gas (Sec. 2.2.2, oracle/tpg.py::temperature): the returned T is
  the 40-digit root of e(T) = e correctly rounded (within half a unit in the last
  place), which the extended-precision final step provides and Newton alone does not.
* Nondimensionalisation (Eq. 7, oracle/rhs.py::primitives): p, mu, kappa, D_s, omega_s
  times their reference scales equal the SI functions at the dimensional state, with
  p = rho R_mix T formed here from the gas constants.
"""
import dataclasses

import mpmath
import numpy as np
import pytest

from oracle import ad as adm
from oracle import chemistry as och
from oracle import rhs as orhs
from oracle import species as sp
from oracle import thermo as oth
from oracle import tpg
from oracle import transport as otr
from paper_2210_05547_amd import fields

RNG = np.random.default_rng(2022)


def _uniform_case(nx=26, ny=22, hx=0.3, hy=0.17, air5=True):
    cfg = fields.get_config("c3" if air5 else "c1").scaled(nx, ny)
    cfg = dataclasses.replace(cfg, ad=True)
    x = hx * (np.arange(nx) - nx // 2)
    y = hy * (np.arange(ny) - ny // 2)
    return orhs.Case(cfg, x, y, np.zeros(1)), x, y


def test_ad_coefficients_closed_form():
    case, x, y = _uniform_case()
    hx, hy = x[1] - x[0], y[1] - y[0]
    Cmu, Cbeta, Ckap, CD, CY = case.cfg.ad_coef
    X, Yc = np.meshgrid(x, y)
    X, Yc = X[None], Yc[None]
    sh = X.shape
    rho = RNG.uniform(0.5, 2.0, sh)
    c = RNG.uniform(0.8, 1.5, sh)
    T = RNG.uniform(1.0, 4.0, sh)
    a_e, b_th, g_s = 0.7, 1.3, 0.002
    e = a_e * X ** 4                          # D4_x = 24 a_e hx^4, D4_y = 0
    theta = -(b_th * Yc ** 4 + 1.0)           # compressive everywhere: f_sw = 1
    zero = np.zeros(sh)
    G = [[theta, zero], [zero, zero]]         # |S| = |theta|, no vorticity
    Ys = np.stack([g_s * X ** 4, g_s * Yc ** 4, np.full(sh, -0.01), np.full(sh, 0.25),
                   np.full(sh, 1.02)])
    P = dict(rho=rho, c=c, T=T, e=e, Y=Ys)
    out = adm.coefficients(P, G, case)
    d4y = 24.0 * b_th * hy ** 4
    rel = lambda a, b: np.max(np.abs(a - b)) / np.max(np.abs(b))  # noqa: E731
    assert rel(out["mu"], Cmu * rho * d4y * hy ** 2) < 1e-9
    assert rel(out["beta"], Cbeta * rho * 1.0 * d4y * hy ** 2) < 1e-9
    assert rel(out["kappa"], Ckap * rho * c / T * (24.0 * a_e * hx ** 4) * hx) < 1e-9
    dbar = np.sqrt(hx * hy)
    D = out["D"]
    assert rel(D[0], c * CD * 24.0 * g_s * hx ** 4 * hx) < 1e-9
    assert rel(D[1], c * CD * 24.0 * g_s * hy ** 4 * hy) < 1e-9
    assert rel(D[2], c * CY * 0.01 * dbar) < 1e-12        # undershoot below 0
    assert np.max(np.abs(D[3])) == 0.0                     # inside [0, 1]: no term
    assert rel(D[4], c * CY * 0.02 * dbar) < 1e-12        # overshoot above 1


def test_ad_switch_off_for_expansion_and_vorticity():
    """beta* vanishes where theta >= 0, and the switch is theta^2/(theta^2 + |omega|^2)."""
    case, x, y = _uniform_case()
    X, Yc = np.meshgrid(x, y)
    sh = (1,) + X.shape
    theta = -np.ones(sh)
    w = np.full(sh, 3.0)                      # G[1][0] - G[0][1] = 3: |omega|^2 = 9
    G = [[theta, np.zeros(sh)], [w, np.zeros(sh)]]
    th, fsw = adm.switch(G, 2)
    assert np.allclose(fsw, 1.0 / (1.0 + 9.0), rtol=1e-15, atol=0)
    G2 = [[np.ones(sh), np.zeros(sh)], [w, np.zeros(sh)]]
    assert np.all(adm.switch(G2, 2)[1] == 0.0)


@pytest.mark.parametrize("wall", [0, 1])
def test_wall_row_update_closed_form(wall):
    cfg = fields.get_config("c2").scaled(20, 16)
    cfg = dataclasses.replace(cfg, wall=wall, T_wall=1500.0)
    Q, Qr, info = fields.initial_field(cfg)
    hold = np.array([5, 6, 7 + cfg.nx], dtype=np.int64)      # two wall points, one row-1 point
    case = orhs.Case(cfg, info["x"], info["y"], info["z"], hold)
    ref = case.ref
    nx = cfg.nx
    j = np.arange(1, 5, dtype=np.float64)
    Y0 = np.array([0.70, 0.18, 0.05, 0.03, 0.04])
    dY = np.array([0.01, -0.006, 0.002, -0.003, -0.003])     # sum zero: Y stays normalised
    T0 = 1800.0 / ref["T_ref"]
    rho_rows = RNG.uniform(0.8, 1.2, (4, nx))
    for m in range(4):
        q = j[m]
        Ym = Y0 + dY * (0.02 * q ** 2 - 0.004 * q ** 3)      # zero slope at the wall
        Tm = T0 * (1.0 + 0.03 * q ** 2 + 0.002 * q ** 3)
        e = oth.mixture_e(np.full(nx, Tm * ref["T_ref"]), Ym[:, None] * np.ones(nx)) / ref["c_inf"] ** 2
        Q[:5, 0, m + 1, :] = rho_rows[m] * Ym[:, None]
        Q[5:7, 0, m + 1, :] = 0.0
        Q[7, 0, m + 1, :] = rho_rows[m] * e
    before = Q.copy()
    rho_w = Q[:5, 0, 0, :].sum(0)
    orhs.apply_bc(Q, case)
    Tw = cfg.T_wall if wall == 1 else T0 * ref["T_ref"]
    ew = oth.mixture_e(np.full(nx, Tw), Y0[:, None] * np.ones(nx)) / ref["c_inf"] ** 2
    i = np.arange(1, nx)
    i = i[(i != 5) & (i != 6)]                                 # held wall points keep Q
    sc = np.max(np.abs(before[:5, 0, 0]))
    assert np.max(np.abs(Q[:5, 0, 0, i] - rho_w[i] * Y0[:, None])) <= 2e-14 * sc
    assert np.all(Q[5:7, 0, 0, i] == 0.0)
    assert np.max(np.abs(Q[7, 0, 0, i] - rho_w[i] * ew[i])) <= 1e-13 * np.max(np.abs(rho_w * ew))
    assert np.array_equal(Q[:, :, 0, [0, 5, 6]], before[:, :, 0, [0, 5, 6]])
    assert np.array_equal(Q[:, :, 1:], before[:, :, 1:])       # interior rows untouched


@pytest.mark.parametrize("T_lo,T_hi", [(300.0, 900.0), (1000.0, 1700.0), (2000.0, 6000.0)])
def test_tpg_inversion_is_the_rounded_root(T_lo, T_hi):
    """The inversion returns the correctly rounded root (within half a unit in the last
    place) of e(T) = e with the definition's own double constants: Newton alone ends
    up to about two units away near the adiabatic wall temperature (1000-1700 K)."""
    g, T_inf = 1.4, 220.0
    k = tpg.constants(g, T_inf)
    T_ref = (g - 1.0) * T_inf
    Tn = RNG.uniform(T_lo, T_hi, 40) / T_ref
    e = tpg.energy(Tn, k["k0"], k["th"], g)
    T, _, ok = tpg.temperature(e, k["k0"], k["th"], g)
    assert ok.all()
    mpmath.mp.dps = 40
    a = mpmath.mpf((g - 1.0) / g)             # the double value the definition uses
    k0, th = mpmath.mpf(k["k0"]), mpmath.mpf(k["th"])
    worst = 0.0
    for ei, Ti in zip(e, T):
        f = lambda t: k0 * t + k0 * a * th / mpmath.expm1(th / t) - a * t - mpmath.mpf(ei)  # noqa: E731
        root = mpmath.findroot(f, mpmath.mpf(Ti))
        worst = max(worst, float(abs(mpmath.mpf(Ti) - root) / mpmath.mpf(np.spacing(Ti))))
    assert worst <= 0.5 + 1e-6, worst


def test_nondimensional_scalings_against_si():
    cfg = fields.get_config("c2").scaled(24, 18)
    Q, Qr, info = fields.initial_field(cfg)
    case = orhs.Case(cfg, info["x"], info["y"], info["z"])
    ref = case.ref
    P = orhs.primitives(Q, case)
    rho_si = P["rho"] * ref["rho_inf"]
    T_si = P["T"] * ref["T_ref"]
    Y = P["Y"]
    R_mix = sum(Y[s] * sp.R_U / sp.M[s] for s in range(5))
    p_si = rho_si * R_mix * T_si
    c2 = ref["c_inf"] ** 2
    rel = lambda a, b: np.max(np.abs(a - b)) / np.max(np.abs(b))  # noqa: E731
    assert rel(P["p"] * ref["rho_inf"] * c2, p_si) < 1e-14
    mu, kap = otr.mixture_viscosity_conductivity(T_si, Y)
    assert rel(P["mu"] * ref["mu_inf"], mu) < 1e-14
    assert rel(P["kappa"] * ref["kappa_inf"], kap) < 1e-14
    D = otr.averaged_diffusion(T_si, p_si, Y)
    for s in range(5):
        assert rel(P["D"][s] * ref["c_inf"] * ref["L_ref"], D[s]) < 1e-13
    w = och.production_rates(Q[:5] * ref["rho_inf"], T_si)
    for s in range(5):
        assert rel(P["wdot"][s] * ref["rho_inf"] * ref["c_inf"] / ref["L_ref"], w[s]) < 1e-13
    # the reference state of Eq. (7) and (11): Re = rho c L / mu, Ec = c^2 / (c_p T_ref) = 1
    assert abs(ref["Re"] - ref["rho_inf"] * ref["c_inf"] * ref["L_ref"] / ref["mu_inf"]) <= \
        1e-13 * ref["Re"]
    assert abs(ref["Ec"] - 1.0) <= 4 * np.finfo(float).eps
