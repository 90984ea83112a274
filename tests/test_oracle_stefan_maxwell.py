"""Pins of the Stefan-Maxwell diffusion oracle (Eqs. 16, 17, 20; oracle/transport.py).

Equal binary coefficients: the exact solution is Ramshaw's flux of Eq. (18) (read with
grad X_s) with D_s = D; a binary mixture: Fick's law J_1 = -rho D_12 grad Y_1; the mass
constraint sum_s J_s = 0; the solution satisfies the unregularised Stefan-Maxwell
relations of every species present; and, on states with an absent species and with
negative mole fractions (the undershoots a discrete field carries), it equals a
40-digit solve of four of the relations plus the mass constraint (a different
closure of the same system than the oracle's), whose absent species' flux follows
from its own relation in closed form.
"""
import mpmath
import numpy as np
import pytest

from oracle import species as sp
from oracle import transport as tr

RNG = np.random.default_rng(11)


def _state(n, zero=()):
    Y = RNG.dirichlet(np.ones(5), n).T
    for s in zero:
        Y[s] = 0.0
    Y = Y / Y.sum(0)
    rho = 10 ** RNG.uniform(-3, 0, n)
    gX = RNG.normal(size=(5, 2, n))
    gX = gX - gX.mean(0)                      # sum_s grad X_s = 0
    return rho, Y, gX


def test_equal_binary_coefficients_give_ramshaw_exactly():
    rho, Y, gX = _state(200)
    D = 3.7e-4
    J = tr.stefan_maxwell_fluxes(rho, Y, gX, np.full((5, 5, 200), D))
    Mbar = 1.0 / np.sum(Y / sp.M[:, None], axis=0)
    a = rho * (sp.M[:, None] / Mbar) * D                   # rho (M_s / Mbar) D_s
    corr = np.sum(a[:, None] * gX, axis=0)
    Jr = -a[:, None] * gX + Y[:, None] * corr
    assert np.max(np.abs(J - Jr)) <= 1e-12 * np.max(np.abs(Jr))


def test_binary_mixture_is_fick():
    rho, Y, gX = _state(100, zero=(2, 3, 4))
    gX[2:] = 0.0
    gX[1] = -gX[0]
    T = RNG.uniform(300.0, 5000.0, 100)
    D = tr.binary_diffusion(T, 1.0e4)
    J = tr.stefan_maxwell_fluxes(rho, Y, gX, D)
    X = tr.mole_fractions(Y)
    Mbar = X[0] * sp.M[0] + X[1] * sp.M[1]
    gY0 = (sp.M[0] * sp.M[1] / Mbar ** 2) * gX[0]           # Y_0 = X_0 M_0 / Mbar
    fick = -rho * D[0, 1] * gY0
    assert np.max(np.abs(J[0] - fick)) <= 1e-12 * np.max(np.abs(fick))
    assert np.max(np.abs(J[2:])) <= 1e-14 * np.max(np.abs(fick))   # absent species: rounding only


def test_mass_constraint_and_stefan_maxwell_relations():
    rho, Y, gX = _state(300)
    T = RNG.uniform(300.0, 8000.0, 300)
    D = tr.binary_diffusion(T, 2.0e4)
    J = tr.stefan_maxwell_fluxes(rho, Y, gX, D)
    scale = np.max(np.abs(J))
    assert np.max(np.abs(J.sum(0))) <= 1e-14 * scale
    X = tr.mole_fractions(Y)
    V = J / (rho * Y)[:, None]
    for s in range(5):
        lhs = sum(X[s] * X[i] / D[s, i] * (V[i] - V[s]) for i in range(5) if i != s)
        assert np.max(np.abs(lhs - gX[s])) <= 1e-11 * np.max(np.abs(gX[s])), s


def _mp_fluxes(rho, Y, g, D, drop):
    """40-digit J_s from the relations of every species but `drop` plus sum_s J_s = 0."""
    mpmath.mp.dps = 40
    Yq = [mpmath.mpf(float(v)) for v in Y]
    nq = [Yq[s] / mpmath.mpf(float(sp.M[s])) for s in range(5)]
    tot = sum(nq)
    X = [v / tot for v in nq]
    A = mpmath.matrix(5, 5)
    b = mpmath.matrix(5, 1)
    rows = [s for s in range(5) if s != drop]
    for r, s in enumerate(rows):
        for i in range(5):
            if i == s:
                continue
            # sum_{i != s} X_s X_i / D_si (V_i - V_s) with V_i = J_i / (rho Y_i) and
            # X_i / Y_i = Mbar / M_i: in the unknowns J_i the coefficients are
            # X_s Mbar / (rho M_i D_si) on J_i and -X_i Mbar / (rho M_s D_si) on J_s
            Dsi = mpmath.mpf(float(D[s, i]))
            A[r, i] += X[s] / (tot * mpmath.mpf(float(rho)) * mpmath.mpf(float(sp.M[i])) * Dsi)
            A[r, s] -= X[i] / (tot * mpmath.mpf(float(rho)) * mpmath.mpf(float(sp.M[s])) * Dsi)
        b[r] = mpmath.mpf(float(g[s]))
    for i in range(5):
        A[4, i] = 1
    b[4] = 0
    J = mpmath.lu_solve(A, b)
    return np.array([float(J[s]) for s in range(5)])


@pytest.mark.parametrize("case", ["absent", "negative", "absent_and_negative"])
def test_zero_and_negative_mole_fractions_against_40_digit_solve(case):
    n = 12
    rho, Y, gX = _state(n)
    if case in ("absent", "absent_and_negative"):
        Y[2] = 0.0                               # NO absent
    if case in ("negative", "absent_and_negative"):
        Y[4] = -RNG.uniform(1e-4, 2e-2, n)       # O undershoot, as after a steep front
        Y[3] = -RNG.uniform(1e-6, 1e-3, n)
    Y = Y / Y.sum(0)
    T = RNG.uniform(500.0, 9000.0, n)
    D = tr.binary_diffusion(T, 3.0e4)
    J = tr.stefan_maxwell_fluxes(rho, Y, gX, D)
    for p in range(n):
        for d in range(2):
            Jm = _mp_fluxes(rho[p], Y[:, p], gX[:, d, p], D[:, :, p], drop=p % 5)
            scale = np.max(np.abs(Jm))
            assert np.max(np.abs(J[:, d, p] - Jm)) <= 1e-13 * scale, (case, p, d)
            if case != "negative":
                # the absent species' own row alone fixes its flux:
                # J_s = -M_s (rho / Mbar) grad X_s / sum_{i != s} X_i / D_si
                X = tr.mole_fractions(Y[:, p:p + 1])[:, 0]
                Mbar = 1.0 / np.sum(Y[:, p] / sp.M)
                den = sum(X[i] / D[2, i, p] for i in range(5) if i != 2)
                J2 = -sp.M[2] * (rho[p] / Mbar) * gX[2, d, p] / den
                assert abs(J[2, d, p] - J2) <= 1e-13 * scale
