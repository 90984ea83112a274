"""Pins of the Stefan-Maxwell diffusion oracle (Eqs. 16, 17, 20; oracle/transport.py).

Equal binary coefficients: the exact solution is Ramshaw's flux of Eq. (18) (read with
grad X_s) with D_s = D; a binary mixture: Fick's law J_1 = -rho D_12 grad Y_1; the mass
constraint sum_s J_s = 0; and the solution satisfies the unregularised Stefan-Maxwell
relations of every species present.
"""
import numpy as np

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
    X = tr.mole_fractions(Y)
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
    # the three absent species enter at the clipped mole fraction 1e-12: a perturbation of
    # that order, not an error of the formula
    assert np.max(np.abs(J[0] - fick)) <= 1e-10 * np.max(np.abs(fick))
    assert np.max(np.abs(J[2:])) <= 1e-11 * np.max(np.abs(fick))   # absent species: the clip only


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
