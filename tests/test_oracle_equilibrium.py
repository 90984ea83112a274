"""Pins of the LTE composition oracle (Sec. 2.2.1, frozen and equilibrium flow;
oracle/equilibrium.py::composition).

* Element balances hold: sum_s a_es c_s equals the mixture's element densities.
* The composition is a minimum of the free energy f(c) over compositions with the same
  elements: f grows along every element-conserving direction (the three reactions
  N2 = 2N, O2 = 2O, NO = N + O span them), in both senses -- checked on f itself, not on
  the balances the solver uses.
* Detailed balance: the five-reaction finite-rate mechanism (FP64 chemistry) has zero
  net production there, and not at a perturbed composition.
* Limits: cold air is molecular N2/O2 at the mixture's element split; hot thin air is
  atomic; a single element (pure nitrogen, pure oxygen) gives the closed form of
  2 c^2/K + c = n and joins the two-element solution continuously.
* Non-finite or out-of-range inputs give status 3.
"""
import mpmath as mp
import numpy as np
import pytest

from oracle import chemistry as ch
from oracle import equilibrium as eq
from oracle import species as sp

RNG = np.random.default_rng(44)


def _conc(rho, Y):
    return Y * rho / sp.M[:, None]


def test_element_balances():
    n = 12
    rho = 10 ** RNG.uniform(-5, 0.5, n)
    T = RNG.uniform(800.0, 16000.0, n)
    xi = RNG.uniform(0.05, 0.95, n)
    Y, st = eq.composition(rho, T, xi)
    assert (st == 0).all()
    c = _conc(rho, Y)
    nN = rho * xi / eq.M_N_ATOM
    nO = rho * (1 - xi) / eq.M_O_ATOM
    el = sp.ELEMENTS.T @ c
    assert np.max(np.abs(el[0] / nN - 1)) < 1e-14
    assert np.max(np.abs(el[1] / nO - 1)) < 1e-14
    assert np.max(np.abs(Y.sum(0) - 1)) < 1e-14


@pytest.mark.parametrize("T,rho", [(2500.0, 0.3), (4500.0, 0.01), (8000.0, 1e-3)])
def test_free_energy_minimum_along_element_conserving_directions(T, rho):
    xi = 0.767082 * 28.0134 / 28.0134      # air's element-N mass fraction
    nN = mp.mpf(rho) * mp.mpf(xi) / mp.mpf(eq.M_N_ATOM)
    nO = mp.mpf(rho) * (1 - mp.mpf(xi)) / mp.mpf(eq.M_O_ATOM)
    c = eq.solve(T, nN, nO)
    f0 = eq.free_energy(T, c)
    cmin = min(c)
    for r in ([-1, 0, 0, 2, 0], [0, -1, 0, 0, 2], [0, 0, -1, 1, 1], [-1, 1, 0, 2, -2]):
        for sgn in (1, -1):
            eps = sgn * cmin * mp.mpf("1e-6")
            cp = [ci + eps * ri for ci, ri in zip(c, r)]
            assert eq.free_energy(T, cp) > f0, (r, sgn)
    # and the stationarity the solver relies on is a genuine condition: a composition off
    # the equilibrium along a reaction has a non-zero directional derivative
    d = [ci + cmin * mp.mpf("1e-3") * ri for ci, ri in zip(c, [-1, 0, 0, 2, 0])]
    assert eq.free_energy(T, d) - f0 > 0


@pytest.mark.parametrize("T,rho,xi", [(2600.0, 0.05, 0.767), (5000.0, 3e-3, 0.6),
                                      (9000.0, 1e-4, 0.85)])
def test_detailed_balance_of_the_mechanism(T, rho, xi):
    Y, st = eq.composition(np.array([rho]), np.array([T]), np.array([xi]))
    rhos = Y * rho
    w = ch.production_rates(rhos, np.array([T]))[:, 0]
    scale = ch.gross_magnitude(rhos, np.array([T]))[0]
    assert np.max(np.abs(w)) / scale < 1e-12
    w2 = ch.production_rates(rhos * np.array([[1.05], [0.97], [1.0], [1.0], [1.0]]),
                             np.array([T]))[:, 0]
    assert np.max(np.abs(w2)) / scale > 1e-6


def test_limits_and_single_elements():
    xi = 0.7671
    Y, _ = eq.composition([1.0], [1000.0], [xi])
    assert Y[3, 0] < 1e-10 and Y[4, 0] < 1e-10 and Y[2, 0] < 1e-4   # molecular, a little NO
    assert abs(Y[0, 0] + Y[2, 0] * sp.M[3] / sp.M[2] - xi) < 1e-14
    Y, _ = eq.composition([1e-4], [20000.0], [xi])
    assert Y[3, 0] + Y[4, 0] > 0.99
    # pure nitrogen: closed form, and continuity with the two-element solve
    T, rho = 7000.0, 2e-3
    Y1, _ = eq.composition([rho], [T], [1.0])
    K1 = eq.Kc(T, [-1, 0, 0, 2, 0])
    cN = Y1[3, 0] * rho / sp.M[3]
    nN = rho / eq.M_N_ATOM
    assert abs(float(2 * mp.mpf(cN) ** 2 / K1 + cN) / nN - 1) < 1e-14
    assert Y1[1, 0] == 0.0 and Y1[2, 0] == 0.0 and Y1[4, 0] == 0.0
    Y2, _ = eq.composition([rho], [T], [1.0 - 1e-12])
    assert abs(Y2[3, 0] - Y1[3, 0]) < 1e-9 and abs(Y2[0, 0] - Y1[0, 0]) < 1e-9
    Y3, _ = eq.composition([rho], [T], [0.0])
    assert Y3[0, 0] == 0.0 and abs(Y3[1, 0] + Y3[4, 0] - 1) < 1e-15


def test_invalid_inputs_status():
    Y, st = eq.composition([np.nan, 1.0, -1.0, 1.0, 1.0], [3000.0, np.inf, 3000.0, 0.0, 3000.0],
                           [0.7, 0.7, 0.7, 0.7, 1.5])
    assert st.tolist() == [3, 3, 3, 3, 3] and np.isnan(Y).all()
