"""Pins of the oracle's difference operators (Sec. 3.1 reading) and AD operators (Sec. 3.3 reading).

Exactness on polynomials is checked against exact rational arithmetic (fractions),
the periodic operator against its closed-form modified wavenumber, the metric
against the analytic derivative of the cubic mapping of Eq. (27).
"""
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle import stencils as st

# the operators written out as exact rationals: independent restatement of the
# stencil weights is not what is checked here; polynomial exactness is
def exact_deriv_poly(k, x):
    return k * x ** (k - 1) if k > 0 else 0 * x


@pytest.mark.parametrize("order,interior_deg,closure_deg", [(6, 6, 4), (4, 4, 4)])
def test_polynomial_exactness(order, interior_deg, closure_deg):
    n = 24
    x = np.arange(n, dtype=np.float64)          # uniform grid, unit spacing
    h = 3 if order == 6 else 2
    for k in range(0, interior_deg + 2):
        f = (x / n) ** k
        d = st.first_derivative(f, 0, order)
        ex = exact_deriv_poly(k, x / n) / n
        err_in = np.max(np.abs(d[h:n - h] - ex[h:n - h]))
        err_bd = np.max(np.abs(np.r_[d[:h], d[n - h:]] - np.r_[ex[:h], ex[n - h:]]))
        scale = 1.0
        if k <= interior_deg:
            assert err_in < 1e-13 * scale, (order, k, err_in)
        else:
            assert err_in > 1e-10, "interior should not be exact beyond its degree"
        if k <= closure_deg:
            assert err_bd < 1e-13, (order, k, err_bd)


def test_polynomial_exactness_rational():
    """Same statement in exact arithmetic for the 6th-order interior and the closures."""
    c6 = [Fr(3, 4), Fr(-3, 20), Fr(1, 60)]
    for k in range(7):
        # interior at i = 0 of the polynomial i^k: sum c_m ((m)^k - (-m)^k) == k * 0^(k-1)
        v = sum(c * (Fr(m) ** k - Fr(-m) ** k) for m, c in enumerate(c6, start=1))
        assert v == (1 if k == 1 else 0)
    b0 = [Fr(-25, 12), Fr(4), Fr(-3), Fr(4, 3), Fr(-1, 4)]
    b1 = [Fr(-1, 4), Fr(-5, 6), Fr(3, 2), Fr(-1, 2), Fr(1, 12)]
    for k in range(5):
        v0 = sum(c * Fr(m) ** k for m, c in enumerate(b0))
        v1 = sum(c * Fr(m) ** k for m, c in enumerate(b1))
        assert v0 == (k * Fr(0) ** (k - 1) if k > 0 else 0)
        assert v1 == (k * Fr(1) ** (k - 1) if k > 0 else 0)
    # and the floats the oracle uses are these rationals
    assert st.C6 == tuple(float(c) for c in c6)
    assert st.B0 == tuple(float(c) for c in b0)
    assert st.B1 == tuple(float(c) for c in b1)


def test_periodic_modified_wavenumber():
    n = 32
    i = np.arange(n)
    for kk in (1, 3, 7):
        w = 2 * np.pi * kk / n
        f = np.sin(w * i)
        d = st.first_derivative(f, 0, 6, periodic=True)
        kmod = 2 * (0.75 * np.sin(w) - 0.15 * np.sin(2 * w) + np.sin(3 * w) / 60.0)
        assert np.max(np.abs(d - kmod * np.cos(w * i))) < 1e-13
        # and it approximates the exact derivative to 6th order
        assert abs(kmod - w) < w ** 7 / 100 + 1e-14


def test_metric_of_cubic_mapping():
    """Eq. (27) maps the index by a cubic, so D x is exact and the metric is analytic."""
    n = 40
    y0, y1, ky = 0.0, 1.6, 0.15
    m = np.arange(n)
    eta = m / (n - 1)
    y = y0 + (y1 - y0) * ((1 - ky) * eta ** 3 + ky * eta)
    dyd_idx = (y1 - y0) * (3 * (1 - ky) * eta ** 2 + ky) / (n - 1)
    assert np.max(np.abs(st.metric(y) * dyd_idx - 1.0)) < 1e-12


def test_fourth_difference_and_filter():
    n = 30
    x = np.arange(n, dtype=np.float64)
    for k in range(4):
        assert np.max(np.abs(st.fourth_difference(x ** k, 0))) < 1e-9
    assert np.allclose(st.fourth_difference(x ** 4, 0), 24.0)
    assert abs(sum(st.GAUSS9[0:1]) + 2 * sum(st.GAUSS9[1:]) - 1.0) < 1e-15
    g = st.gaussian_filter(np.ones(n), 0)
    assert np.max(np.abs(g - 1.0)) < 1e-15
    g = st.gaussian_filter(x, 0)
    assert np.max(np.abs(g[4:-4] - x[4:-4])) < 1e-12
    g = st.gaussian_filter(x ** 2, 0)
    assert np.max(np.abs(g[4:-4] - (x[4:-4] ** 2 + 4.0 / 3.0))) < 1e-11
    # periodic filter preserves the mean exactly and damps the Nyquist mode
    f = np.cos(np.pi * x[:16])
    gp = st.gaussian_filter(f, 0, periodic=True)
    assert abs(gp.sum()) < 1e-12
    assert np.max(np.abs(gp)) < 0.05
