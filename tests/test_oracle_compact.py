"""Pins of the compact (Pade) first-derivative oracle (Sec. 3.1 reading; oracle/compact.py).

* Each row kind satisfies its defining identity exactly, in rational arithmetic, for
  every polynomial up to its order (6 for the sixth-order interior rows, 4 for the
  Pade rows, 3 for the one-sided boundary rows) and fails for the next degree; the
  float coefficients are the intended rationals.
* The whole non-periodic operator therefore differentiates cubics exactly (to
  rounding), whatever the grid length.
* On a periodic grid a Fourier mode e^{ikx} is an eigenfunction: D gives i k'(k) with
  the modified wavenumber k' = (2 a1 sin k + 2 a2 sin 2k) / (1 + 2 alpha cos k).
* Convergence on smooth functions: slopes 6 and 4 on periodic grids; at least 3 (the
  boundary closure's order) on non-periodic ones.
* The right-hand sides formed from differences equal the dense operator B applied to f.
"""
from fractions import Fraction as Fr

import numpy as np
import pytest

from oracle import compact as cp


def _fr(x):
    return Fr(x).limit_denominator(1000)


def _row_residual(kind, deg):
    """LHS - RHS of one row of the given kind at i = 2 (i = 0 for 'b0') for f = x^deg,
    in exact rationals; rows use offsets -2..2 around i."""
    f = lambda x: Fr(x) ** deg                    # noqa: E731
    df = lambda x: deg * Fr(x) ** (deg - 1) if deg else Fr(0)   # noqa: E731
    if kind == "b0":
        lhs = df(0) + _fr(cp.B_ALPHA) * df(1)
        rhs = sum(_fr(w) * f(m) for m, w in enumerate(cp.B_RHS))
        return lhs - rhs
    al, a1, a2 = cp.ROW6 if kind == "p6" else cp.ROW4
    al, a1, a2 = _fr(al), _fr(a1), _fr(a2)
    i = 3                                          # any point; x = i
    lhs = al * df(i - 1) + df(i) + al * df(i + 1)
    rhs = a1 * (f(i + 1) - f(i - 1)) + a2 * (f(i + 2) - f(i - 2))
    return lhs - rhs


@pytest.mark.parametrize("kind,order", [("p6", 6), ("p4", 4), ("b0", 3)])
def test_row_identities_exact_to_their_order(kind, order):
    for deg in range(order + 1):
        assert _row_residual(kind, deg) == 0, (kind, deg)
    assert _row_residual(kind, order + 1) != 0
    # the float constants are exactly the intended rationals' nearest doubles
    assert cp.ROW6 == (1.0 / 3.0, 7.0 / 9.0, 1.0 / 36.0)
    assert cp.ROW4 == (0.25, 0.75, 0.0)
    assert cp.B_RHS == (-2.5, 2.0, 0.5) and cp.B_ALPHA == 2.0


@pytest.mark.parametrize("order", [4, 6])
@pytest.mark.parametrize("n", [7, 12, 33])
def test_cubics_differentiated_exactly(order, n):
    x = np.arange(n, dtype=np.float64) - n / 3.0
    rng = np.random.default_rng(n + order)
    for _ in range(3):
        c = rng.normal(size=4)
        f = c[0] + c[1] * x + c[2] * x ** 2 + c[3] * x ** 3
        ex = c[1] + 2 * c[2] * x + 3 * c[3] * x ** 2
        d = cp.first_derivative(f, 0, order)
        assert np.max(np.abs(d - ex)) <= 1e-12 * np.max(np.abs(ex))
    # and the mirrored end: reversing the grid reverses the derivative's sign
    d1 = cp.first_derivative(f[::-1], 0, order)
    assert np.max(np.abs(d1[::-1] + cp.first_derivative(f, 0, order))) <= 1e-12 * np.max(np.abs(ex))


@pytest.mark.parametrize("order", [4, 6])
def test_periodic_modified_wavenumber(order):
    n = 48
    x = np.arange(n, dtype=np.float64)
    al, a1, a2 = cp.ROW6 if order == 6 else cp.ROW4
    for m in (1, 5, 11, 17):
        k = 2 * np.pi * m / n
        kp = (2 * a1 * np.sin(k) + 2 * a2 * np.sin(2 * k)) / (1 + 2 * al * np.cos(k))
        d = cp.first_derivative(np.sin(k * x), 0, order, periodic=True)
        assert np.max(np.abs(d - kp * np.cos(k * x))) <= 1e-13
        d = cp.first_derivative(np.cos(k * x), 0, order, periodic=True)
        assert np.max(np.abs(d + kp * np.sin(k * x))) <= 1e-13
    # resolving efficiency: the sixth-order scheme keeps k' within 1e-3 of k up to
    # about 2.2 points per half wavelength's fraction (k ~ 1.2); the fourth-order less
    k = 1.0
    kp = (2 * a1 * np.sin(k) + 2 * a2 * np.sin(2 * k)) / (1 + 2 * al * np.cos(k))
    assert abs(kp - k) / k < (2e-3 if order == 6 else 1e-2)


@pytest.mark.parametrize("order", [4, 6])
def test_convergence_slopes(order):
    def err(n, periodic):
        if periodic:
            h = 2 * np.pi / n
            x = h * np.arange(n)
        else:
            x = np.linspace(0.3, 2.7, n)
            h = x[1] - x[0]
        f = np.sin(x) * np.exp(0.3 * np.cos(x))
        ex = (np.cos(x) - 0.3 * np.sin(x) ** 2) * np.exp(0.3 * np.cos(x))
        d = cp.first_derivative(f, 0, order, periodic=periodic) / h
        return np.max(np.abs(d - ex))
    s = np.log2(err(40, True) / err(80, True))
    assert abs(s - order) < 0.3, s
    s = np.log2(err(41, False) / err(81, False))
    assert s > 2.8, s


def test_metric_of_uniform_and_cubic_grids():
    xi = np.arange(30, dtype=np.float64)
    assert np.allclose(cp.metric(0.25 * xi + 3.0), 4.0, rtol=1e-14, atol=0)
    x = 0.1 * xi + 0.002 * xi ** 2 + 1e-4 * xi ** 3
    dx = 0.1 + 0.004 * xi + 3e-4 * xi ** 2
    assert np.max(np.abs(cp.metric(x) - 1.0 / dx)) <= 1e-12 * np.max(1.0 / dx)


@pytest.mark.parametrize("order", [4, 6])
def test_difference_form_equals_dense_operator(order):
    rng = np.random.default_rng(order)
    for n in (8, 9, 21):
        g = rng.normal(size=(n, 3))
        _, B = cp.matrices(n, order)
        assert np.max(np.abs(cp.rhs(g, order) - B @ g)) <= 1e-14
        _, Bp = cp.periodic_matrices(n, order)
        assert np.max(np.abs(cp.rhs(g, order, periodic=True) - Bp @ g)) <= 1e-14
