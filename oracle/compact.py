"""Compact (Pade) first derivatives in index space (oracle; test infrastructure only).

Sec. 3.1 discretises in space with fourth- or sixth-order compact finite differences
(it cites Lele's compact schemes) on a staggered grid.  Reading taken for this path:
the collocated tridiagonal schemes of that family, every point carrying all variables
(the staggered layout is not built).  With unit spacing and f' the unknown derivative:

  6th-order interior (2 <= i <= n-3):
      1/3 f'_{i-1} + f'_i + 1/3 f'_{i+1} = 7/9 (f_{i+1} - f_{i-1}) + 1/36 (f_{i+2} - f_{i-2})
  4th-order (Pade) rows, the whole interior of the 4th-order scheme and the points
  1 and n-2 of the 6th-order scheme:
      1/4 f'_{i-1} + f'_i + 1/4 f'_{i+1} = 3/4 (f_{i+1} - f_{i-1})
  boundary point 0 (third-order one-sided compact closure):
      f'_0 + 2 f'_1 = -5/2 f_0 + 2 f_1 + 1/2 f_2 = 2 (f_1 - f_0) + 1/2 (f_2 - f_0)
  point n-1: its mirror image, f'_{n-1} + 2 f'_{n-2} = 5/2 f_{n-1} - 2 f_{n-2} - 1/2 f_{n-3}
  periodic direction: the interior row at every point, indices wrapped.

Each system is solved as it stands: the non-periodic tridiagonal system with LAPACK's
banded solver (partial pivoting), the periodic one as a dense system.  Physical
derivatives use metrics d(xi)/dx = 1 / (D x) with D the same operator on the coordinate
array (a periodic direction is uniform: 1/dz), as for the explicit stencils.
"""
import numpy as np
from scipy.linalg import solve_banded

# interior rows: (alpha, a1, a2) with alpha f'_{i-1} + f'_i + alpha f'_{i+1}
#                = a1 (f_{i+1} - f_{i-1}) + a2 (f_{i+2} - f_{i-2})
ROW6 = (1.0 / 3.0, 7.0 / 9.0, 1.0 / 36.0)
ROW4 = (1.0 / 4.0, 3.0 / 4.0, 0.0)
# boundary row 0: f'_0 + B_ALPHA f'_1 = sum_m B_RHS[m] f_m
B_ALPHA = 2.0
B_RHS = (-5.0 / 2.0, 2.0, 1.0 / 2.0)


def _rows(n, order):
    """Row kinds of the non-periodic operator: 'b0', 'p4', 'p6', 'bn'."""
    kinds = []
    for i in range(n):
        if i == 0:
            kinds.append("b0")
        elif i == n - 1:
            kinds.append("bn")
        elif order == 6 and 2 <= i <= n - 3:
            kinds.append("p6")
        else:
            kinds.append("p4")
    return kinds


def matrices(n, order):
    """Left-hand tridiagonal matrix (banded form ab[3][n] for solve_banded) and the
    dense right-hand-side matrix B [n][n] of the non-periodic operator: A f' = B f."""
    ab = np.zeros((3, n))
    B = np.zeros((n, n))
    for i, k in enumerate(_rows(n, order)):
        ab[1, i] = 1.0
        if k == "b0":
            ab[0, 1] = B_ALPHA                      # super-diagonal entry A[0][1]
            for m, w in enumerate(B_RHS):
                B[0, m] = w
        elif k == "bn":
            ab[2, n - 2] = B_ALPHA                  # sub-diagonal entry A[n-1][n-2]
            for m, w in enumerate(B_RHS):
                B[n - 1, n - 1 - m] = -w
        else:
            al, a1, a2 = ROW6 if k == "p6" else ROW4
            ab[0, i + 1] = al                       # A[i][i+1]
            ab[2, i - 1] = al                       # A[i][i-1]
            B[i, i + 1] += a1
            B[i, i - 1] -= a1
            if a2:
                B[i, i + 2] += a2
                B[i, i - 2] -= a2
    return ab, B


def periodic_matrices(n, order):
    """Dense A, B of the periodic operator (interior row of the order at every point)."""
    al, a1, a2 = ROW6 if order == 6 else ROW4
    A = np.eye(n)
    B = np.zeros((n, n))
    for i in range(n):
        A[i, (i + 1) % n] += al
        A[i, (i - 1) % n] += al
        B[i, (i + 1) % n] += a1
        B[i, (i - 1) % n] -= a1
        if a2:
            B[i, (i + 2) % n] += a2
            B[i, (i - 2) % n] -= a2
    return A, B


def rhs(g, order, periodic=False):
    """Right-hand sides of the rows for lines along axis 0 of g [n][m], each formed from
    the differences the row's definition writes (module doc)."""
    n = g.shape[0]
    r = np.empty_like(g)
    if periodic:
        al, a1, a2 = ROW6 if order == 6 else ROW4
        p1, m1 = np.roll(g, -1, 0), np.roll(g, 1, 0)
        r[:] = a1 * (p1 - m1)
        if a2:
            r += a2 * (np.roll(g, -2, 0) - np.roll(g, 2, 0))
        return r
    for i, k in enumerate(_rows(n, order)):
        if k == "b0":
            r[0] = B_RHS[1] * (g[1] - g[0]) + B_RHS[2] * (g[2] - g[0])
        elif k == "bn":
            r[n - 1] = -(B_RHS[1] * (g[n - 2] - g[n - 1]) + B_RHS[2] * (g[n - 3] - g[n - 1]))
        elif k == "p6":
            r[i] = ROW6[1] * (g[i + 1] - g[i - 1]) + ROW6[2] * (g[i + 2] - g[i - 2])
        else:
            r[i] = ROW4[1] * (g[i + 1] - g[i - 1])
    return r


def first_derivative(f, axis, order=6, periodic=False):
    """Index-space compact first derivative D f along ``axis`` (no metric)."""
    f = np.asarray(f, dtype=np.float64)
    n = f.shape[axis]
    g = np.moveaxis(f, axis, 0).reshape(n, -1)
    r = rhs(g, order, periodic)
    if periodic:
        A, _ = periodic_matrices(n, order)
        d = np.linalg.solve(A, r)
    else:
        ab, _ = matrices(n, order)
        d = solve_banded((1, 1), ab, r)
    return np.moveaxis(d.reshape((n,) + tuple(np.delete(f.shape, axis))), 0, axis)


def metric(coord, order=6):
    """d(xi)/dx = 1 / (D x) of a non-periodic coordinate array."""
    return 1.0 / first_derivative(np.asarray(coord, dtype=np.float64), 0, order)
