"""Finite-difference operators in index space (oracle; test infrastructure only).

The paper discretises with 4th/6th-order compact differences on a staggered grid
(Sec. 3.1).  Reading taken for this path: collocated explicit central differences
of the same orders, with one-sided closures at non-periodic ends:

  6th-order interior: [3/4 (f+1 - f-1) - 3/20 (f+2 - f-2) + 1/60 (f+3 - f-3)]
  4th-order interior: [2/3 (f+1 - f-1) - 1/12 (f+2 - f-2)]
  point 0           : -25/12 f0 + 4 f1 - 3 f2 + 4/3 f3 - 1/4 f4
  point 1           : -1/4 f0 - 5/6 f1 + 3/2 f2 - 1/2 f3 + 1/12 f4
  point 2 (6th only): the 4th-order central stencil
  far end           : the mirror images with the sign flipped.

Physical derivatives use separable metrics d(xi)/dx = 1 / (D x), where D x is the
same operator applied to the coordinate array (a periodic direction is uniform and
uses 1/dz).  The artificial-diffusivity operators (Sec. 3.3 reading) are the
fourth difference (1, -4, 6, -4, 1) and a 9-point truncated Gaussian filter.
"""
import numpy as np

C6 = (3.0 / 4.0, -3.0 / 20.0, 1.0 / 60.0)
C4 = (2.0 / 3.0, -1.0 / 12.0)
B0 = (-25.0 / 12.0, 4.0, -3.0, 4.0 / 3.0, -1.0 / 4.0)
B1 = (-1.0 / 4.0, -5.0 / 6.0, 3.0 / 2.0, -1.0 / 2.0, 1.0 / 12.0)

# Gaussian filter weights for offsets 0, 1, 2, 3, 4 (symmetric)
GAUSS9 = (3565.0 / 10368.0, 3091.0 / 12960.0, 1997.0 / 25920.0, 149.0 / 12960.0,
          107.0 / 103680.0)


def _take(f, axis, idx):
    return np.take(f, idx, axis=axis)


def first_derivative(f, axis, order=6, periodic=False):
    """Index-space first derivative D f along ``axis`` (no metric)."""
    f = np.asarray(f, dtype=np.float64)
    n = f.shape[axis]
    out = np.zeros_like(f)
    i = np.arange(n)
    coef = C6 if order == 6 else C4
    if periodic:
        acc = 0.0
        for k, c in enumerate(coef, start=1):
            acc = acc + c * (_take(f, axis, (i + k) % n) - _take(f, axis, (i - k) % n))
        return acc
    h = len(coef)                          # interior half-width
    if n < 2 * h + 2:
        raise ValueError("line too short for the stencil")
    inner = np.arange(h, n - h)
    acc = 0.0
    for k, c in enumerate(coef, start=1):
        acc = acc + c * (_take(f, axis, inner + k) - _take(f, axis, inner - k))
    sl = [slice(None)] * f.ndim

    def put(idx, val):
        s = list(sl); s[axis] = idx
        out[tuple(s)] = val

    put(slice(h, n - h), acc)
    # closures at the start
    put(0, sum(c * _take(f, axis, m) for m, c in enumerate(B0)))
    put(1, sum(c * _take(f, axis, m) for m, c in enumerate(B1)))
    # and their mirror images at the end (sign flipped)
    put(n - 1, -sum(c * _take(f, axis, n - 1 - m) for m, c in enumerate(B0)))
    put(n - 2, -sum(c * _take(f, axis, n - 1 - m) for m, c in enumerate(B1)))
    if order == 6:
        for j in (2, n - 3):
            put(j, C4[0] * (_take(f, axis, j + 1) - _take(f, axis, j - 1))
                + C4[1] * (_take(f, axis, j + 2) - _take(f, axis, j - 2)))
    return out


def metric(coord, order=6):
    """d(xi)/dx = 1 / (D x) for a non-periodic coordinate array."""
    return 1.0 / first_derivative(coord, 0, order)


def metric_periodic(coord):
    """Uniform periodic direction: d(xi)/dz = 1 / dz."""
    return np.full(len(coord), 1.0 / (coord[1] - coord[0]))


def spacing(coord, periodic=False):
    """Local grid spacing Delta_l = dx/d(xi) used by the artificial diffusivity."""
    if periodic:
        return np.full(len(coord), coord[1] - coord[0])
    return 1.0 / metric(coord, 6)


def fourth_difference(f, axis, periodic=False):
    """(1, -4, 6, -4, 1) stencil; non-periodic ends copy the nearest interior value."""
    f = np.asarray(f, dtype=np.float64)
    n = f.shape[axis]
    if periodic:
        i = np.arange(n)
        return (_take(f, axis, (i - 2) % n) - 4.0 * _take(f, axis, (i - 1) % n) + 6.0 * f
                - 4.0 * _take(f, axis, (i + 1) % n) + _take(f, axis, (i + 2) % n))
    inner = np.arange(2, n - 2)
    d = (_take(f, axis, inner - 2) - 4.0 * _take(f, axis, inner - 1) + 6.0 * _take(f, axis, inner)
         - 4.0 * _take(f, axis, inner + 1) + _take(f, axis, inner + 2))
    idx = np.clip(np.arange(n), 2, n - 3) - 2
    return _take(d, axis, idx)


def gaussian_filter(f, axis, periodic=False):
    """9-point truncated Gaussian filter along ``axis``; truncated and renormalised at ends."""
    f = np.asarray(f, dtype=np.float64)
    n = f.shape[axis]
    i = np.arange(n)
    if periodic:
        acc = GAUSS9[0] * f
        for k in range(1, 5):
            acc = acc + GAUSS9[k] * (_take(f, axis, (i - k) % n) + _take(f, axis, (i + k) % n))
        return acc
    acc = np.zeros_like(f)
    wsum = np.zeros(n)
    for k in range(-4, 5):
        w = GAUSS9[abs(k)]
        j = i + k
        ok = (j >= 0) & (j < n)
        wk = np.where(ok, w, 0.0)
        sh = [1] * f.ndim; sh[axis] = n
        acc = acc + wk.reshape(sh) * _take(f, axis, np.clip(j, 0, n - 1))
        wsum = wsum + wk
    sh = [1] * f.ndim; sh[axis] = n
    return acc / wsum.reshape(sh)
