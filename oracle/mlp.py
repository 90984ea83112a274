"""Surrogate network reference: forward, backward, Adam (oracle; test infrastructure only).

The paper closes by pointing at machine learning as a way to replace the costly
calls of its thermochemical library (Sec. 5).  The network

    h1 = f(W1 x + b1), h2 = f(W2 h1 + b2), h3 = f(W3 h2 + b3), y = W4 h3 + b4,
    f(z) = max(z, 0)^2   (squared rectifier, f' = 2 max(z, 0))

has widths 7 -> 64 -> 64 -> 64 -> 8; x and y are the surrogate's standardised
features and targets (the composition around the network lives with the tests'
training data).  Parameters are one flat vector in the order
[W1 (64x7, row = output unit), b1, W2 (64x64), b2, W3 (64x64), b3, W4 (8x64), b4],
9352 values.  With ``bf16=True`` every matrix-product operand (weights and layer
inputs) is first rounded to bfloat16 (round to nearest even, from float32), as the
matrix-core path does, except the network's own inputs, which enter as the sum of
two bfloat16 numbers bf16(x) + bf16(x - bf16(x)) (x in float32); everything else
stays float64.  In the backward pass the
same rounding applies to the weights and to the saved layer inputs (the operands the
forward pass consumed); the back-propagated deltas stay unrounded.
"""
import numpy as np

SIZES = (7, 64, 64, 64, 8)
NPARAM = sum(SIZES[i + 1] * SIZES[i] + SIZES[i + 1] for i in range(4))


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    out = []
    o = 0
    for i in range(4):
        n_in, n_out = SIZES[i], SIZES[i + 1]
        W = theta[o:o + n_out * n_in].reshape(n_out, n_in); o += n_out * n_in
        b = theta[o:o + n_out]; o += n_out
        out.append((W, b))
    return out


def pack(layers):
    return np.concatenate([np.concatenate([W.reshape(-1), b]) for W, b in layers])


def to_bf16(a):
    """Round to bfloat16 (RNE) via float32; returned as float64 values."""
    f = np.asarray(a, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    out = r.view(np.float32).astype(np.float64)
    return np.where(np.isnan(f), np.nan, out)


def to_split_bf16(a):
    """bf16(x) + bf16(x - bf16(x)) of float32 x: the two-term input representation."""
    x = np.asarray(a, dtype=np.float32)
    hi = to_bf16(x).astype(np.float32)
    lo = to_bf16((x - hi).astype(np.float32))
    return hi.astype(np.float64) + lo


def activation(z):
    """Squared rectifier max(z, 0)^2."""
    r = np.maximum(z, 0.0)
    return r * r


def activation_slope(a):
    """f'(z) written with the output a = f(z) >= 0: f'(z) = 2 max(z, 0) = 2 sqrt(a)."""
    return 2.0 * np.sqrt(a)


def init_params(seed=0):
    """Glorot-uniform weights, zero biases."""
    rng = np.random.Generator(np.random.PCG64(seed))
    layers = []
    for i in range(4):
        n_in, n_out = SIZES[i], SIZES[i + 1]
        lim = np.sqrt(6.0 / (n_in + n_out))
        layers.append((rng.uniform(-lim, lim, (n_out, n_in)), np.zeros(n_out)))
    return pack(layers)


def forward(theta, X, bf16=False):
    """X [n][7] -> (Y [n][8], cache).  Layer inputs and weights rounded when bf16."""
    layers = unpack(theta)
    q = to_bf16 if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    a = np.asarray(X, dtype=np.float64)
    acts = [a]
    for li, (W, b) in enumerate(layers):
        qa = (to_split_bf16 if (bf16 and li == 0) else q)(a)
        z = qa @ q(W).T + b
        a = activation(z) if li < 3 else z
        acts.append(a)
    return a, acts


def backward(theta, acts, dY, bf16=False):
    """Gradient of a loss with dL/dY = dY [n][8] with respect to theta (flat)."""
    layers = unpack(theta)
    q = to_bf16 if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    grads = [None] * 4
    d = np.asarray(dY, dtype=np.float64)           # dL/dz of the current layer
    for li in range(3, -1, -1):
        W, b = layers[li]
        a_in = acts[li]
        gW = d.T @ (to_split_bf16 if (bf16 and li == 0) else q)(a_in)
        gb = d.sum(axis=0)
        grads[li] = (gW, gb)
        if li > 0:
            da = d @ q(W)
            d = da * activation_slope(acts[li])
    return pack(grads)


def mse_grad(Yhat, Yt):
    """L = mean over n and the 8 outputs of (Yhat - Yt)^2 and dL/dYhat."""
    r = Yhat - Yt
    return float(np.mean(r * r)), 2.0 * r / r.size


def adam(theta, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam step (t counts from 1); returns new (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * g
    v = b2 * v + (1.0 - b2) * g * g
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
