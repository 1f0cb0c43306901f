"""FP64 reference of the per-subsystem warm-start network — TEST INFRASTRUCTURE ONLY.

Only ``tests/`` use this module; the library's HIP kernels are checked against it.

The warm start (the better initial point that Section V names as future work) predicts, for
every subsystem g, the Phi-comp row multipliers alpha of its own rows from the d-hop slice of
x0. One network per subsystem (separate weights):

    h1 = gelu(x W1 + b1),  h2 = gelu(h1 W2 + b2),  y = [h2, x] W3 + b3,
    gelu(z) = z Phi(z) = z (1 + erf(z / sqrt 2)) / 2,

where [h2, x] is the concatenation (the output layer also sees the input directly: without
inequality constraints the optimal multipliers are a linear function of that slice of x0).

with x = (x0 of the patch members in ascending order) / x_scale, zero-padded to IN, and
alpha = y_scale * y. Training minimises the mean squared error over all subsystems, samples
and outputs with Adam (Kingma & Ba, with bias correction).

Shapes: X [G, S, IN], W1 [G, IN, H], b1 [G, H], W2 [G, H, H], b2 [G, H], W3 [G, H + IN, OUT],
b3 [G, OUT]; the flat parameter vector is their concatenation in that order (row-major).
"""
from __future__ import annotations

import numpy as np
from scipy.special import erf

SQRT2 = np.sqrt(2.0)


def gelu(z):
    return 0.5 * z * (1.0 + erf(z / SQRT2))


def gelu_grad(z):
    return 0.5 * (1.0 + erf(z / SQRT2)) + z * np.exp(-0.5 * z * z) / np.sqrt(2.0 * np.pi)


def shapes(G, IN, H, OUT):
    return [(G, IN, H), (G, H), (G, H, H), (G, H), (G, H + IN, OUT), (G, OUT)]


def unflatten(flat, G, IN, H, OUT):
    out, o = [], 0
    for shp in shapes(G, IN, H, OUT):
        n = int(np.prod(shp))
        out.append(np.asarray(flat[o:o + n], dtype=np.float64).reshape(shp))
        o += n
    return out


def flatten(params):
    return np.concatenate([p.ravel() for p in params])


def forward(params, X):
    W1, b1, W2, b2, W3, b3 = params
    Z1 = np.einsum("gsi,gih->gsh", X, W1) + b1[:, None, :]
    A1 = gelu(Z1)
    Z2 = np.einsum("gsi,gih->gsh", A1, W2) + b2[:, None, :]
    A2 = gelu(Z2)
    A2X = np.concatenate([A2, X], axis=2)
    Y = np.einsum("gsi,gio->gso", A2X, W3) + b3[:, None, :]
    return Y, (Z1, A1, Z2, A2X)


def loss_and_grads(params, X, Yt):
    """L = sum (Y - Yt)^2 / (G S OUT) and dL/dparams (backpropagation)."""
    W1, b1, W2, b2, W3, b3 = params
    Y, (Z1, A1, Z2, A2X) = forward(params, X)
    H = Z2.shape[2]
    n = Y.size
    L = float(np.sum((Y - Yt) ** 2) / n)
    dY = 2.0 * (Y - Yt) / n
    dW3 = np.einsum("gsh,gso->gho", A2X, dY)
    db3 = dY.sum(axis=1)
    dZ2 = np.einsum("gso,gho->gsh", dY, W3[:, :H, :]) * gelu_grad(Z2)
    dW2 = np.einsum("gsh,gsk->ghk", A1, dZ2)
    db2 = dZ2.sum(axis=1)
    dZ1 = np.einsum("gsk,ghk->gsh", dZ2, W2) * gelu_grad(Z1)
    dW1 = np.einsum("gsi,gsh->gih", X, dZ1)
    db1 = dZ1.sum(axis=1)
    return L, [dW1, db1, dW2, db2, dW3, db3]


def adam_step(theta, g, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update of the flat vectors (t is the 1-based step count)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
