"""Pins of the FP64 warm-start network reference (no GPU): GELU and its derivative from the
erf definition, backpropagated gradients against central finite differences, and one Adam
step against the update written out by hand."""
import numpy as np

from oracle import mlp_ref as M


def test_gelu_definition_and_derivative():
    z = np.linspace(-5, 5, 101)
    # known values: gelu(0) = 0, gelu(z) -> z for large z, gelu(-z) -> 0
    assert M.gelu(np.array([0.0]))[0] == 0.0
    assert abs(M.gelu(np.array([6.0]))[0] - 6.0) < 1e-7
    assert abs(M.gelu(np.array([-6.0]))[0]) < 1e-7
    h = 1e-6
    fd = (M.gelu(z + h) - M.gelu(z - h)) / (2 * h)
    assert np.abs(fd - M.gelu_grad(z)).max() < 1e-8


def test_backprop_matches_finite_differences():
    rng = np.random.default_rng(0)
    G, S, IN, H, OUT = 3, 5, 4, 6, 3
    params = [0.5 * rng.standard_normal(s) for s in M.shapes(G, IN, H, OUT)]
    X = rng.standard_normal((G, S, IN))
    Yt = rng.standard_normal((G, S, OUT))
    L, grads = M.loss_and_grads(params, X, Yt)
    flat, gflat = M.flatten(params), M.flatten(grads)
    h = 1e-6
    offs = np.cumsum([0] + [int(np.prod(s)) for s in M.shapes(G, IN, H, OUT)])
    picks = np.concatenate([rng.choice(np.arange(a, b), 8, replace=False) for a, b in zip(offs[:-1], offs[1:])])
    for idx in picks:  # eight entries of every parameter block
        p = flat.copy()
        p[idx] += h
        lp, _ = M.loss_and_grads(M.unflatten(p, G, IN, H, OUT), X, Yt)
        p[idx] -= 2 * h
        lm, _ = M.loss_and_grads(M.unflatten(p, G, IN, H, OUT), X, Yt)
        assert abs((lp - lm) / (2 * h) - gflat[idx]) < 1e-7 * max(1.0, abs(gflat[idx]))


def test_skip_path_is_linear_map():
    """With zero hidden weights and biases the hidden activations are gelu(0) = 0, so the network
    is the affine map x -> x W3[H:] + b3 of its input."""
    rng = np.random.default_rng(1)
    G, S, IN, H, OUT = 2, 7, 5, 4, 3
    W1, b1, W2, b2 = (np.zeros(s) for s in M.shapes(G, IN, H, OUT)[:4])
    W3 = rng.standard_normal((G, H + IN, OUT))
    b3 = rng.standard_normal((G, OUT))
    X = rng.standard_normal((G, S, IN))
    Y, _ = M.forward([W1, b1, W2, b2, W3, b3], X)
    for g in range(G):
        assert np.allclose(Y[g], X[g] @ W3[g, H:] + b3[g], rtol=1e-14, atol=1e-14)


def test_adam_step_by_hand():
    th, g = np.array([1.0, -2.0]), np.array([0.5, -0.25])
    m0, v0 = np.zeros(2), np.zeros(2)
    th1, m1, v1 = M.adam_step(th, g, m0, v0, 1, 0.1)
    # first step: m_hat = g, v_hat = g^2 -> theta - lr * g / (|g| + eps)
    assert np.allclose(th1, th - 0.1 * g / (np.abs(g) + 1e-8))
    assert np.allclose(m1, 0.1 * g) and np.allclose(v1, 0.001 * g * g)
