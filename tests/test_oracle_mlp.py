"""Pins of the warm-start network oracle (FP64 CPU) against facts that do not
come from the oracle itself: torch's BF16 conversion, closed forms of the
normal distribution, a library matmul for the one-layer case, central finite
differences of the loss, and closed forms of Adam's first steps."""
import math

import numpy as np
import pytest

import oracle

torch = pytest.importorskip("torch")


def _params(widths, rng, scale=1.0):
    parts = [rng.normal(0, scale / math.sqrt(widths[l]), widths[l] * widths[l + 1]) for l in range(len(widths) - 1)]
    parts += [rng.normal(0, 0.1, widths[l + 1]) for l in range(len(widths) - 1)]
    return np.concatenate(parts)


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 1, 2000), rng.normal(0, 1e-3, 500) * 10.0 ** rng.integers(-40, 38, 500),
                        np.array([1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -(1.0 + 2 ** -8), 1e-40, -3e-39, 0.0])])
    x = x.astype(np.float32).astype(np.float64)  # torch converts from float32
    want = torch.tensor(x, dtype=torch.float32).to(torch.bfloat16).double().numpy()
    np.testing.assert_array_equal(oracle.bf16(x), want)


def test_gelu_closed_forms():
    # gelu(z) = z Phi(z): Phi(1) and Phi(2) are textbook values of the
    # standard normal distribution function
    assert oracle.gelu(0.0) == 0.0
    assert oracle.gelu(1.0) == pytest.approx(0.8413447460685429, rel=1e-14)
    assert oracle.gelu(2.0) == pytest.approx(2 * 0.9772498680518208, rel=1e-14)
    # Phi(z) + Phi(-z) = 1  =>  gelu(z) - gelu(-z) = z
    for z in (-3.1, -0.4, 0.7, 5.0):
        assert oracle.gelu(z) - oracle.gelu(-z) == pytest.approx(z, rel=1e-14)
    # derivative: gelu'(0) = 1/2; central differences elsewhere
    assert oracle.gelu_prime(0.0) == 0.5
    h = 1e-6
    for z in (-2.3, -0.5, 0.3, 1.9):
        fd = (oracle.gelu(z + h) - oracle.gelu(z - h)) / (2 * h)
        assert oracle.gelu_prime(z) == pytest.approx(fd, abs=1e-9)


def test_single_layer_is_affine_map():
    rng = np.random.default_rng(1)
    w = [7, 5]
    p = _params(w, rng)
    X = rng.normal(0, 1, (9, 7))
    W, b = p[:35].reshape(7, 5), p[35:]
    np.testing.assert_allclose(oracle.mlp_forward(w, p, X, quant=False), X @ W + b, rtol=1e-13, atol=1e-13)
    # with BF16 rounding, the product is that of the rounded operands
    Wq = torch.tensor(W, dtype=torch.float32).to(torch.bfloat16).double().numpy()
    Xq = torch.tensor(X, dtype=torch.float32).to(torch.bfloat16).double().numpy()
    np.testing.assert_allclose(oracle.mlp_forward(w, p, X.astype(np.float32).astype(np.float64), quant=True),
                               Xq @ Wq + b, rtol=1e-13, atol=1e-13)


def test_two_layer_network_by_hand():
    # widths 2 -> 3 -> 1, small enough to write the network out with the
    # normal distribution function from math.erf
    rng = np.random.default_rng(2)
    w = [2, 3, 1]
    p = _params(w, rng)
    W0, W1 = p[:6].reshape(2, 3), p[6:9].reshape(3, 1)
    b0, b1 = p[9:12], p[12:13]
    X = rng.normal(0, 1, (4, 2))

    def gelu(z):
        return z * 0.5 * (1 + math.erf(z / math.sqrt(2)))

    want = np.array([[sum(gelu(X[m] @ W0[:, j] + b0[j]) * W1[j, 0] for j in range(3)) + b1[0]] for m in range(4)])
    np.testing.assert_allclose(oracle.mlp_forward(w, p, X, quant=False), want, rtol=1e-13)


@pytest.mark.parametrize("widths", [[5, 7, 6, 3], [4, 9, 2]])
def test_gradient_matches_finite_differences(widths):
    rng = np.random.default_rng(3)
    p = _params(widths, rng)
    X = rng.normal(0, 1, (6, widths[0]))
    T = rng.normal(0, 1, (6, widths[-1]))
    loss, g = oracle.mlp_loss_grad(widths, p, X, T, quant=False)
    Y = oracle.mlp_forward(widths, p, X, quant=False)
    assert loss == pytest.approx(np.mean((Y - T) ** 2), rel=1e-14)
    h = 1e-6
    for i in range(p.size):  # every weight and bias of every layer
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        fd = (oracle.mlp_loss_grad(widths, pp, X, T, quant=False)[0] -
              oracle.mlp_loss_grad(widths, pm, X, T, quant=False)[0]) / (2 * h)
        assert g[i] == pytest.approx(fd, abs=1e-8, rel=1e-6), i


def test_gradient_vanishes_at_exact_fit():
    rng = np.random.default_rng(4)
    w = [3, 6, 2]
    p = _params(w, rng)
    X = rng.normal(0, 1, (5, 3))
    T = oracle.mlp_forward(w, p, X, quant=False)
    loss, g = oracle.mlp_loss_grad(w, p, X, T, quant=False)
    assert loss == 0.0 and np.all(g == 0.0)


def test_quantised_gradient_is_close_to_exact():
    # the BF16 rounding points perturb the gradient by about the BF16 unit
    # roundoff (2^-9) relative, far from a sign or index error
    rng = np.random.default_rng(5)
    w = [8, 16, 16, 4]
    p = _params(w, rng)
    X = rng.normal(0, 1, (32, 8))
    T = rng.normal(0, 1, (32, 4))
    _, g0 = oracle.mlp_loss_grad(w, p, X, T, quant=False)
    _, g1 = oracle.mlp_loss_grad(w, p, X, T, quant=True)
    err = np.abs(g1 - g0).max() / np.abs(g0).max()
    assert 0 < err < 0.03


def test_adam_closed_forms():
    rng = np.random.default_rng(6)
    n = 50
    g = rng.normal(0, 1, n) * 10.0 ** rng.integers(-3, 3, n)
    lr, eps = 1e-3, 1e-8
    p = rng.normal(0, 1, n)
    p0 = p.copy()
    m, v = np.zeros(n), np.zeros(n)
    # with a constant gradient the bias-corrected moments are g and g^2
    # after every step, so each step moves by lr g / (|g| + eps)
    for t in range(1, 6):
        oracle.adam(p, g, m, v, t, lr, eps=eps)
        np.testing.assert_allclose(p, p0 - t * lr * g / (np.abs(g) + eps), rtol=0, atol=1e-15)
    # a zero gradient from a zero state changes nothing
    q = p.copy()
    oracle.adam(q, np.zeros(n), np.zeros(n), np.zeros(n), 1, lr)
    np.testing.assert_array_equal(q, p)
