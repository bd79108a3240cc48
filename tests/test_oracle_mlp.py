"""Pins of the order-network oracle: its gradient against central finite
differences of its loss, its forward pass against the formula written out
per unit, and the bfloat16 rounding against hand-checked cases."""
import numpy as np

from oracle import mlp


def _setup(seed=3, n=40):
    rng = np.random.default_rng(seed)
    w = rng.normal(0, 0.3, mlp.NW)
    f = rng.normal(0, 1, (n, mlp.IN))
    lab = rng.uniform(4, 40, n)
    return w, f, lab


def test_gradient_matches_finite_differences():
    w, f, lab = _setup()
    g = mlp.grad(w, f, lab)
    rng = np.random.default_rng(0)
    for k in list(rng.choice(mlp.NW, 60, replace=False)) + [mlp.NW - 1, 0, 511, 512]:
        h = 1e-6 * max(1.0, abs(w[k]))
        wp, wm = w.copy(), w.copy()
        wp[k] += h
        wm[k] -= h
        fd = (mlp.loss(wp, f, lab) - mlp.loss(wm, f, lab)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])), k


def test_forward_written_out():
    w, f, lab = _setup(n=3)
    y, _ = mlp.forward(w, f)
    W1, b1, W2, b2, w3, b3 = mlp.unpack(w)
    for s in range(3):
        h1 = [max(0.0, sum(W1[i, j] * f[s, j] for j in range(mlp.IN)) + b1[i]) for i in range(mlp.HID)]
        h2 = [max(0.0, sum(W2[i, j] * h1[j] for j in range(mlp.HID)) + b2[i]) for i in range(mlp.HID)]
        ys = sum(w3[i] * h2[i] for i in range(mlp.HID)) + b3
        assert abs(ys - y[s]) <= 1e-12 * max(1.0, abs(ys))


def test_bf16_rounding_cases():
    one = np.float32(1.0)
    cases = {
        1.0: 1.0,
        1.0 + 2.0 ** -8: 1.0,                  # halfway, ties to even (down)
        1.0 + 3 * 2.0 ** -8: 1.0 + 2.0 ** -6,  # halfway, ties to even (up)
        1.0 + 2.0 ** -7: 1.0 + 2.0 ** -7,      # representable
        -2.5: -2.5,
        3.0e-3: 0.0030059814453125,
    }
    for x, want in cases.items():
        assert float(mlp.bf16(np.float32(x))) == want, x
    assert mlp.bf16(one).dtype == np.float32
