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


def _bf16_torch(x):
    """bfloat16 rounding by torch's own conversion (round to nearest even),
    a second implementation next to the oracle's bit manipulation."""
    import torch
    return float(torch.tensor(float(x), dtype=torch.float32).to(torch.bfloat16).to(torch.float32))


def test_forward_bf16_written_out():
    """The bfloat16 inference written out per unit: every weight and bias,
    every input feature and both hidden layers' activations (after the ReLU)
    rounded to bfloat16; the sums themselves exact (FP64 here)."""
    w, f, _ = _setup(seed=8, n=3)
    w = w.astype(np.float32)
    f = f.astype(np.float32)
    y = mlp.forward_bf16(w, f)
    wb = [_bf16_torch(v) for v in w]
    W1, b1, W2, b2, w3, b3 = mlp.unpack(np.array(wb))
    for s in range(3):
        x = [_bf16_torch(f[s, j]) for j in range(mlp.IN)]
        h1 = [_bf16_torch(np.float32(max(0.0, sum(W1[i, j] * x[j] for j in range(mlp.IN)) + b1[i])))
              for i in range(mlp.HID)]
        h2 = [_bf16_torch(np.float32(max(0.0, sum(W2[i, j] * h1[j] for j in range(mlp.HID)) + b2[i])))
              for i in range(mlp.HID)]
        ys = sum(w3[i] * h2[i] for i in range(mlp.HID)) + b3
        assert abs(ys - y[s]) <= 1e-6 * max(1.0, abs(ys)), s


def test_forward_bf16_rounds_where_stated():
    """Hand-built networks whose output shows each rounding on its own:
    1 + 2^-9 is not a bfloat16 value and rounds to 1, 1 + 2^-7 is one."""
    e9, e7 = 2.0 ** -9, 2.0 ** -7

    def net(w1=1.0, b1=0.0, w2=1.0, b2=0.0, w3=1.0, b3=0.0):
        w = np.zeros(mlp.NW, np.float32)
        W1, bb1, W2, bb2, ww3, _ = (0, mlp.HID * mlp.IN, mlp.HID * mlp.IN + mlp.HID,
                                    mlp.HID * mlp.IN + mlp.HID + mlp.HID * mlp.HID,
                                    mlp.HID * mlp.IN + 2 * mlp.HID + mlp.HID * mlp.HID, 0)
        w[W1] = w1           # unit 0 of layer 1 reads feature 0
        w[bb1] = b1
        w[W2] = w2           # unit 0 of layer 2 reads unit 0 of layer 1
        w[bb2] = b2
        w[ww3] = w3          # the output reads unit 0 of layer 2
        w[-1] = b3
        return w

    f = np.zeros((1, mlp.IN), np.float32)
    f[0, 0] = 1.0
    # exact values pass through unchanged
    assert mlp.forward_bf16(net(), f)[0] == 1.0
    # a weight of 1 + 2^-9 (rounded to 1) in each layer
    for k in ("w1", "w2", "w3"):
        assert mlp.forward_bf16(net(**{k: 1.0 + e9}), f)[0] == 1.0, k
        assert mlp.forward_bf16(net(**{k: 1.0 + e7}), f)[0] == 1.0 + e7, k
    # the input feature is rounded
    f2 = f.copy()
    f2[0, 0] = 1.0 + e9
    assert mlp.forward_bf16(net(), f2)[0] == 1.0
    # the hidden activations are rounded after the bias: 1 + 2^-8 + 2^-9 is
    # not exact, the first layer's output rounds to 1 + 2^-7 (nearest)
    y = mlp.forward_bf16(net(b1=2.0 ** -8 + e9), f)[0]
    assert y == 1.0 + e7
    # the same through the second layer's bias
    y = mlp.forward_bf16(net(b2=2.0 ** -8 + e9), f)[0]
    assert y == 1.0 + e7
    # the output bias is rounded as a weight but the output sum is not
    y = mlp.forward_bf16(net(b3=e7), f)[0]
    assert y == 1.0 + e7
