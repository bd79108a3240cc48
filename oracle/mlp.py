"""CPU oracle of the order network (test infrastructure only).

The per-interaction order policy uses a small network: 8 features -> 64 ReLU
-> 64 ReLU -> 1, weights in one flat array (W1 [64][8], b1, W2 [64][64], b2,
w3 [64], b3), trained on the loss mean(w(r) r^2), r = y - label, w = 4 for
r < 0 else 1.  This module is the plain FP64 reference of its forward pass,
its loss and the gradient by hand-written backpropagation, and an emulation
of the bfloat16 inference (weights, inputs and hidden activations rounded to
bfloat16, FP32 sums).  It shares no code with the GPU kernels.
"""
import numpy as np

IN, HID = 8, 64
NW = HID * IN + HID + HID * HID + HID + HID + 1
UNDER = 4.0


def unpack(w):
    w = np.asarray(w, dtype=np.float64)
    assert w.shape == (NW,)
    o = 0
    W1 = w[o:o + HID * IN].reshape(HID, IN); o += HID * IN
    b1 = w[o:o + HID]; o += HID
    W2 = w[o:o + HID * HID].reshape(HID, HID); o += HID * HID
    b2 = w[o:o + HID]; o += HID
    w3 = w[o:o + HID]; o += HID
    b3 = w[o]
    return W1, b1, W2, b2, w3, b3


def forward(w, f):
    """y [n] for features f [n][8]; also returns the activations."""
    W1, b1, W2, b2, w3, b3 = unpack(w)
    f = np.asarray(f, dtype=np.float64)
    z1 = f @ W1.T + b1
    h1 = np.maximum(z1, 0.0)
    z2 = h1 @ W2.T + b2
    h2 = np.maximum(z2, 0.0)
    y = h2 @ w3 + b3
    return y, (f, z1, h1, z2, h2)


def loss(w, f, label):
    y, _ = forward(w, f)
    r = y - np.asarray(label, dtype=np.float64)
    return float(np.mean(np.where(r < 0, UNDER, 1.0) * r * r))


def grad(w, f, label):
    """Gradient of loss() by backpropagation, in the flat weight layout."""
    W1, b1, W2, b2, w3, b3 = unpack(w)
    y, (f, z1, h1, z2, h2) = forward(w, f)
    n = f.shape[0]
    r = y - np.asarray(label, dtype=np.float64)
    g = 2.0 * np.where(r < 0, UNDER, 1.0) * r / n          # dL/dy per sample
    d2 = np.outer(g, w3) * (z2 > 0)                       # dL/dz2
    d1 = (d2 @ W2) * (z1 > 0)                             # dL/dz1
    return np.concatenate([(d1.T @ f).ravel(), d1.sum(0), (d2.T @ h1).ravel(), d2.sum(0),
                           h2.T @ g, [g.sum()]])


def bf16(x):
    """Round FP32 values to bfloat16 (nearest, ties to even), as FP32."""
    u = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32)


def forward_bf16(w, f):
    """Inference with bfloat16 weights, inputs and hidden activations and
    sums in FP64 (the GPU sums in FP32: agreement to ~1e-6 relative)."""
    wb = bf16(np.asarray(w, np.float32)).astype(np.float64)
    W1, b1, W2, b2, w3, b3 = unpack(wb)
    fb = bf16(np.asarray(f, np.float32)).astype(np.float64)
    h1 = bf16(np.maximum(fb @ W1.T + b1, 0.0).astype(np.float32)).astype(np.float64)
    h2 = bf16(np.maximum(h1 @ W2.T + b2, 0.0).astype(np.float32)).astype(np.float64)
    return h2 @ w3 + b3
