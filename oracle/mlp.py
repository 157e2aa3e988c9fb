"""Plain FP64 reference of the learned sampler's network (TEST INFRASTRUCTURE ONLY: used
by tests/ to check the library's forward pass, gradients and training data; never by the
product package).

The network is a perceptron 4 -> 128 -> 128 -> 128 -> 3 with SiLU(z) = z / (1 + e^-z)
after each hidden layer.  It maps the normalised inputs of an NCS emission to the
normalised outputs of the sampler:

    x0 = (log10 chi + 0.65) / 2.35      (chi in [1e-3, 50]  ->  x0 in [-1, 1])
    x1 = S.b,  x2 = S.n                  (spin components in the local frame)
    x3 = 2 r - 1                         (the energy draw r in (0, 1))
    y0 = t / 40^(1/3),  y1 = mean xi3,  y2 = mean xi2

Parameters are one flat vector: W1 (4 x 128, row = input), b1, W2 (128 x 128), b2, W3,
b3, W4 (128 x 3), b4 -- 34,051 numbers.  The loss of a batch is
(1/B) sum_i sum_o w_o (y_io - target_io)^2.  Everything here is the textbook definition
(matrix products, chain rule) written out; nothing is fused or reordered.
"""
from __future__ import annotations

import numpy as np

SIZES = [(4, 128), (128, 128), (128, 128), (128, 3)]
N_PARAMS = sum(i * o + o for i, o in SIZES)
T_MAX = 40.0 ** (1.0 / 3.0)


def unpack(theta: np.ndarray):
    """Flat parameter vector -> [(W, b), ...] (views)."""
    out, k = [], 0
    for i, o in SIZES:
        W = theta[k:k + i * o].reshape(i, o)
        k += i * o
        b = theta[k:k + o]
        k += o
        out.append((W, b))
    assert k == len(theta) == N_PARAMS
    return out


def normalise_inputs(chi, s, c, r) -> np.ndarray:
    chi, s, c, r = (np.asarray(v, dtype=np.float64) for v in (chi, s, c, r))
    return np.stack([(np.log10(chi) + 0.65) / 2.35, s, c, 2.0 * r - 1.0], axis=1)


def normalise_targets(T: np.ndarray) -> np.ndarray:
    """[n, 3] (t, xi3, xi2) -> network outputs."""
    return np.stack([T[:, 0] / T_MAX, T[:, 1], T[:, 2]], axis=1)


def silu(z):
    return z / (1.0 + np.exp(-z))


def silu_prime(z):
    sg = 1.0 / (1.0 + np.exp(-z))
    return sg * (1.0 + z * (1.0 - sg))


def forward(theta: np.ndarray, X: np.ndarray):
    """Outputs [n, 3] and the per-layer pre-activations / activations for backward."""
    layers = unpack(np.asarray(theta, dtype=np.float64))
    h = np.asarray(X, dtype=np.float64)
    hs, zs = [h], []
    for k, (W, b) in enumerate(layers):
        z = h @ W + b
        zs.append(z)
        h = silu(z) if k < len(layers) - 1 else z
        hs.append(h)
    return h, (hs, zs)


def loss_and_grad(theta: np.ndarray, X: np.ndarray, Y: np.ndarray, w=(1.0, 1.0, 1.0)):
    """Loss and its gradient with respect to the flat parameters (backpropagation)."""
    layers = unpack(np.asarray(theta, dtype=np.float64))
    out, (hs, zs) = forward(theta, X)
    B = X.shape[0]
    w = np.asarray(w, dtype=np.float64)
    diff = out - Y
    loss = float(np.sum(w * diff * diff) / B)
    delta = 2.0 * w * diff / B                 # dL/dz of the last layer
    grads = []
    for k in range(len(layers) - 1, -1, -1):
        W, _ = layers[k]
        gW = hs[k].T @ delta
        gb = delta.sum(axis=0)
        grads.append((gW, gb))
        if k > 0:
            delta = (delta @ W.T) * silu_prime(zs[k - 1])
    flat = []
    for gW, gb in reversed(grads):
        flat.append(gW.ravel())
        flat.append(gb)
    return loss, np.concatenate(flat)


def bf16_round(a: np.ndarray) -> np.ndarray:
    """Round to the nearest bfloat16 (ties to even), returned as float64."""
    f = np.asarray(a, dtype=np.float32).copy()
    u = f.view(np.uint32)
    u = (u + np.uint32(0x7FFF) + ((u >> np.uint32(16)) & np.uint32(1))) & np.uint32(0xFFFF0000)
    return u.view(np.float32).astype(np.float64)


def forward_bf16(theta: np.ndarray, X: np.ndarray) -> np.ndarray:
    """The same network with the two 128 x 128 weight matrices and the inputs of layers
    2, 3 and 4 rounded to bfloat16 (the storage precision of a matrix-core forward pass);
    every product and sum in FP64."""
    layers = unpack(np.asarray(theta, dtype=np.float64))
    h = np.asarray(X, dtype=np.float64)
    for k, (W, b) in enumerate(layers):
        if k > 0:
            h = bf16_round(h)
        if k in (1, 2):
            W = bf16_round(W)
        z = h @ W + b
        h = silu(z) if k < len(layers) - 1 else z
    return h

