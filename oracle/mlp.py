"""Float64 reference of the parameter-selector network.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``). The paper has no
learned component, so nothing here is pinned by it ("parity unpinned" by the
paper); the tests pin this module by central finite differences of the loss,
closed forms (zero weights, a single labelled output) and the first Adam
steps written out by hand.

Network: 16 inputs -> 64 ReLU -> 64 ReLU -> C linear outputs (C = 64), one
predicted cost per candidate parameter triple. Parameters are one flat
vector, in this order: W1 [64][16], b1 [64], W2 [64][64], b2 [64], W3 [C][64],
b3 [C] (row-major, rows are output units).

Loss of a batch: the mean over the labelled (sample, candidate) entries of
the squared error, ``sum_{b,c} M[b,c] (Y[b,c] - T[b,c])^2 / sum M``.

Adam (Kingma & Ba): m <- b1 m + (1-b1) g; v <- b2 v + (1-b2) g^2;
p <- p - lr * (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps).
"""

from __future__ import annotations

import numpy as np

N_IN = 16
N_HID = 64
N_OUT = 64


def param_count(C: int = N_OUT) -> int:
    return N_HID * N_IN + N_HID + N_HID * N_HID + N_HID + C * N_HID + C


def unpack(params: np.ndarray, C: int = N_OUT):
    p = np.asarray(params, dtype=np.float64)
    assert p.size == param_count(C)
    o = 0
    W1 = p[o:o + N_HID * N_IN].reshape(N_HID, N_IN); o += N_HID * N_IN
    b1 = p[o:o + N_HID]; o += N_HID
    W2 = p[o:o + N_HID * N_HID].reshape(N_HID, N_HID); o += N_HID * N_HID
    b2 = p[o:o + N_HID]; o += N_HID
    W3 = p[o:o + C * N_HID].reshape(C, N_HID); o += C * N_HID
    b3 = p[o:o + C]; o += C
    return W1, b1, W2, b2, W3, b3


def pack(W1, b1, W2, b2, W3, b3) -> np.ndarray:
    return np.concatenate([np.ravel(a) for a in (W1, b1, W2, b2, W3, b3)]).astype(np.float64)


def init_params(rng: np.random.Generator, C: int = N_OUT) -> np.ndarray:
    """He-normal weights, zero biases."""
    W1 = rng.normal(0.0, np.sqrt(2.0 / N_IN), (N_HID, N_IN))
    W2 = rng.normal(0.0, np.sqrt(2.0 / N_HID), (N_HID, N_HID))
    W3 = rng.normal(0.0, np.sqrt(1.0 / N_HID), (C, N_HID))
    return pack(W1, np.zeros(N_HID), W2, np.zeros(N_HID), W3, np.zeros(C))


def forward(params, X, C: int = N_OUT):
    """Outputs [B, C] and the activations the backward pass needs."""
    W1, b1, W2, b2, W3, b3 = unpack(params, C)
    X = np.asarray(X, dtype=np.float64)
    Z1 = X @ W1.T + b1
    H1 = np.maximum(Z1, 0.0)
    Z2 = H1 @ W2.T + b2
    H2 = np.maximum(Z2, 0.0)
    Y = H2 @ W3.T + b3
    return Y, (X, Z1, H1, Z2, H2)


def loss(params, X, T, M, C: int = N_OUT) -> float:
    Y, _ = forward(params, X, C)
    M = np.asarray(M, dtype=np.float64)
    n = M.sum()
    if n == 0:
        return 0.0
    return float((M * (Y - np.asarray(T, dtype=np.float64)) ** 2).sum() / n)


def loss_and_grad(params, X, T, M, C: int = N_OUT):
    """Loss and its gradient with respect to the flat parameter vector, by
    the chain rule through the three layers (ReLU derivative: 1 where the
    pre-activation is positive, else 0)."""
    W1, b1, W2, b2, W3, b3 = unpack(params, C)
    Y, (X, Z1, H1, Z2, H2) = forward(params, X, C)
    M = np.asarray(M, dtype=np.float64)
    n = M.sum()
    if n == 0:
        return 0.0, np.zeros(param_count(C))
    R = M * (Y - np.asarray(T, dtype=np.float64))
    L = float((R * (Y - np.asarray(T, dtype=np.float64))).sum() / n)
    dY = 2.0 * R / n                       # [B, C]
    dW3 = dY.T @ H2
    db3 = dY.sum(axis=0)
    dH2 = dY @ W3
    dZ2 = dH2 * (Z2 > 0)
    dW2 = dZ2.T @ H1
    db2 = dZ2.sum(axis=0)
    dH1 = dZ2 @ W2
    dZ1 = dH1 * (Z1 > 0)
    dW1 = dZ1.T @ X
    db1 = dZ1.sum(axis=0)
    return L, pack(dW1, db1, dW2, db2, dW3, db3)


def adam_step(params, grad, m, v, t: int, lr: float, beta1: float = 0.9,
              beta2: float = 0.999, eps: float = 1e-8):
    """One Adam update at step t (1-based); returns (params, m, v)."""
    g = np.asarray(grad, dtype=np.float64)
    m = beta1 * np.asarray(m, dtype=np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, dtype=np.float64) + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** t)
    vhat = v / (1.0 - beta2 ** t)
    p = np.asarray(params, dtype=np.float64) - lr * mhat / (np.sqrt(vhat) + eps)
    return p, m, v


def select(params, X, feasible, C: int = N_OUT) -> np.ndarray:
    """Per sample the feasible candidate with the smallest predicted cost
    (ties to the lowest index), -1 when none is feasible."""
    Y, _ = forward(params, X, C)
    F = np.asarray(feasible, dtype=bool)
    Yf = np.where(F, Y, np.inf)
    pick = np.argmin(Yf, axis=1)
    pick[~F.any(axis=1)] = -1
    return pick
