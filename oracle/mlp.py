"""FP64 reference of the learned warm-start network (TEST INFRASTRUCTURE ONLY).

The network maps theta (8 parameters of the matrix family) to the n^2 entries of the
sign-canonicalised eigenvector matrix: 8 -> 1024 -> ReLU -> 1024 -> ReLU -> n^2.  The GPU
implementation computes every matrix product with bfloat16 operands and FP32 accumulation; this
reference follows the same precision model -- every product operand is rounded to bfloat16
(round to nearest even, from the value rounded to FP32 first) -- and does everything else in FP64.
With bf16=False all rounding is switched off, which the finite-difference pins use.

Loss: mean squared error over all B * n^2 outputs.  Optimiser: AdamW with decoupled weight decay
(Loshchilov & Hutter):  m = b1 m + (1 - b1) g,  v = b2 v + (1 - b2) g^2,
p -= lr (m / (1 - b1^t) / (sqrt(v / (1 - b2^t)) + eps) + wd p).
Parameters are packed as [W1 (H x I), b1 (H), W2 (H x H), b2 (H), W3 (O x H), b3 (O)], row-major.
"""
from __future__ import annotations

import numpy as np


def bf16(x: np.ndarray) -> np.ndarray:
    """Round to bfloat16 (via FP32, nearest even) and return as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


def shapes(I: int, H: int, O: int):
    return [(H, I), (H,), (H, H), (H,), (O, H), (O,)]


def unpack(p: np.ndarray, I: int, H: int, O: int):
    out, o = [], 0
    for s in shapes(I, H, O):
        k = int(np.prod(s))
        out.append(p[o:o + k].reshape(s))
        o += k
    return out


def forward(p, X, I, H, O, use_bf16=True):
    r = bf16 if use_bf16 else (lambda a: np.asarray(a, np.float64))
    W1, b1, W2, b2, W3, b3 = unpack(np.asarray(p, np.float64), I, H, O)
    Xb = r(X)
    Z1 = Xb @ r(W1).T + b1
    H1 = np.maximum(Z1, 0.0)
    Z2 = r(H1) @ r(W2).T + b2
    H2 = np.maximum(Z2, 0.0)
    Y = r(H2) @ r(W3).T + b3
    return Y, (Xb, Z1, H1, Z2, H2)


def loss_and_grads(p, X, T, I, H, O, use_bf16=True):
    """Mean squared error and its gradient with respect to the packed parameters."""
    r = bf16 if use_bf16 else (lambda a: np.asarray(a, np.float64))
    W1, b1, W2, b2, W3, b3 = unpack(np.asarray(p, np.float64), I, H, O)
    Y, (Xb, Z1, H1, Z2, H2) = forward(p, X, I, H, O, use_bf16)
    B = X.shape[0]
    D = Y - np.asarray(T, np.float64)
    loss = float(np.mean(D * D))
    dY = 2.0 * D / (B * O)
    dW3 = r(dY).T @ r(H2)
    db3 = dY.sum(0)
    dH2 = r(dY) @ r(W3)
    dZ2 = dH2 * (Z2 > 0)
    dW2 = r(dZ2).T @ r(H1)
    db2 = dZ2.sum(0)
    dH1 = r(dZ2) @ r(W2)
    dZ1 = dH1 * (Z1 > 0)
    dW1 = r(dZ1).T @ Xb
    db1 = dZ1.sum(0)
    g = np.concatenate([a.ravel() for a in (dW1, db1, dW2, db2, dW3, db3)])
    return loss, g


def adamw(p, g, m, v, t, lr, wd, b1=0.9, b2=0.999, eps=1e-8):
    """One AdamW step (t counts from 1); returns new (p, m, v)."""
    m = b1 * m + (1 - b1) * g
    v = b2 * v + (1 - b2) * g * g
    mh = m / (1 - b1 ** t)
    vh = v / (1 - b2 ** t)
    p = p - lr * (mh / (np.sqrt(vh) + eps) + wd * p)
    return p, m, v


def canonical_signs(V: np.ndarray) -> np.ndarray:
    """Sign convention of the training targets: in every column the entry of largest magnitude
    (the first one on ties) is made positive."""
    V = np.array(V, dtype=np.float64, copy=True)
    idx = np.argmax(np.abs(V), axis=0)
    s = np.sign(V[idx, np.arange(V.shape[1])])
    s[s == 0] = 1.0
    return V * s[None, :]
