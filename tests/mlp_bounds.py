"""Per-element error bounds for the network's GPU arithmetic (test helper).

The GPU network rounds every product operand to bfloat16 and accumulates the products in FP32; the
reference (oracle/mlp.py) rounds the same operands and accumulates in FP64.  Two things separate
the two results entry by entry:

* FP32 accumulation: a K-term sum of exact products (bfloat16 x bfloat16 is exact in FP32) plus a
  bias, accumulated in any order and stored in FP32, is within (K + 4) u sum |terms| of the exact
  sum, u = 2^-24 (the standard gamma_K bound, with slack for the split-K slice sum and the store).
* Operand rounding: a GPU intermediate x_g within e of the reference value x_r may round to a
  different bfloat16 value.  Rounding is monotone, so bf16(x_g) and bf16(x_r) both lie in
  [bf16(x_r - e), bf16(x_r + e)]; that interval's width bounds their difference (zero whenever no
  rounding boundary lies within e of x_r, which is the usual case).
* ReLU masks: where |z_r| <= e the GPU's mask may differ from the reference's, and the masked
  value may differ by its whole size.

The functions below carry these bounds through the forward pass and the backward pass layer by
layer, so that every output and every gradient entry is compared against its own bound.
"""
from __future__ import annotations

import numpy as np

from oracle import mlp as ref

U32 = 2.0 ** -24


def _gamma(k: int) -> float:
    return (k + 4) * U32


def _flip(x: np.ndarray, e: np.ndarray) -> np.ndarray:
    """Largest possible |bf16(x_g) - bf16(x)| for any x_g with |x_g - x| <= e."""
    e = e + 2 * U32 * np.abs(x)          # the GPU rounds from its FP32 value
    return ref.bf16(x + e) - ref.bf16(x - e)


def forward(p, X, I, H, O):
    """Reference forward pass (bfloat16 operands, FP64 sums) with per-element bounds of the GPU's
    deviation for every intermediate.  Returns a dict of reference values and bounds."""
    W1, b1, W2, b2, W3, b3 = ref.unpack(np.asarray(p, np.float64), I, H, O)
    r = ref.bf16
    Xb, W1b, W2b, W3b = r(X), r(W1), r(W2), r(W3)
    aW1, aW2, aW3 = np.abs(W1b), np.abs(W2b), np.abs(W3b)
    Z1 = Xb @ W1b.T + b1
    eZ1 = _gamma(I) * (np.abs(Xb) @ aW1.T + np.abs(b1))
    H1 = np.maximum(Z1, 0.0)
    H1b = r(H1)
    d1 = _flip(H1, eZ1)
    Z2 = H1b @ W2b.T + b2
    eZ2 = d1 @ aW2.T + _gamma(H) * ((np.abs(H1b) + d1) @ aW2.T + np.abs(b2))
    H2 = np.maximum(Z2, 0.0)
    H2b = r(H2)
    d2 = _flip(H2, eZ2)
    Y = H2b @ W3b.T + b3
    eY = d2 @ aW3.T + _gamma(H) * ((np.abs(H2b) + d2) @ aW3.T + np.abs(b3))
    return dict(Xb=Xb, W1b=W1b, W2b=W2b, W3b=W3b, Z1=Z1, eZ1=eZ1, H1=H1, H1b=H1b, d1=d1, Z2=Z2, eZ2=eZ2,
                H2=H2, H2b=H2b, d2=d2, Y=Y, eY=eY)


def _outer_bound(A, dA, B, dB, k):
    """Bound of |bf(A_g)^T bf(B_g) - bf(A)^T bf(B)| (entry-wise, summing over the k rows) plus the
    FP32 accumulation of the GPU's product; A, B are the bfloat16-rounded reference operands."""
    aA, aB = np.abs(A), np.abs(B)
    return dA.T @ aB + aA.T @ dB + dA.T @ dB + _gamma(k) * ((aA + dA).T @ (aB + dB))


def grads(p, X, T, I, H, O):
    """Reference loss and gradient (as oracle/mlp.py computes them) with a per-element bound of the
    GPU's deviation for every gradient entry, packed like the parameters, and for the loss."""
    f = forward(p, X, I, H, O)
    B = X.shape[0]
    r = ref.bf16
    T = np.asarray(T, np.float64)
    scale = 2.0 / (B * O)
    D = f["Y"] - T
    loss = float(np.mean(D * D))
    eD = f["eY"] + 2 * U32 * (np.abs(f["Y"]) + np.abs(T))
    eloss = (2 * np.abs(D) * eD + eD * eD).sum() / (B * O) + _gamma(B * O) * loss
    dY = scale * D
    edY = scale * eD + 2 * U32 * np.abs(dY)
    dYb = r(dY)
    ddY = _flip(dY, edY)
    # output layer
    gW3 = dYb.T @ f["H2b"]
    egW3 = _outer_bound(dYb, ddY, f["H2b"], f["d2"], B)
    gb3 = dY.sum(0)
    egb3 = edY.sum(0) + _gamma(B) * np.abs(dY).sum(0)
    aW3 = np.abs(f["W3b"])
    dH2 = dYb @ f["W3b"]
    edH2 = ddY @ aW3 + _gamma(O) * ((np.abs(dYb) + ddY) @ aW3)
    mask2 = f["Z2"] > 0
    unsure2 = np.abs(f["Z2"]) <= f["eZ2"]
    dZ2 = dH2 * mask2
    edZ2 = np.where(unsure2, np.abs(dH2) + edH2, edH2 * mask2)
    # hidden layer 2
    dZ2b = r(dZ2)
    ddZ2 = _flip(dZ2, edZ2)
    gW2 = dZ2b.T @ f["H1b"]
    egW2 = _outer_bound(dZ2b, ddZ2, f["H1b"], f["d1"], B)
    gb2 = dZ2.sum(0)
    egb2 = edZ2.sum(0) + _gamma(B) * np.abs(dZ2).sum(0)
    aW2 = np.abs(f["W2b"])
    dH1 = dZ2b @ f["W2b"]
    edH1 = ddZ2 @ aW2 + _gamma(H) * ((np.abs(dZ2b) + ddZ2) @ aW2)
    mask1 = f["Z1"] > 0
    unsure1 = np.abs(f["Z1"]) <= f["eZ1"]
    dZ1 = dH1 * mask1
    edZ1 = np.where(unsure1, np.abs(dH1) + edH1, edH1 * mask1)
    # first layer (X is rounded identically on both sides)
    dZ1b = r(dZ1)
    ddZ1 = _flip(dZ1, edZ1)
    gW1 = dZ1b.T @ f["Xb"]
    egW1 = _outer_bound(dZ1b, ddZ1, f["Xb"], np.zeros_like(f["Xb"]), B)
    gb1 = dZ1.sum(0)
    egb1 = edZ1.sum(0) + _gamma(B) * np.abs(dZ1).sum(0)
    g = np.concatenate([a.ravel() for a in (gW1, gb1, gW2, gb2, gW3, gb3)])
    eg = np.concatenate([a.ravel() for a in (egW1, egb1, egW2, egb2, egW3, egb3)])
    return loss, eloss, g, eg


def adamw_bound(p, m, v, g, t, lr, wd, b1, b2, eps, ep, em, ev):
    """One AdamW step in FP64 (oracle/mlp.py) and the per-element bound of an FP32 evaluation of
    the same step, given bounds ep, em, ev of the FP32 state going in (the gradient g is the same
    on both sides).  Each FP32 operation adds at most u of its result; the FP32 constants b1, b2,
    lr, wd, eps and the bias corrections add at most u relative each."""
    pn, mn, vn = ref.adamw(p, g, m, v, t, lr, wd, b1=b1, b2=b2, eps=eps)
    em_n = b1 * em + 6 * U32 * (b1 * np.abs(m) + (1 - b1) * np.abs(g))
    ev_n = b2 * ev + 6 * U32 * (b2 * np.abs(v) + (1 - b2) * g * g)
    c1, c2 = 1.0 / (1 - b1 ** t), 1.0 / (1 - b2 ** t)
    num = mn * c1
    sq = np.sqrt(vn * c2)
    den = sq + eps
    e_num = c1 * em_n + 4 * U32 * np.abs(num)
    e_sq = np.where(sq > 0, c2 * ev_n / (2 * np.maximum(sq, 1e-300)), np.sqrt(c2 * ev_n)) + 4 * U32 * sq
    e_den = e_sq + 2 * U32 * den
    upd = num / den
    e_upd = e_num / den + np.abs(num) * e_den / (den * (den - e_den).clip(min=den * 0.5)) + 2 * U32 * np.abs(upd)
    ep_n = ep * (1 + lr * wd) + lr * e_upd + 6 * U32 * (np.abs(p) + lr * np.abs(upd) + lr * wd * np.abs(p))
    return pn, mn, vn, ep_n, em_n, ev_n
