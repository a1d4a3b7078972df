"""The per-element bounds of tests/mlp_bounds.py, checked on the CPU against an FP32 emulation of the
GPU network's arithmetic (bfloat16 operands, FP32 sums), so that the GPU tests compare against
bounds that are known to hold for a correct FP32 implementation and are tight enough to catch a
wrong one (a planted error of a few bfloat16 units in one weight exceeds them)."""
import numpy as np

import mlp_bounds as mb
from oracle import mlp as ref
from paper_2211_03339_amd import testmats as tm

I, H, n = 8, 96, 16
O = n * n


def bf(x):
    return ref.bf16(x).astype(np.float32)


def bf_trunc(x):
    """A plausible mistake: bfloat16 by truncation instead of round-to-nearest-even."""
    u = np.asarray(x, np.float32).view(np.uint32) & np.uint32(0xFFFF0000)
    return u.view(np.float32)


def emulate(p, X, T, bf=bf):
    """FP32 network as the GPU computes it: products of bfloat16 operands summed in FP32."""
    W1, b1, W2, b2, W3, b3 = [a.astype(np.float32) for a in ref.unpack(np.asarray(p, np.float64), I, H, O)]
    Xb = bf(X)
    Z1 = Xb @ bf(W1).T + b1
    H1 = np.maximum(Z1, 0)
    Z2 = bf(H1) @ bf(W2).T + b2
    H2 = np.maximum(Z2, 0)
    Y = bf(H2) @ bf(W3).T + b3
    B = X.shape[0]
    dY = np.float32(2.0 / (B * O)) * (Y - T.astype(np.float32))
    gW3 = bf(dY).T @ bf(H2)
    gb3 = dY.sum(0)
    dZ2 = (bf(dY) @ bf(W3)) * (H2 > 0)
    gW2 = bf(dZ2).T @ bf(H1)
    gb2 = dZ2.sum(0)
    dZ1 = (bf(dZ2) @ bf(W2)) * (H1 > 0)
    gW1 = bf(dZ1).T @ Xb
    gb1 = dZ1.sum(0)
    g = np.concatenate([a.ravel() for a in (gW1, gb1, gW2, gb2, gW3, gb3)]).astype(np.float64)
    return Y.astype(np.float64), g


def test_bounds_hold_for_fp32_emulation_and_are_tight():
    B = 37
    p = tm.mlp_params(I, H, O, seed=6)
    X = tm.mlp_inputs(B, I, seed=7)
    T = tm.bf16_value(tm.bf16_bits((B, O), seed=8))
    Yg, gg = emulate(p, X, T)
    f = mb.forward(p.astype(np.float64), X.astype(np.float64), I, H, O)
    assert np.all(np.abs(Yg - f["Y"]) <= f["eY"])
    # tight enough to catch a truncating bfloat16 conversion in the forward pass
    Yt, _ = emulate(p, X, T, bf=bf_trunc)
    assert np.any(np.abs(Yt - f["Y"]) > f["eY"])
    loss, eloss, g, eg = mb.grads(p.astype(np.float64), X.astype(np.float64), T, I, H, O)
    assert np.all(np.abs(gg - g) <= eg)
    # a planted error of 4 bfloat16 units in one W2 entry moves gradient entries beyond their bounds
    q = p.astype(np.float64).copy()
    k = I * H + H + 5 * H + 7
    q[k] *= 1 + 4 * 2.0 ** -8
    _, gq = emulate(q.astype(np.float32), X, T)
    assert np.any(np.abs(gq - g) > eg)


def test_adamw_bound_holds_for_fp32_steps():
    g0 = tm.rng(3)
    P = 5000
    p = g0.standard_normal(P).astype(np.float32)
    m = np.zeros(P, np.float32)
    v = np.zeros(P, np.float32)
    pr, mr, vr = p.astype(np.float64), np.zeros(P), np.zeros(P)
    ep, em, ev = np.zeros(P), np.zeros(P), np.zeros(P)
    lr, wd, b1, b2, eps = 1e-2, 0.1, 0.9, 0.999, 1e-8
    f32 = np.float32
    for t in range(1, 5):
        gr = g0.standard_normal(P).astype(np.float32)
        c1, c2 = f32(1 / (1 - b1 ** t)), f32(1 / (1 - b2 ** t))
        m = f32(b1) * m + f32(1 - b1) * gr
        v = f32(b2) * v + f32(1 - b2) * gr * gr
        p = p - f32(lr) * ((m * c1) / (np.sqrt(v * c2) + f32(eps)) + f32(wd) * p)
        pr, mr, vr, ep, em, ev = mb.adamw_bound(pr, mr, vr, gr.astype(np.float64), t, lr, wd, b1, b2, eps,
                                                ep, em, ev)
        assert np.all(np.abs(p - pr) <= 2 * ep)
        assert np.all(np.abs(m - mr) <= 2 * em)
        assert np.all(np.abs(v - vr) <= 2 * ev)
    assert np.median(ep / np.abs(pr)) < 1e-5
