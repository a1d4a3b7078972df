"""Learned warm start (a project addition): training data from the method's own solves, the
training loop and the evaluation against the FP32 start and plain Jacobi.

Matrix family: A(theta) = A0 + sum_k theta_k B_k with A0, B_k symmetric (0.5 (G + G^T),
G ~ N(0, 1)), B_k scaled by 0.1 and theta ~ U[-1, 1]^k.  Every training matrix is solved by the
batched FP64 Jacobi path (syev_jacobi_batched); its eigenvectors, aligned to the constant start
Z0 within windows of nearby eigenvalues (window_align; without Z0: in ascending eigenvalue order),
become bfloat16 targets (jac_mlp_pack_targets; eigenvalue-ordered ones with their signs made
canonical, aligned ones with the signs the alignment gave them).  Training runs jac_mlp_train_step
over shuffled mini-batches with a cosine-decayed learning rate.  The network starts as the
constant start -- the eigenvectors Z0 of A0 (theta = 0), which every member of the family can
take -- with its last layer zero and its output bias vec(Z0), so it learns a correction to Z0.
Evaluation solves held-out matrices with the learned start (fallback to the FP32 start when the
start residual ||off(Q^T A Q)||_F / ||A||_F exceeds the threshold), with the constant start Z0,
with the FP32 start and with plain Jacobi.

Usage (one GPU): python -m paper_2211_03339_amd.learned [--n 256] [--hidden 1024] [--train 50000]
    [--eval 5000] [--epochs 20] [--out result.json]
"""
from __future__ import annotations

import argparse
import ctypes
import json
import math
import sys
import time

import numpy as np
import torch

from . import jacobi
from . import testmats as tm

THETA_TRAIN_SEED, THETA_EVAL_SEED, THETA_VAL_SEED = 40, 41, 42


def family(n: int, k: int = 8, seed: int = 4):
    """(A0, B) on the device: A0 (n x n), B (k x n x n)."""
    A0, B = tm.param_family(n, k, seed)
    return torch.from_numpy(np.ascontiguousarray(A0)).cuda(), torch.from_numpy(B).cuda()


def matrices(A0: torch.Tensor, B: torch.Tensor, theta: torch.Tensor) -> torch.Tensor:
    """A(theta_c) for a (count, k) FP64 batch of parameters, symmetrised: (count, n, n)."""
    k, n, _ = B.shape
    A = A0.unsqueeze(0) + (theta @ B.reshape(k, n * n)).reshape(-1, n, n)
    return 0.5 * (A + A.transpose(1, 2))


def constant_start(A0: torch.Tensor, with_eigenvalues: bool = False):
    """Z0: the eigenvectors of A0 in ascending eigenvalue order with every column's largest-|entry|
    positive (the sign convention of the training targets); columns are the vectors.  With
    with_eigenvalues, (Z0, lam0)."""
    W, V, _, _ = jacobi.syev_jacobi_ex(A0, precond="fp32")
    V = V.contiguous()
    idx = V.abs().argmax(dim=0)
    sgn = torch.sign(V[idx, torch.arange(V.shape[1], device=V.device)])
    sgn[sgn == 0] = 1.0
    Z0 = (V * sgn[None, :]).contiguous()
    return (Z0, W) if with_eigenvalues else Z0


def init_as_correction(net: jacobi.Mlp, Z0: torch.Tensor):
    """Set the network's last layer to zero and its output bias to vec(Z0) (column-major), so
    that its output is exactly Z0 for every theta and training learns a correction to it."""
    p = net.get()
    I, H, O = net.n_in, net.hidden, net.n * net.n
    w3 = H * I + H + H * H + H
    p[w3: w3 + O * H] = 0.0
    p[w3 + O * H:] = Z0.t().contiguous().reshape(-1).cpu().numpy().astype(np.float32)
    net.set(p)


def start_residual(A: torch.Tensor, Z: torch.Tensor) -> float:
    """||off(Z^T A Z)||_F / ||A||_F for an orthonormal Z (the library's step 3)."""
    T = jacobi.jac_similarity(A, Z)
    nA = torch.linalg.norm(A).item()
    off2 = float((T * T).sum().item() - (torch.diagonal(T) ** 2).sum().item())
    return math.sqrt(max(off2, 0.0)) / nA


class BatchedSolver:
    """Fixed device buffers for syev_jacobi_batched over `count` matrices of order n, so that
    repeated calls replay one captured graph."""

    def __init__(self, n: int, count: int):
        self.n, self.count = n, count
        self.A = torch.empty((count, n, n), dtype=torch.float64, device="cuda")
        self.W = torch.empty((count, n), dtype=torch.float64, device="cuda")
        self.V = torch.empty((count, n, n), dtype=torch.float64, device="cuda")
        self.sweeps = torch.zeros(count, dtype=torch.int32, device="cuda")
        self.info = torch.zeros(count, dtype=torch.int32, device="cuda")
        I = ctypes.c_int * count
        P = ctypes.c_void_p * count
        self.c_n = I(*([n] * count))
        self.c_A = P(*[self.A[i].data_ptr() for i in range(count)])
        self.c_W = P(*[self.W[i].data_ptr() for i in range(count)])
        self.c_V = P(*[self.V[i].data_ptr() for i in range(count)])

    def solve(self, A: torch.Tensor):
        """A: (count, n, n) symmetric.  After the call self.V[c] is the row-major buffer of the
        column-major eigenvector matrix (ascending eigenvalues)."""
        self.A.copy_(A)
        L = jacobi.load()
        code = L.syev_jacobi_batched(self.count, self.c_n, self.c_A, self.c_n, self.c_W, self.c_V, self.c_n, 0.0,
                                     ctypes.c_void_p(self.sweeps.data_ptr()), ctypes.c_void_p(self.info.data_ptr()),
                                     jacobi._stream())
        jacobi._check("syev_jacobi_batched", code)


def window_align(V: torch.Tensor, lam: torch.Tensor, Z0: torch.Tensor, lam0: torch.Tensor, delta: float = 2.0,
                 iters: int = 12) -> torch.Tensor:
    """Targets that follow the constant start where the spectrum lets them.  V: (count, n, n) with
    V[c][:, i] the eigenvector of A(theta_c) for eigenvalue lam[c, i]; Z0, lam0: the eigenpairs of
    A0.  Target c is V[c] P with P the orthogonal polar factor of the overlaps V[c]^T Z0 kept only
    where |lam_i - lam0_j| <= delta: column j mixes only eigenvectors whose eigenvalues lie within
    delta of Z0's eigenvalue j, so it stays close to an invariant subspace (a good start), and the
    arbitrary rotations inside groups of nearby eigenvalues, which make the eigenvectors themselves
    jump as theta moves, are taken out (it varies smoothly with theta).  The polar factor comes from
    Newton-Schulz steps X <- X (3 I - X^T X) / 2 (the products by the library's GEMM), started from
    the masked overlaps scaled below unit 2-norm by sqrt(||X||_1 ||X||_inf)."""
    count, n, _ = V.shape
    out = torch.empty_like(V)
    for c in range(count):
        M = jacobi.jac_gemm(V[c].contiguous(), Z0, transa=True)            # M[i, j] = v_i . z0_j
        M = M * ((lam[c][:, None] - lam0[None, :]).abs() <= delta)
        s = math.sqrt(float(M.abs().sum(0).max()) * float(M.abs().sum(1).max()))
        X = (M / max(s, 1e-300)).contiguous()
        for _ in range(iters):
            G = jacobi.jac_gemm(X, X, transa=True)
            X = (1.5 * X - 0.5 * jacobi.jac_gemm(X, G)).contiguous()
        out[c] = jacobi.jac_gemm(V[c].contiguous(), X)
    return out


def make_dataset(A0, B, thetas: np.ndarray, chunk: int = 4096, Z0: torch.Tensor | None = None,
                 lam0: torch.Tensor | None = None, delta: float = 2.0, log=None):
    """Targets (count, n^2) int16 bfloat16 bits and theta (count, k) float32, on the device.  With Z0
    (and A0's eigenvalues lam0) the eigenvectors are aligned to Z0 (window_align) before packing."""
    n = A0.shape[0]
    count = thetas.shape[0]
    O = n * n
    T = torch.empty((count, O), dtype=torch.int16, device="cuda")
    th64 = torch.from_numpy(thetas).cuda()
    chunk = min(chunk, count)
    solver = BatchedSolver(n, chunk)
    unconverged = 0
    t0 = time.perf_counter()
    for c0 in range(0, count, chunk):
        c1 = min(count, c0 + chunk)
        th = th64[c0:c1]
        if c1 - c0 < chunk:   # pad the last chunk with repeats of its first matrix
            th = torch.cat([th, th[:1].expand(chunk - (c1 - c0), -1)])
        solver.solve(matrices(A0, B, th))
        # solver.V[c] holds column-major eigenvectors: its transpose as a (n, n) tensor has
        # columns = eigenvectors, which is the layout jac_mlp_pack_targets reads.
        Vc = solver.V[: c1 - c0].transpose(1, 2)
        if Z0 is not None:   # aligned to Z0, signs included: packed as they are
            Vc = window_align(Vc, solver.W[: c1 - c0], Z0, lam0, delta)
        jacobi.jac_mlp_pack_targets(Vc, out=T[c0:c1], canonical=Z0 is None)
        unconverged += int((solver.info[: c1 - c0] != 0).sum().item())
        if log:
            log(f"[data] {c1}/{count} solved ({time.perf_counter() - t0:.1f} s)")
    torch.cuda.synchronize()
    return th64.float(), T, {"seconds": time.perf_counter() - t0, "unconverged": unconverged}


def net_start_residual(net: jacobi.Mlp, mats, thetas32) -> float:
    """Mean start residual ||off(Q^T A Q)||_F / ||A||_F of the network's start (Q = the QR factor of
    the prediction, as step 2 computes it) over validation matrices."""
    r = []
    for A, th in zip(mats, thetas32):
        Q, _ = jacobi.jac_qr_orth(net.predict(th))
        r.append(start_residual(A, Q))
    return float(np.mean(r))


def validation_set(A0, B, thetas: np.ndarray):
    th64 = torch.from_numpy(thetas).cuda()
    mats = [matrices(A0, B, th64[i:i + 1])[0].contiguous() for i in range(thetas.shape[0])]
    return mats, torch.from_numpy(thetas.astype(np.float32)).cuda()


def train(net: jacobi.Mlp, theta: torch.Tensor, T: torch.Tensor, epochs: int, batch: int = 256,
          lr: float = 1e-3, weight_decay: float = 1e-4, seed: int = 0, val=None, log=None):
    """AdamW over shuffled mini-batches, learning rate lr * (1 + cos(pi s / S)) / 2.  With
    val = (matrices, thetas) the network's start residual on them is measured before training and
    after every epoch, and the parameters with the lowest one are kept (so the result is never
    worse, on those matrices, than the network it started from)."""
    count = theta.shape[0]
    batch = min(batch, count, net.max_batch)
    per_epoch = max(1, count // batch)
    total = epochs * per_epoch
    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    hist = []
    t0 = time.perf_counter()
    step = 0
    val_hist, best, best_ep = [], None, 0
    if val is not None:
        val_hist.append(net_start_residual(net, *val))
        best = net.get()
    for ep in range(epochs):
        perm = torch.randperm(count, device="cuda", generator=gen)
        acc = torch.zeros(1, dtype=torch.float32, device="cuda")
        for b in range(per_epoch):
            idx = perm[b * batch:(b + 1) * batch]
            lr_t = lr * 0.5 * (1.0 + math.cos(math.pi * step / total))
            net.train_step(theta.index_select(0, idx).contiguous(), T.index_select(0, idx), lr_t, weight_decay,
                           loss)
            acc += loss
            step += 1
        hist.append(acc.item() / per_epoch)
        if val is not None:
            val_hist.append(net_start_residual(net, *val))
            if val_hist[-1] < min(val_hist[:-1]):
                best, best_ep = net.get(), ep + 1
        if log:
            log(f"[train] epoch {ep + 1}/{epochs} loss {hist[-1]:.4e}"
                + (f" val start residual {val_hist[-1]:.4f}" if val is not None else "")
                + f" ({time.perf_counter() - t0:.1f} s)")
    if val is not None and best_ep != epochs:
        net.set(best)
    torch.cuda.synchronize()
    return {"loss_per_epoch": hist, "steps": step, "seconds": time.perf_counter() - t0, "batch": batch,
            "val_start_resid": val_hist, "kept_epoch": best_ep if val is not None else epochs}


def evaluate(net: jacobi.Mlp, A0, B, thetas: np.ndarray, fallback_tol: float = 1e-2, check: bool = True,
             forced: bool = True, Z0: torch.Tensor | None = None, log=None):
    """Per held-out theta: the learned start (with fallback), the learned start always accepted
    (forced), the constant start Z0 (when given), the FP32 start and plain Jacobi.  Returns
    per-mode mean sweeps, wall-clock and the worst residual / orthogonality, plus the learned
    start's residual and fallback rate and the constant start's residual."""
    modes = {"mlp": dict(precond="mlp", fallback_tol=fallback_tol), "fp32": dict(precond="fp32"),
             "plain": dict(precond="none")}
    if forced:
        modes["mlp_forced"] = dict(precond="mlp", fallback_tol=1e300)
    if Z0 is not None:
        modes["const"] = dict(precond="const")
    out = {m: {"sweeps": [], "ms": [], "res": 0.0, "orth": 0.0} for m in modes}
    start_resid, fallback, off_a, const_resid = [], 0, [], []
    th32 = torch.from_numpy(thetas.astype(np.float32)).cuda()
    th64 = torch.from_numpy(thetas).cuda()
    for i in range(thetas.shape[0]):
        A = matrices(A0, B, th64[i:i + 1])[0].contiguous()
        nA = torch.linalg.norm(A).item()
        off_a.append(math.sqrt(max(nA ** 2 - float((torch.diagonal(A) ** 2).sum().item()), 0.0)) / nA)
        if Z0 is not None:
            const_resid.append(start_residual(A, Z0))
        for m, kw in modes.items():
            extra = dict(mlp=net, theta=th32[i]) if kw["precond"] == "mlp" else {}
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            if kw["precond"] == "const":
                W, V, st, _ = jacobi.syev_jacobi_warm(A, Z0)
            else:
                W, V, st, _ = jacobi.syev_jacobi_ex(A, **kw, **extra)
            torch.cuda.synchronize()
            out[m]["ms"].append((time.perf_counter() - t0) * 1e3)
            out[m]["sweeps"].append(st["sweeps"])
            if m == "mlp":
                start_resid.append(st["start_resid"])
                fallback += st["used_fallback"]
            if check:
                Ah, Wh, Vh = A.cpu().numpy(), W.cpu().numpy(), V.cpu().numpy()
                res = np.linalg.norm(Ah @ Vh - Vh * Wh[None, :]) / np.linalg.norm(Ah)
                orth = np.linalg.norm(Vh.T @ Vh - np.eye(Ah.shape[0]))
                out[m]["res"] = max(out[m]["res"], float(res))
                out[m]["orth"] = max(out[m]["orth"], float(orth))
        if log and (i + 1) % 100 == 0:
            log(f"[eval] {i + 1}/{thetas.shape[0]}")
    summary = {m: {"mean_sweeps": float(np.mean(v["sweeps"])), "max_sweeps": int(np.max(v["sweeps"])),
                   "mean_ms": float(np.mean(v["ms"])), "max_res": v["res"], "max_orth": v["orth"]}
               for m, v in out.items()}
    summary["learned_start"] = {"mean_start_resid": float(np.mean(start_resid)),
                                "median_start_resid": float(np.median(start_resid)),
                                "min_start_resid": float(np.min(start_resid)),
                                "fallback_rate": fallback / thetas.shape[0],
                                "mean_identity_start_resid": float(np.mean(off_a))}
    if Z0 is not None:
        summary["const_start"] = {"mean_start_resid": float(np.mean(const_resid)),
                                  "min_start_resid": float(np.min(const_resid))}
    return summary


def run(n=256, hidden=1024, n_train=50000, n_eval=5000, epochs=20, batch=256, lr=1e-4, weight_decay=0.0,
        fallback_tol=1e-2, seed=0, correction=True, log=None):
    A0, B = family(n)
    th_train = tm.param_thetas(n_train, THETA_TRAIN_SEED)
    th_eval = tm.param_thetas(n_eval, THETA_EVAL_SEED)
    Z0, lam0 = constant_start(A0, with_eigenvalues=True)
    theta, T, data = make_dataset(A0, B, th_train, Z0=Z0 if correction else None, lam0=lam0, log=log)
    net = jacobi.Mlp(th_train.shape[1], hidden, n, batch, seed=seed)
    if correction:
        init_as_correction(net, Z0)
    untrained = evaluate(net, A0, B, th_eval[: min(n_eval, 64)], fallback_tol, check=False, forced=False)
    val = validation_set(A0, B, tm.param_thetas(32, THETA_VAL_SEED))
    tr = train(net, theta, T, epochs, batch, lr, weight_decay, seed, val=val, log=log)
    del T
    torch.cuda.empty_cache()
    ev = evaluate(net, A0, B, th_eval, fallback_tol, Z0=Z0, log=log)
    return {"n": n, "hidden": hidden, "params": net.P, "train_solves": n_train, "eval_solves": n_eval,
            "data": data, "train": tr, "eval": ev,
            "untrained_start_resid": untrained["learned_start"]["mean_start_resid"]}, net


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--n", type=int, default=256)
    ap.add_argument("--hidden", type=int, default=1024)
    ap.add_argument("--train", type=int, default=50000)
    ap.add_argument("--eval", type=int, default=5000)
    ap.add_argument("--epochs", type=int, default=20)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=1e-4)
    ap.add_argument("--wd", type=float, default=0.0)
    ap.add_argument("--fallback-tol", type=float, default=1e-2)
    ap.add_argument("--no-correction", action="store_true", help="train from the random initialisation")
    ap.add_argument("--out", default=None)
    a = ap.parse_args(argv)

    def log(m):
        print(m, file=sys.stderr, flush=True)

    res, _ = run(a.n, a.hidden, a.train, a.eval, a.epochs, a.batch, a.lr, a.wd, a.fallback_tol,
                 correction=not a.no_correction, log=log)
    txt = json.dumps(res)
    if a.out:
        with open(a.out, "w") as f:
            f.write(txt + "\n")
    print(txt, flush=True)


if __name__ == "__main__":
    main()
