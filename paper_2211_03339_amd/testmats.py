"""Seeded synthetic test matrices.

This module only draws inputs; it holds none of the eigensolver's arithmetic
and is the one piece of code that both the GPU path's tests/benchmarks and
the CPU oracle's tests use.  All generation is FP64 NumPy (PCG64 streams).

Families:
  * symmetric A = Q diag(lambda) Q^T with Q Haar-distributed (QR of an FP64
    N(0,1) matrix with the signs of R's diagonal folded into Q) and the
    spectra used in the workloads: U[-1,1], signed geometric 10^(-d i/(n-1)),
    and ten clusters of width 1e-6 around U[-1,1] centres;
  * the SPD families of the paper's experiments (Section 6, Examples 6.1 and
    6.2): prescribed eigenvalues with one large / one small / geometric /
    arithmetic / log-uniform distribution and condition kappa, and an r-fold
    multiple spectrum;
  * the parametric family A(theta) = A0 + sum_k theta_k B_k for the learned
    warm start, and rectangular U diag(sigma) V^T inputs for the SVD.
Matrices are returned column-major (Fortran order) float64 arrays.
"""
from __future__ import annotations

import numpy as np


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


def haar(n: int, g: np.random.Generator, m: int | None = None) -> np.ndarray:
    """m x n (default n x n) matrix with Haar-distributed orthonormal columns."""
    m = n if m is None else m
    G = g.standard_normal((m, n))
    Q, R = np.linalg.qr(G)
    Q = Q * np.sign(np.diag(R))[None, :]
    return np.asfortranarray(Q)


def from_spectrum(lam: np.ndarray, g: np.random.Generator) -> np.ndarray:
    """A = Q diag(lam) Q^T, symmetrised exactly as (A + A^T)/2."""
    lam = np.asarray(lam, np.float64)
    Q = haar(lam.size, g)
    A = (Q * lam[None, :]) @ Q.T
    A = 0.5 * (A + A.T)
    return np.asfortranarray(A)


def spectrum(kind: str, n: int, g: np.random.Generator, decades: float = 8.0) -> np.ndarray:
    if kind == "uniform":
        return g.uniform(-1.0, 1.0, n)
    if kind == "geometric":
        i = np.arange(n)
        mag = 10.0 ** (-decades * i / max(n - 1, 1))
        sgn = np.where(g.uniform(size=n) < 0.5, -1.0, 1.0)
        return sgn * mag
    if kind == "clusters":
        centres = g.uniform(-1.0, 1.0, 10)
        return centres[np.arange(n) % 10] + 1e-6 * g.uniform(-1.0, 1.0, n)
    raise ValueError(kind)


SPECTRA = ("uniform", "geometric", "clusters")


def sym_matrix(n: int, kind: str = "uniform", seed: int = 0, decades: float = 8.0):
    """(A, lam) for one symmetric test matrix; the Haar factor is drawn after lam."""
    g = rng(seed)
    lam = spectrum(kind, n, g, decades)
    return from_spectrum(lam, g), lam


def small_plain_case():
    """n = 128, lambda ~ U[-1,1], seed 101 (plain FP64 Jacobi workload)."""
    return sym_matrix(128, "uniform", 101)


def precond_seed(n: int, kind: str) -> int:
    return 2_000_000 + 10_000 * (SPECTRA.index(kind) + 1) + n


def precond_case(n: int, kind: str = "uniform"):
    """Preconditioned-pipeline workload at order n with the given spectrum."""
    return sym_matrix(n, kind, precond_seed(n, kind))


def large_case(n: int = 8192):
    """Order-8192 matrix with a signed geometric spectrum of condition 1e10."""
    return sym_matrix(n, "geometric", 5_000_000 + n, decades=10.0)


# ---- Section 6 families (SPD, prescribed condition number) -----------------

def randsvd_eigs(n: int, kappa: float, mode: int, g: np.random.Generator) -> np.ndarray:
    """Eigenvalues of Example 6.1's modes 1-5 (largest 1, smallest 1/kappa)."""
    i = np.arange(n)
    if mode == 1:
        lam = np.full(n, 1.0 / kappa); lam[0] = 1.0
    elif mode == 2:
        lam = np.ones(n); lam[-1] = 1.0 / kappa
    elif mode == 3:
        lam = kappa ** (-i / max(n - 1, 1))
    elif mode == 4:
        lam = 1.0 - (1.0 - 1.0 / kappa) * i / max(n - 1, 1)
    elif mode == 5:
        lam = np.exp(-np.log(kappa) * g.uniform(size=n))
    else:
        raise ValueError(mode)
    return lam


def example61(n: int, kappa: float, mode: int, seed: int = 0):
    g = rng(seed)
    lam = randsvd_eigs(n, kappa, mode, g)
    return from_spectrum(lam, g), lam


def example62(n: int, kappa: float, mode: int, r: int = 4, seed: int = 0):
    """A = P diag(lam kron 1_r) P^T, n = r s (Example 6.2, modes 3 and 5 read
    with elementwise powers so that A is positive definite)."""
    s = n // r
    g = rng(seed)
    if mode == 1:
        lam = np.full(s, 1.0 / kappa); lam[0] = 1.0
    elif mode == 2:
        lam = np.ones(s); lam[-1] = 1.0 / kappa
    elif mode == 3:
        lam = kappa ** np.linspace(-1.0, 0.0, s)
    elif mode == 4:
        lam = 1.0 - (1.0 - 1.0 / kappa) * np.linspace(0.0, 1.0, s)
    elif mode == 5:
        lam = kappa ** (-g.uniform(size=s))
    else:
        raise ValueError(mode)
    full = np.kron(lam, np.ones(r))
    return from_spectrum(full, g), full


# ---- batched workload -------------------------------------------------------

def batched_sizes(count: int = 4096, seed: int = 3, lo: int = 32, hi: int = 512, step: int = 32):
    g = rng(seed)
    return step * g.integers(lo // step, hi // step + 1, size=count)


def batched_matrix(i: int, n: int):
    return sym_matrix(int(n), "uniform", 3_000_000 + i)


# ---- learned warm start: parametric family ----------------------------------

def param_family(n: int = 256, k: int = 8, seed: int = 4):
    """A0 and B_1..B_k: symmetric (G + G^T)/2 with G ~ N(0,1), B_k scaled by 0.1."""
    g = rng(seed)
    G = g.standard_normal((k + 1, n, n))
    A0 = 0.5 * (G[0] + G[0].T)
    B = 0.1 * 0.5 * (G[1:] + np.transpose(G[1:], (0, 2, 1)))
    return np.asfortranarray(A0), np.ascontiguousarray(B)


def param_thetas(count: int, seed: int, k: int = 8):
    return rng(seed).uniform(-1.0, 1.0, (count, k))


def param_matrix(A0, B, theta) -> np.ndarray:
    A = A0 + np.tensordot(np.asarray(theta), B, axes=(0, 0))
    return np.asfortranarray(0.5 * (A + A.T))


# ---- learned warm start: network parameters, inputs and targets -----------------

def mlp_params(I: int, H: int, O: int, seed: int = 6) -> np.ndarray:
    """Packed float32 parameters [W1 (H x I), b1, W2 (H x H), b2, W3 (O x H), b3] drawn N(0, s^2)
    with s = sqrt(2/fan_in) (W1, W2), sqrt(1/H) (W3), 0.1 (biases)."""
    g = rng(seed)
    parts = [g.standard_normal(H * I) * np.sqrt(2.0 / I), 0.1 * g.standard_normal(H),
             g.standard_normal(H * H) * np.sqrt(2.0 / H), 0.1 * g.standard_normal(H),
             g.standard_normal(O * H) * np.sqrt(1.0 / H), 0.1 * g.standard_normal(O)]
    return np.concatenate(parts).astype(np.float32)


def mlp_inputs(B: int, I: int, seed: int = 7) -> np.ndarray:
    return rng(seed).uniform(-1.0, 1.0, (B, I)).astype(np.float32)


def bf16_bits(shape, seed: int = 8, emin: int = 118, emax: int = 126) -> np.ndarray:
    """Random bfloat16 bit patterns (int16): random sign and mantissa, biased exponent uniform in
    [emin, emax] (magnitudes in [2^(emin-127), 2^(emax-126)))."""
    g = rng(seed)
    sign = g.integers(0, 2, shape, dtype=np.uint32)
    exp = g.integers(emin, emax + 1, shape, dtype=np.uint32)
    man = g.integers(0, 128, shape, dtype=np.uint32)
    return ((sign << 15) | (exp << 7) | man).astype(np.uint16).view(np.int16)


def bf16_value(bits: np.ndarray) -> np.ndarray:
    """float64 value of bfloat16 bit patterns (exact)."""
    return (np.asarray(bits).view(np.uint16).astype(np.uint32) << 16).view(np.float32).astype(np.float64)


# ---- rectangular SVD inputs ---------------------------------------------------

def svd_case(m: int, n: int, decades: float = 6.0, seed: int = 5_002_048):
    """A = U diag(sigma) V^T, U m x n and V n x n Haar, sigma_i = 10^(-d i/(n-1))."""
    g = rng(seed)
    U = haar(n, g, m)
    V = haar(n, g)
    sig = 10.0 ** (-decades * np.arange(n) / max(n - 1, 1))
    A = (U * sig[None, :]) @ V.T
    return np.asfortranarray(A), sig
