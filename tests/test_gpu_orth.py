"""Step 2 as the pipeline runs it (jac_qr_orth): the orthonormal QR factor of the start with a
positive R diagonal -- the factor the oracle's modified Gram-Schmidt returns -- evaluated by passes
of the second-order series when the start is nearly orthonormal (||Z^T Z - I||_F <= 0.1; one pass
when it is at most 2e-5, more until the result is orthonormal to rounding level) and by block MGS
otherwise.  Both are compared entry by entry with the oracle's MGS: the QR factor is unique, so
the two agree to O(n u64) for well-conditioned inputs."""
import numpy as np
import pytest
import torch

import oracle
from paper_2211_03339_amd import jacobi
from paper_2211_03339_amd import testmats as tm

pytestmark = pytest.mark.gpu
U64 = 2.0 ** -53


def _run(Z):
    Q, method = jacobi.jac_qr_orth(torch.from_numpy(np.ascontiguousarray(Z)).cuda())
    return Q.contiguous().cpu().numpy(), method


@pytest.mark.parametrize("n,pert", [(1, 0.0), (2, 1e-7), (64, 1e-7), (257, 1e-7), (1024, 1e-7), (700, 1e-5),
                                    (2048, 1e-7)])
def test_series_matches_mgs_on_nearly_orthonormal_starts(n, pert):
    """A Haar matrix rounded to FP32 (what an FP32 eigensolver hands over), optionally with an extra
    perturbation: the series runs (method 1) and returns the oracle's MGS factor."""
    g = tm.rng(2000 + n)
    Z = tm.haar(n, g).astype(np.float32).astype(np.float64)
    if pert:
        Z = Z + pert * g.standard_normal((n, n)) / np.sqrt(n)
    print(f"[qr series] n={n} ||Z^T Z - I||_F = {np.linalg.norm(Z.T @ Z - np.eye(n)):.2e}", flush=True)
    Q, method = _run(Z)
    assert method == 1
    Qo, Ro, info = oracle.mgs(Z)
    assert info == 0
    assert np.abs(Q - Qo).max() <= 64 * n * U64
    assert np.linalg.norm(Q.T @ Q - np.eye(n)) <= 8 * n * U64
    # R = Q^T Z is upper triangular with a positive diagonal
    R = Q.T @ Z
    assert np.abs(np.tril(R, -1)).max() <= 16 * n * U64
    assert np.all(np.diag(R) > 0)


@pytest.mark.parametrize("n,size", [(300, 5e-4), (300, 2e-2), (130, 4e-2)])
def test_series_passes_on_structured_errors(n, size):
    """A start whose orthogonality error is one direction (Z = Q (I + s u u^T)): the error of one
    pass is about ||E||^3 with no 1/n relief, 1e-10 and above here -- so the series takes further
    passes, and still returns the oracle's MGS factor to rounding level."""
    g = tm.rng(2200 + n)
    Q0 = tm.haar(n, g)
    u = g.standard_normal(n)
    u /= np.linalg.norm(u)
    Z = Q0 @ (np.eye(n) + size * np.outer(u, u))
    e = np.linalg.norm(Z.T @ Z - np.eye(n))
    print(f"[qr passes] n={n} ||Z^T Z - I||_F = {e:.2e}", flush=True)
    assert e ** 3 > 1e-11
    Q, method = _run(Z)
    assert method == 1
    Qo, Ro, info = oracle.mgs(Z)
    assert info == 0
    assert np.abs(Q - Qo).max() <= 64 * n * U64
    assert np.linalg.norm(Q.T @ Q - np.eye(n)) <= 8 * n * U64


@pytest.mark.parametrize("n", [5, 100, 300])
def test_block_mgs_fallback_for_general_starts(n):
    """A Gaussian start is far from orthonormal: block MGS runs (method 2) and matches the oracle up
    to its conditioning."""
    Z = tm.rng(2100 + n).standard_normal((n, n))
    Q, method = _run(Z)
    assert method == 2
    Qo, Ro, info = oracle.mgs(Z)
    kappa = np.linalg.cond(Z)
    assert np.abs(Q - Qo).max() <= 64 * n * U64 * kappa
