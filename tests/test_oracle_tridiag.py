"""Pins for the tridiagonalization route of the oracle (oracle/tridiag.c), the FP64 reference of
the tridiagonal FP32 step 1: each test checks it against closed forms, library routines or the
defining properties, not against itself.  No GPU needed."""
import numpy as np
import pytest
import scipy.linalg as sla

import oracle
from paper_2211_03339_amd import testmats as tm

U = 2.0 ** -53


def tri(d, e):
    return np.diag(d) + np.diag(e, 1) + np.diag(e, -1)


@pytest.mark.parametrize("n,kind", [(2, "uniform"), (3, "uniform"), (37, "uniform"), (64, "geometric"),
                                    (101, "clusters")])
def test_sytrd_is_an_orthogonal_similarity(n, kind):
    """Q = H_0 ... H_{n-3} is orthogonal, Q^T A Q is the tridiagonal (d, e), and its eigenvalues
    (LAPACK's tridiagonal solver) are the prescribed spectrum."""
    A, lam = tm.sym_matrix(n, kind, seed=900 + n)
    d, e, tau, Uv = oracle.sytrd(A)
    Q = oracle.apply_reflectors(Uv, tau, np.eye(n))
    nA = np.linalg.norm(A)
    assert np.linalg.norm(Q.T @ Q - np.eye(n)) <= 8 * n * U
    assert np.linalg.norm(Q.T @ A @ Q - tri(d, e)) <= 8 * n * U * nA
    w = sla.eigvalsh_tridiagonal(d, e) if n > 1 else d
    assert np.abs(np.sort(w) - np.sort(lam)).max() <= 8 * n * U * np.abs(lam).max()
    # the reflector vectors: u_k(k+1) = 1, zero above, tau in [0, 2]
    for k in range(n - 2):
        assert Uv[k + 1, k] == 1.0 and not np.any(Uv[: k + 1, k])
        assert 0.0 <= tau[k] <= 2.0


@pytest.mark.parametrize("b", [0.7, -0.4, 0.0])
def test_sytrd_3x3_by_hand(b):
    """Order 3: one reflector.  beta = -sign(b) sqrt(b^2 + c^2) (sign(0) = +1); the trailing 2x2
    block is P B P with P the reflection I - 2 v v^T / v^T v, v = x - beta e_1, which maps
    x = (b, c) to (beta, 0)."""
    a, c, dd, f, g = 0.3, 0.9, -1.2, 0.25, 0.6
    A = np.array([[a, b, c], [b, dd, f], [c, f, g]])
    d, e, tau, _ = oracle.sytrd(A)
    r = np.hypot(b, c)
    beta = -r if b >= 0 else r
    x = np.array([b, c])
    v = x - np.array([beta, 0.0])
    P = np.eye(2) - 2.0 * np.outer(v, v) / (v @ v)
    assert np.allclose(P @ x, [beta, 0.0], atol=1e-15)
    B = P @ np.array([[dd, f], [f, g]]) @ P
    assert d[0] == a
    assert abs(e[0] - beta) <= 4 * U * r
    assert np.allclose([d[1], e[1], d[2]], [B[0, 0], B[1, 0], B[1, 1]], rtol=0, atol=16 * U)


def test_sytrd_leaves_a_tridiagonal_matrix_alone():
    """A tridiagonal input has nothing below the subdiagonal: every reflector is the identity
    (tau = 0) and d, e are the input's diagonals exactly."""
    g = tm.rng(77)
    n = 40
    d0, e0 = g.uniform(-1, 1, n), g.uniform(-1, 1, n - 1)
    d, e, tau, _ = oracle.sytrd(tri(d0, e0))
    assert np.array_equal(d, d0) and np.array_equal(e, e0) and not np.any(tau)


@pytest.mark.parametrize("n,a,b", [(1, 0.5, 0.0), (2, 1.0, -0.5), (50, 2.0, 1.0), (333, -0.3, 0.45)])
def test_bisection_toeplitz_closed_form(n, a, b):
    """Tridiagonal Toeplitz (a on the diagonal, b beside it): eigenvalues a + 2 b cos(k pi/(n+1));
    the Sturm count below a point between two of them is the number of smaller ones."""
    d, e = np.full(n, a), np.full(n - 1, b)
    w = oracle.tridiag_eigvals(d, e)
    ref = np.sort(a + 2 * b * np.cos(np.arange(1, n + 1) * np.pi / (n + 1)))
    assert np.abs(w - ref).max() <= 8 * U * (abs(a) + 2 * abs(b))
    if n > 1:
        mids = 0.5 * (ref[1:] + ref[:-1])
        for k in range(0, n - 1, max(1, (n - 1) // 7)):
            assert oracle.sturm_count(d, e, mids[k]) == k + 1


def test_bisection_matches_lapack():
    """Against LAPACK's bisection (dstebz): the computed Sturm count is exact for T with each
    entry perturbed by a few units of roundoff (Kahan), so two bisections agree within a few
    u max(|d| + 2|e|); against the dense QR-based solver within its O(n u) error."""
    g = tm.rng(78)
    for n in (5, 64, 257):
        d, e = g.standard_normal(n), g.standard_normal(n - 1)
        w = oracle.tridiag_eigvals(d, e)
        scale = np.abs(d).max() + 2 * np.abs(e).max()
        assert np.abs(w - sla.eigvalsh_tridiagonal(d, e, lapack_driver="stebz")).max() <= 8 * U * scale
        assert np.abs(w - np.linalg.eigvalsh(tri(d, e))).max() <= 2 * n * U * scale


def test_inverse_iteration_toeplitz_vectors():
    """Toeplitz eigenvectors sqrt(2/(n+1)) sin(j k pi/(n+1)), compared up to sign."""
    n, a, b = 60, 0.2, -0.7
    d, e = np.full(n, a), np.full(n - 1, b)
    k = np.arange(1, n + 1)
    lam = a + 2 * b * np.cos(k * np.pi / (n + 1))
    order = np.argsort(lam)
    Z = oracle.tridiag_vectors(d, e, lam[order])
    j = np.arange(1, n + 1)[:, None]
    ref = np.sqrt(2.0 / (n + 1)) * np.sin(j * k[order][None, :] * np.pi / (n + 1))
    sgn = np.sign((Z * ref).sum(0))
    assert np.abs(Z - ref * sgn[None, :]).max() <= 1e-11


def test_inverse_iteration_residual_and_lapack_vectors():
    g = tm.rng(79)
    n = 120
    d, e = g.uniform(-1, 1, n), g.uniform(-1, 1, n - 1)
    w = oracle.tridiag_eigvals(d, e)
    Z = oracle.tridiag_vectors(d, e, w)
    T = tri(d, e)
    tn = np.abs(T).sum(0).max()
    assert np.abs(T @ Z - Z * w[None, :]).max() <= 64 * U * tn
    wr, Zr = sla.eigh_tridiagonal(d, e)
    gap = np.minimum(np.append(np.diff(wr), np.inf), np.insert(np.diff(wr), 0, np.inf))
    sgn = np.sign((Z * Zr).sum(0))
    err = np.abs(Z - Zr * sgn[None, :]).max(0)
    assert np.all(err <= 64 * U * tn * np.sqrt(n) / gap + 1e-14)


def test_whole_route_recovers_the_spectrum():
    A, lam = tm.sym_matrix(150, "uniform", seed=80)
    W, Z = oracle.syev_tridiag(A)
    nA = np.linalg.norm(A)
    assert np.abs(W - np.sort(lam)).max() <= 64 * U * np.abs(lam).max()
    assert np.linalg.norm(A @ Z - Z * W[None, :]) / nA <= 64 * U * np.sqrt(150)
