"""GPU parity of the one-sided Jacobi SVD (Algorithms 5.1 / 5.2) against known singular values and
the CPU oracle.  Bars: |sigma_i - sigma_ref,i| <= 1e-12 sigma_1, ||A V - U Sigma||_F / ||A||_F <=
1e-13, ||V^T V - I||_F <= 1e-13 (raw for n <= 1024; the paper's sqrt(n)-normalised OR form beyond).
U = C Sigma^-1 is orthogonal only as far as the rotation rule drives the columns of C: a pair is left
alone once |c_i.c_j| <= m eps ||c_i|| ||c_j|| (eps = 2^-53), and the sweeps stop when fewer than
2e-4 n(n-1)/2 pairs were rotated, so the bar for U is on each pair, |u_i.u_j| <= 4 m eps (a later
rotation of a neighbouring pair can mix two such cosines, growing their maximum by up to sqrt 2),
and |u_i.u_i - 1| <= 1e-14; ||U^T U - I||_F, which grows like n m eps, is printed."""
import numpy as np
import pytest
import torch

import oracle
from paper_2211_03339_amd import jacobi
from paper_2211_03339_amd import testmats as tm

pytestmark = pytest.mark.gpu


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).to("cuda")


def host(x):
    return x.detach().cpu().numpy()


def check_svd(A, S, U, V, sig=None):
    m, n = A.shape
    assert np.all(np.diff(S) <= 0)
    res = np.linalg.norm(A @ V - U * S[None, :]) / np.linalg.norm(A)
    G = U.T @ U - np.eye(n)
    ou = np.linalg.norm(G)
    ov = np.linalg.norm(V.T @ V - np.eye(n))
    bar = 1e-13 if n <= 1024 else 1e-13 * np.sqrt(n)
    assert res <= 1e-13, res
    assert ov <= bar, ov
    assert np.abs(np.diag(G)).max() <= 1e-14, np.abs(np.diag(G)).max()
    cmax = np.abs(G - np.diag(np.diag(G))).max() if n > 1 else 0.0
    assert cmax <= 4 * m * 2.0 ** -53, (cmax, m)
    print(f"  res={res:.2e} ||V^T V - I||={ov:.2e} ||U^T U - I||={ou:.2e} max|u_i.u_j|={cmax:.2e}", flush=True)
    if sig is not None:
        assert np.abs(S - np.sort(sig)[::-1]).max() <= 1e-12 * np.abs(sig).max()
    return res, ou, ov


@pytest.mark.parametrize("m,n", [(1, 1), (5, 3), (60, 24), (200, 64), (300, 130), (513, 257)])
@pytest.mark.parametrize("pre", ["none", "fp32"])
def test_svd_known_sigma(m, n, pre):
    A, sig = tm.svd_case(m, n, decades=4.0, seed=7 + m + n)
    print(f"[svd m={m} n={n} {pre}]", flush=True)
    S, U, V, st, info = jacobi.gesvd_jacobi_ex(dev(A), precond=pre)
    check_svd(A, host(S), host(U), host(V), sig)
    if n <= 130 and n > 1:
        ref = oracle.gesvd(A)
        assert np.abs(host(S) - ref.S).max() <= 1e-12 * ref.S[0]


def test_svd_preconditioned_fewer_sweeps():
    A, sig = tm.svd_case(1024, 256, decades=6.0, seed=11)
    S1, U1, V1, st1, _ = jacobi.gesvd_jacobi_ex(dev(A), precond="none")
    S2, U2, V2, st2, _ = jacobi.gesvd_jacobi_ex(dev(A), precond="fp32")
    check_svd(A, host(S2), host(U2), host(V2), sig)
    print(f"[svd sweeps] plain={st1['sweeps']} precond={st2['sweeps']}", flush=True)
    assert st2["sweeps"] < st1["sweeps"]


def test_svd_error_codes():
    A, _ = tm.svd_case(20, 10, seed=1)
    with pytest.raises(jacobi.JacobiError) as e:
        jacobi.gesvd_jacobi_ex(dev(A.T.copy()))     # m < n
    assert e.value.code == -3
    bad = A.copy()
    bad[3, 4] = np.inf
    with pytest.raises(jacobi.JacobiError) as e:
        jacobi.gesvd_jacobi_ex(dev(bad))
    assert e.value.code == 2


def test_gesvd_jacobi_default_entry_point():
    """The plain C entry point gesvd_jacobi (Algorithm 5.2, default options, null stream) against
    the known singular values and the oracle's one-sided Jacobi."""
    m, n = 300, 130
    A, sig = tm.svd_case(m, n, decades=5.0, seed=77)
    print(f"[gesvd_jacobi] {m}x{n}", flush=True)
    S, U, V, sweeps, info = jacobi.gesvd_jacobi(dev(A))
    assert info == 0 and sweeps >= 1
    S, U, V = host(S), host(U), host(V)
    check_svd(A, S, U, V, sig)
    ref = oracle.gesvd(A)
    assert np.abs(S - ref.S).max() <= 1e-12 * sig.max()


@pytest.mark.parametrize("m,n,pre", [(700, 40, "fp32"), (2000, 100, "none"), (2048, 128, "fp32"),
                                     (4096, 256, "fp32"), (8192, 512, "fp32")])
def test_svd_qr_first(m, n, pre):
    """QR preconditioning for m >> n (the remark after Algorithm 5.2): A = Q_A B by two passes of
    block MGS, the SVD of the n x n B, U = Q_A U_B.  The same bars as the direct form, the known
    singular values, and the direct form's singular values."""
    A, sig = tm.svd_case(m, n, decades=6.0, seed=31 + m + n)
    print(f"[svd qr-first m={m} n={n} {pre}]", flush=True)
    S, U, V, st, info = jacobi.gesvd_jacobi_ex(dev(A), precond=pre, svd_qr="on")
    assert info == 0 and st["svd_qr_used"] == 1
    check_svd(A, host(S), host(U), host(V), sig)
    S2, U2, V2, st2, info2 = jacobi.gesvd_jacobi_ex(dev(A), precond=pre, svd_qr="off")
    assert st2["svd_qr_used"] == 0
    assert np.abs(host(S) - host(S2)).max() <= 1e-12 * sig.max()
    print(f"  qr-first {st['stage_ms']['total']:.2f} ms ({st['sweeps']} sweeps, QR {st['qr_ms']:.2f} ms) vs "
          f"direct {st2['stage_ms']['total']:.2f} ms ({st2['sweeps']} sweeps)", flush=True)
    if n <= 64:
        ref = oracle.gesvd(A)
        assert np.abs(host(S) - ref.S).max() <= 1e-12 * ref.S[0]


def test_svd_qr_first_rule_and_limit():
    A, _ = tm.svd_case(4096, 512, seed=5)
    _, _, _, st, _ = jacobi.gesvd_jacobi_ex(dev(A))            # m >= 8 n, n >= 512: QR first
    assert st["svd_qr_used"] == 1
    A, _ = tm.svd_case(1024, 100, seed=5)
    _, _, _, st, _ = jacobi.gesvd_jacobi_ex(dev(A))            # n < 512: direct
    assert st["svd_qr_used"] == 0
    A, _ = tm.svd_case(2048, 512, seed=6)
    _, _, _, st, _ = jacobi.gesvd_jacobi_ex(dev(A))            # m < 8 n: direct
    assert st["svd_qr_used"] == 0
    A, sig = tm.svd_case(8200, 8, seed=7)
    _, _, _, st, _ = jacobi.gesvd_jacobi_ex(dev(A))            # beyond the measured rows: direct
    assert st["svd_qr_used"] == 0
    S, U, V, st, _ = jacobi.gesvd_jacobi_ex(dev(A), svd_qr="on")   # forced: two-column MGS panels
    assert st["svd_qr_used"] == 1
    assert np.abs(host(S) - np.sort(sig)[::-1]).max() <= 1e-13 * sig.max()
    U = host(U)
    assert np.linalg.norm(U.T @ U - np.eye(8)) <= 1e-13
    A, _ = tm.svd_case(32769, 8, seed=8)
    with pytest.raises(jacobi.JacobiError) as e:
        jacobi.gesvd_jacobi_ex(dev(A), svd_qr="on")            # beyond the MGS rows
    assert e.value.code == -2
