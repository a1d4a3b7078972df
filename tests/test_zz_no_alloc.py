"""The allocation-free entry point syev_jacobi_noalloc against syev_jacobi_ex on the same inputs:
two calls in a row, the second of smaller order, for the plain and the FP32-preconditioned start.
Both run the same kernels on the same data (the allocation-free call keeps K whole in the Q^T A Q
GEMMs, which at these orders the pooled call does as well), so the results are expected to agree
bit for bit; the test asserts the accuracy bars of both, agreement of W within 1e-12 ||A||_2 and of
every eigenvector up to sign within 1e-10, equal sweep counts, and reports bitwise equality."""
import numpy as np
import pytest
import torch

from paper_2211_03339_amd import jacobi
from paper_2211_03339_amd import testmats as tm

pytestmark = pytest.mark.gpu


def _check(Ad, W, V, lam):
    n = Ad.shape[0]
    V = V.contiguous()
    nA = float(torch.linalg.norm(Ad))
    res = float(torch.linalg.norm(Ad @ V - V * W[None, :])) / nA
    orth = float(torch.linalg.norm(V.t().contiguous() @ V - torch.eye(n, dtype=torch.float64, device=V.device)))
    lam_err = float(np.abs(W.cpu().numpy() - np.sort(lam)).max() / np.abs(lam).max())
    assert res <= 1e-13 and orth <= 1e-13 and lam_err <= 1e-12, (res, orth, lam_err)


@pytest.mark.parametrize("precond", ["none", "fp32"])
def test_noalloc_matches_pooled_two_calls(precond):
    for n, seed in [(384, 7001), (200, 7002)]:
        print(f"[noalloc] precond={precond} n={n}", flush=True)
        A, lam = tm.sym_matrix(n, "uniform", seed=seed)
        Ad = torch.from_numpy(A).cuda()
        W1, V1, st1, c1 = jacobi.syev_jacobi_noalloc(Ad, tol=1e-15, precond=precond)
        W0, V0, st0, c0 = jacobi.syev_jacobi_ex(Ad, tol=1e-15, precond=precond)
        assert c1 == 0 and c0 == 0
        _check(Ad, W1, V1, lam)
        _check(Ad, W0, V0, lam)
        nrm2 = float(np.abs(lam).max())
        assert float((W1 - W0).abs().max()) <= 1e-12 * nrm2
        dots = (V1 * V0).sum(dim=0)
        sgn = torch.where(dots < 0, -1.0, 1.0).to(torch.float64)
        assert float((V1 - V0 * sgn[None, :]).abs().max()) <= 1e-10
        assert st1["sweeps"] == st0["sweeps"]
        assert st1["stage_ms"]["total"] == 0.0   # no events were created
        bitwise = bool(torch.equal(W1, W0) and torch.equal(V1, V0))
        print(f"  sweeps={st1['sweeps']} bitwise_equal={bitwise}", flush=True)


def test_noalloc_rejects_oversize_and_learned_start():
    cap = jacobi.noalloc_bytes()
    L = jacobi.load()
    n = 64
    while L.jac_workspace_bytes(n, jacobi.ctypes.byref(jacobi._opts("fp32"))) <= cap:
        n += 64
    A = torch.zeros((n, n), dtype=torch.float64, device="cuda")
    _, _, _, code = jacobi.syev_jacobi_noalloc(A, precond="fp32", check=False)
    assert code == -2 and "fixed device array" in jacobi.last_error()
    A = torch.eye(8, dtype=torch.float64, device="cuda")
    _, _, _, code = jacobi.syev_jacobi_noalloc(A, precond="mlp", check=False)
    assert code == -8
