"""Full-size parity: the preconditioned pipeline at n = 1024, 2048 and 4096 on the three spectra, the
order-8192 matrix with a signed geometric spectrum of condition 1e10, and the one-sided SVD of an
8192 x 2048 matrix with singular values 10^(-6 i / 2047).  At these sizes the oracle would take
hours, so the results are checked against the prescribed spectra (|lambda_i - lambda_ref,i| <=
1e-12 ||A||_2, sigma likewise) and by their defining properties: ||A V - V Lambda||_F / ||A||_F <=
1e-13 and the orthogonality bar of the raw / sqrt(n)-normalised reading (raw for preconditioned
n <= 1024).  The products for the checks use torch's own FP64 GEMM, independent of the library.
"""
import numpy as np
import pytest
import torch

from paper_2211_03339_amd import jacobi
from paper_2211_03339_amd import testmats as tm

pytestmark = [pytest.mark.gpu, pytest.mark.slow]


def _fro(x):
    return float(torch.linalg.norm(x).item())


def check_eig_dev(Ad, W, V, lam, raw_orth):
    n = Ad.shape[0]
    V = V.contiguous()
    res = _fro(Ad @ V - V * W[None, :]) / _fro(Ad)
    orth = _fro(V.t().contiguous() @ V - torch.eye(n, dtype=torch.float64, device=V.device))
    lam_err = float(np.abs(W.cpu().numpy() - np.sort(lam)).max() / np.abs(lam).max())
    assert bool(torch.all(W[1:] >= W[:-1]))
    assert res <= 1e-13, res
    bar = 1e-13 if raw_orth else 1e-13 * np.sqrt(n)
    assert orth <= bar, (orth, bar)
    assert lam_err <= 1e-12, lam_err
    return res, orth, lam_err


@pytest.mark.parametrize("n", [1024, 2048, 4096])
@pytest.mark.parametrize("kind", tm.SPECTRA)
def test_preconditioned_full_sizes(n, kind):
    print(f"[large] n={n} {kind}", flush=True)
    A, lam = tm.precond_case(n, kind)
    Ad = torch.from_numpy(A).cuda()
    W, V, st, _ = jacobi.syev_jacobi_ex(Ad, precond="fp32")
    res, orth, le = check_eig_dev(Ad, W, V, lam, raw_orth=n <= 1024)
    print(f"  sweeps={st['sweeps']} fp32_sweeps={st['fp32_sweeps']} res={res:.2e} orth={orth:.2e} "
          f"lam_err={le:.2e} ms={st['stage_ms']['total']:.1f}", flush=True)
    assert st["sweeps"] <= 16


def test_plain_n1024_for_comparison():
    A, lam = tm.precond_case(1024, "uniform")
    Ad = torch.from_numpy(A).cuda()
    W, V, st, _ = jacobi.syev_jacobi_ex(Ad, precond="none")
    res, orth, le = check_eig_dev(Ad, W, V, lam, raw_orth=False)
    print(f"[large] plain n=1024 sweeps={st['sweeps']} res={res:.2e} orth={orth:.2e}", flush=True)


def test_order_8192_geometric_1e10():
    print("[large] n=8192 geometric 1e10: generating", flush=True)
    A, lam = tm.large_case(8192)
    Ad = torch.from_numpy(A).cuda()
    del A
    print("[large] n=8192 solving", flush=True)
    W, V, st, _ = jacobi.syev_jacobi_ex(Ad, precond="fp32")
    res, orth, le = check_eig_dev(Ad, W, V, lam, raw_orth=False)
    print(f"  sweeps={st['sweeps']} fp32_sweeps={st['fp32_sweeps']} res={res:.2e} orth={orth:.2e} "
          f"lam_err={le:.2e} ms={st['stage_ms']['total']:.1f}", flush=True)


def test_preconditioned_above_8192():
    """An order above 8192 (the old row limit of step 2's block MGS): the Jacobi start, the series
    QR factor and the FP64 sweeps."""
    n = 8320
    print(f"[large] n={n} uniform: generating", flush=True)
    A, lam = tm.sym_matrix(n, "uniform", 5_100_000 + n)
    Ad = torch.from_numpy(A).cuda()
    del A
    print(f"[large] n={n} solving", flush=True)
    W, V, st, _ = jacobi.syev_jacobi_ex(Ad, precond="fp32")
    res, orth, le = check_eig_dev(Ad, W, V, lam, raw_orth=False)
    print(f"  sweeps={st['sweeps']} fp32_sweeps={st['fp32_sweeps']} res={res:.2e} orth={orth:.2e} "
          f"lam_err={le:.2e} ms={st['stage_ms']['total']:.1f}", flush=True)


def test_svd_8192_by_2048():
    print("[large] SVD 8192 x 2048: generating", flush=True)
    A, sig = tm.svd_case(8192, 2048)
    Ad = torch.from_numpy(np.ascontiguousarray(A)).cuda()
    m, n = A.shape
    print("[large] SVD solving", flush=True)
    S, U, V, st, _ = jacobi.gesvd_jacobi_ex(Ad, precond="fp32")
    U, V = U.contiguous(), V.contiguous()
    res = _fro(Ad @ V - U * S[None, :]) / _fro(Ad)
    ov = _fro(V.t().contiguous() @ V - torch.eye(n, dtype=torch.float64, device=V.device))
    G = U.t().contiguous() @ U - torch.eye(n, dtype=torch.float64, device=U.device)
    dmax = float(G.diagonal().abs().max().item())
    cmax = float((G - torch.diag(G.diagonal())).abs().max().item())
    s_err = float(np.abs(S.cpu().numpy() - np.sort(sig)[::-1]).max() / sig.max())
    print(f"  sweeps={st['sweeps']} res={res:.2e} ||V^T V - I||={ov:.2e} max|u_i.u_j|={cmax:.2e} "
          f"sigma_err={s_err:.2e} ms={st['stage_ms']['total']:.1f}", flush=True)
    assert bool(torch.all(S[1:] <= S[:-1]))
    assert res <= 1e-13, res
    assert ov <= 1e-13 * np.sqrt(n), ov
    assert dmax <= 1e-14, dmax
    assert cmax <= 4 * m * 2.0 ** -53, cmax
    assert s_err <= 1e-12, s_err


@pytest.mark.parametrize("n", [512, 1024, 2048])
@pytest.mark.parametrize("kind", ["uniform", "geometric"])
def test_element_variant_full_sizes(n, kind):
    """The element-wise variant (n/2 disjoint 2x2 rotations per launch, T and V streamed through
    HBM) end to end at full size, preconditioned: the path whose step kernel is placed on the HBM
    roofline.  Every rotation is applied to V on its own (n - 1 roundings per column per sweep,
    against n/64 - 1 block updates in the blocked variant), so the raw orthogonality bar binds up to
    n = 512; from n = 1024 the normalised form of the Section 6 OR-P metric is asserted (the
    element-wise CPU Jacobi already sits at 0.8-1.0e-13 raw there)."""
    print(f"[large element] n={n} {kind}", flush=True)
    A, lam = tm.precond_case(n, kind)
    Ad = torch.from_numpy(A).cuda()
    W, V, st, _ = jacobi.syev_jacobi_ex(Ad, precond="fp32", variant="element")
    res, orth, le = check_eig_dev(Ad, W, V, lam, raw_orth=n <= 512)
    print(f"  sweeps={st['sweeps']} fp32_sweeps={st['fp32_sweeps']} res={res:.2e} orth={orth:.2e} "
          f"lam_err={le:.2e} ms={st['stage_ms']['total']:.1f}", flush=True)


def test_element_variant_plain_n1024():
    A, lam = tm.precond_case(1024, "uniform")
    Ad = torch.from_numpy(A).cuda()
    print("[large element] plain n=1024", flush=True)
    W, V, st, _ = jacobi.syev_jacobi_ex(Ad, precond="none", variant="element")
    res, orth, le = check_eig_dev(Ad, W, V, lam, raw_orth=False)
    print(f"  sweeps={st['sweeps']} res={res:.2e} orth={orth:.2e} lam_err={le:.2e}", flush=True)
