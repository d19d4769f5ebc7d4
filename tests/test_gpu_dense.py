"""GPU parity of the dense building blocks of the low-rank stage: the FP64
matrix-core GEMM (all transpose combinations, ragged tiles, split
reductions) against numpy's FP64 product."""
import numpy as np
import pytest
import torch

from gpu_util import announce, require_gpu

pytestmark = pytest.mark.gpu


def _bound(Ao, Bo, K):
    # |fl(A B) - A B| <= gamma_K |A| |B| elementwise (plus summation-order slack)
    return 4 * (K + 2) * 2.0 ** -53 * (np.abs(Ao) @ np.abs(Bo)) + 1e-300


@pytest.mark.parametrize("ta,tb", [(False, False), (True, False), (False, True), (True, True)])
@pytest.mark.parametrize("m,n,k", [(1, 1, 1), (64, 64, 16), (130, 70, 37), (257, 129, 300), (200, 64, 20000),
                                   (96, 33, 0)])
def test_dgemm_matches_numpy(ta, tb, m, n, k):
    require_gpu()
    from paper_2308_14490_amd import azrbf
    announce("dgemm", ta, tb, m, n, k)
    rng = np.random.default_rng(m * 7 + n * 3 + k)
    Ao = rng.standard_normal((m, k))
    Bo = rng.standard_normal((k, n))
    Co = rng.standard_normal((m, n))
    As = Ao.T if ta else Ao            # stored matrix
    Bs = Bo.T if tb else Bo
    dev = torch.device("cuda", 0)
    # column-major storage as (cols, rows) tensors, with a padded leading dimension
    def cm(X, pad=3):
        t = torch.zeros((X.shape[1], X.shape[0] + pad), dtype=torch.float64, device=dev)
        t[:, :X.shape[0]] = torch.from_numpy(X.T.copy())
        return t[:, :X.shape[0]]
    A, B, C = cm(As), cm(Bs), cm(Co)
    alpha, beta = 1.25, -0.5
    out = azrbf.dgemm(A, B, C, transa=ta, transb=tb, alpha=alpha, beta=beta)
    torch.cuda.synchronize()
    got = out.cpu().numpy().T
    ref = alpha * (Ao @ Bo) + beta * Co
    err = np.abs(got - ref)
    assert np.all(err <= abs(alpha) * _bound(Ao, Bo, k) + 4 * 2.0 ** -53 * np.abs(beta * Co) + 1e-15 * (k == 0))


def test_dgemm_beta_zero_ignores_nan():
    require_gpu()
    from paper_2308_14490_amd import azrbf
    dev = torch.device("cuda", 0)
    A = torch.ones((5, 70), dtype=torch.float64, device=dev)     # 70 x 5
    B = torch.ones((3, 5), dtype=torch.float64, device=dev)      # 5 x 3
    C = torch.full((3, 70), float("nan"), dtype=torch.float64, device=dev)
    azrbf.dgemm(A, B, C)
    torch.cuda.synchronize()
    assert torch.all(C == 5.0)
