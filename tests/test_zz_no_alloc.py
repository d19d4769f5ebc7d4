"""azrbf_dgemm_noalloc, the GEMM entry point that allocates nothing (split-K
partials in the library's fixed per-GPU array), against azrbf_dgemm, which
allocates them: called through the C ABI twice in a row, the second time on
a smaller product, and compared bit for bit (same split, same kernels) and
with the FP64 product on the CPU to the GEMM's rounding bound."""
import ctypes

import numpy as np
import pytest
import torch

from gpu_util import announce, require_gpu

pytestmark = pytest.mark.gpu
U = 2.0 ** -53


def _call(fn, ta, tb, m, n, k, alpha, A, lda, B, ldb, beta, C, ldc):
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return fn(ta, tb, m, n, k, alpha, A.data_ptr(), lda, B.data_ptr(), ldb, beta, C.data_ptr(), ldc, st)


def _case(lib, ta, tb, m, n, k, alpha, beta, seed):
    """Column-major operands held as (cols, ld) tensors."""
    announce("dgemm_noalloc", ta, tb, m, n, k, alpha, beta)
    rng = np.random.default_rng(seed)
    ar, ac = (k, m) if ta else (m, k)
    br, bc = (n, k) if tb else (k, n)
    lda, ldb, ldc = ar + 3, br + 1, m + 5
    A = rng.standard_normal((ac, lda))
    B = rng.standard_normal((bc, ldb))
    C0 = rng.standard_normal((n, ldc))
    Ad, Bd = torch.from_numpy(A).cuda(), torch.from_numpy(B).cuda()
    C1, C2 = torch.from_numpy(C0).cuda(), torch.from_numpy(C0).cuda()
    assert _call(lib.azrbf_dgemm, ta, tb, m, n, k, alpha, Ad, lda, Bd, ldb, beta, C1, ldc) == 0
    assert _call(lib.azrbf_dgemm_noalloc, ta, tb, m, n, k, alpha, Ad, lda, Bd, ldb, beta, C2, ldc) == 0
    torch.cuda.synchronize()
    assert torch.equal(C1, C2)
    Am = A[:, :ar].T                                       # the stored ar x ac matrix
    Bm = B[:, :br].T
    oA = Am.T if ta else Am
    oB = Bm.T if tb else Bm
    want = alpha * (oA @ oB) + beta * C0[:, :m].T
    bound = (k + 2) * U * (abs(alpha) * (np.abs(oA) @ np.abs(oB)) + abs(beta) * np.abs(C0[:, :m].T))
    got = C2.cpu().numpy()[:, :m].T
    assert np.all(np.abs(got - want) <= bound + 1e-300)
    # rows past m of each column (ld padding) are untouched
    assert np.array_equal(C2.cpu().numpy()[:, m:], C0[:, m:])


def test_noalloc_gemm_matches_allocating_entry_point():
    require_gpu()
    from paper_2308_14490_amd import azrbf
    lib = azrbf._lib()
    # tall-skinny Q^T C shape (split over 256 blocks), then a smaller product
    # on the same array (split over 19 blocks), then an unsplit one
    _case(lib, 1, 0, 32, 64, 65552, 1.0, 0.0, 1)
    _case(lib, 1, 0, 16, 8, 5000, -0.5, 2.0, 2)
    _case(lib, 0, 1, 300, 200, 96, 1.0, 1.0, 3)


def test_noalloc_gemm_rejects_a_split_beyond_its_array():
    """960 x 960 output, reduction 4096: the split needs 4.6 M doubles, more
    than the 2^20 of the fixed array, so the call returns ESCRATCH and leaves
    C unchanged."""
    require_gpu()
    from paper_2308_14490_amd import azrbf
    lib = azrbf._lib()
    m = n = 960
    k = 4096
    A = torch.ones((m, k), dtype=torch.float64, device="cuda")     # op(A) = A^T, k x m stored
    B = torch.ones((n, k), dtype=torch.float64, device="cuda")
    C = torch.full((n, m), 7.0, dtype=torch.float64, device="cuda")
    rc = _call(lib.azrbf_dgemm_noalloc, 1, 0, m, n, k, 1.0, A, k, B, k, 0.0, C, m)
    torch.cuda.synchronize()
    assert rc == azrbf.ESCRATCH
    assert b"scratch" in lib.azrbf_strerror(rc)
    assert float(C.min()) == 7.0 and float(C.max()) == 7.0
    # the allocating entry point computes it
    assert _call(lib.azrbf_dgemm, 1, 0, m, n, k, 1.0, A, k, B, k, 0.0, C, m) == 0
    torch.cuda.synchronize()
    assert float(C.min()) == float(k) and float(C.max()) == float(k)
