"""Truncated-SVD least squares: the oracle's solver.

For the rectangular systems of the paper (eq. Ax_is_b, eq. Aa_is_b_2d) the
regularised least-squares solution is
    x = sum_{sigma_i > tau * sigma_1} v_i (u_i^T b) / sigma_i,
the truncated SVD solution that the frame analysis cited in section 4.1
relies on.  The SVD is LAPACK's divide-and-conquer (numpy.linalg.svd).
"""
import numpy as np


def tsvd(A):
    return np.linalg.svd(A, full_matrices=False)


def tsvd_solve(A, b, tau=1e-12, svd=None, sigma_ref=None):
    """Truncated-SVD solution; b may hold several right-hand sides as columns.

    Returns (x, rank).  Singular values at or below tau * sigma_ref are
    dropped (sigma_ref defaults to the largest singular value).
    """
    U, S, Vt = tsvd(A) if svd is None else svd
    ref = S[0] if sigma_ref is None else sigma_ref
    keep = S > tau * ref
    r = int(np.count_nonzero(keep))
    Ur, Sr, Vr = U[:, keep], S[keep], Vt[keep].T
    coef = (Ur.T @ b)
    coef = coef / (Sr[:, None] if coef.ndim == 2 else Sr)
    return Vr @ coef, r


def numerical_rank(A, tau):
    S = np.linalg.svd(A, compute_uv=False)
    return int(np.count_nonzero(S > tau * S[0])) if S.size else 0
