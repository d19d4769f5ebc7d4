"""The AZ algorithm (section 3.2, Algorithm 1) with dense matrices.

Given A (M x N), the incomplete generalised inverse Z* (N x M) and b:
  step 1  solve (I - A Z*) A x1 = (I - A Z*) b        (a low-rank system)
  step 2  x2 = Z* (b - A x1)
  step 3  x = x1 + x2
Naming: the step-1 solution is x1 and the step-2 part x2, as in Lemma 4.1;
Algorithm 1 prints the two labels the other way round.

Step 1 is a least-squares solve with a numerically low-rank matrix.  The
paper solves it with randomized linear algebra (section 3.2.3): r + p products
with a random matrix, then an SVD of the sketch.  With a sketch matrix Omega
(N x k): W = (A - A Z* A) Omega, y = truncated-SVD solution of
W y = (I - A Z*) b, x1 = Omega y.  Without Omega the truncated SVD of
A - A Z* A itself is used.

Truncation of the sketch: singular values of W at or below
tau * normA * sqrt(k) are dropped.  A Gaussian N x k sketch of a low-rank
matrix scales its singular values by about sqrt(k), so this keeps the
directions of A - A Z* A above tau * normA.  normA is the norm of the
periodic operator, sqrt(max diag(B*B)).

Refinement (not in Algorithm 1): ``refine`` further passes of the same three
steps applied to the current residual, reusing the step-1 factor.  The
final residual of each pass is (I - A Z*)(r - A x1) (Algorithm 1, steps 2-3),
so a pass can only reduce it within the retained subspace.
"""
import numpy as np

from .lstsq import tsvd, tsvd_solve


def az_factor(A, Z, Omega, tau, normA):
    """SVD of the sketch W = (A - A Z* A) Omega, truncated.

    Returns (G, rank, W) with G = V_r S_r^{-1} U_r^T, so y = G c.
    """
    K = A - (A @ Z) @ A
    W = K @ Omega
    U, S, Vt = tsvd(W)
    keep = S > tau * normA * np.sqrt(Omega.shape[1])
    G = (Vt[keep].T / S[keep]) @ U[:, keep].T
    return G, int(np.count_nonzero(keep)), W


def az_solve(A, Z, b, tau=1e-12, Omega=None, normA=None, refine=0):
    """Returns dict(x, x1, x2, rank, W, resid) (x1, x2 of the first pass)."""
    if normA is None:
        normA = np.linalg.norm(A, 2)
    AZ = A @ Z
    if Omega is None:
        K = A - AZ @ A

        def step1(c):
            return tsvd_solve(K, c, tau, sigma_ref=normA)[0]
        rank = None
        W = None
    else:
        G, rank, W = az_factor(A, Z, Omega, tau, normA)

        def step1(c):
            return Omega @ (G @ c)
    x = np.zeros((A.shape[1],) + b.shape[1:])
    r = b.copy()
    first = None
    for _ in range(refine + 1):
        c = r - AZ @ r                   # (I - A Z*) r
        x1 = step1(c)
        r1 = r - A @ x1
        x2 = Z @ r1                      # step 2
        x = x + x1 + x2                  # step 3
        r = b - A @ x
        if first is None:
            first = (x1, x2)
    return dict(x=x, x1=first[0], x2=first[1], rank=rank, W=W, resid=r)
