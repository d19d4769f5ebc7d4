"""Centres, the oversampled grid and collocation subsets.

c_j = -T + (j-1) 2T/N,  j = 1..N                 eq. (set_centers)
x~_i = -T + (i-1) 2T/L, i = 1..L, L = sN          eq. (set_Xtilde)
X = { x in X~ : x in Omega }                       eq. (set_X)
X = (X~ x Y~) intersect Omega  (2D)                eq. (set_X_2d)
(in 2D each axis has its own centre count and box half-width, section 5.1)

Indices here are 0-based.  2D grids are ordered with x slow and y fast,
j = jx * Ny + jy, matching the coefficient ordering of section 5.1.  The
collocation points keep the natural (ascending, row-major) grid order; the
paper orders them by the permutation Pi instead, which permutes rows of the
least-squares system and does not change its solution.
"""
import numpy as np


def centres(n, T):
    return -T + np.arange(n, dtype=np.float64) * (2.0 * T / n)


def fine_grid(n, s, T):
    L = s * n
    return -T + np.arange(L, dtype=np.float64) * (2.0 * T / L)


def collocation_1d(n, s, T, domain):
    """Indices into the fine grid of points inside ``domain`` and the points."""
    xt = fine_grid(n, s, T)
    idx = np.nonzero(domain.contains(xt))[0]
    return idx, xt[idx]


def collocation_2d(n, s, T, domain, ny=None, Ty=None):
    """Flat indices ix*Ly + iy of fine-grid points inside ``domain``; (M, 2).
    The y axis has ny centres on [-Ty, Ty) (default: n, T)."""
    xt = fine_grid(n, s, T)
    yt = fine_grid(n if ny is None else ny, s, T if Ty is None else Ty)
    X, Y = np.meshgrid(xt, yt, indexing="ij")
    flat = domain.contains(X, Y).ravel()
    idx = np.nonzero(flat)[0]
    Ly = yt.size
    pts = np.stack([xt[idx // Ly], yt[idx % Ly]], axis=1)
    return idx, pts


def collocation(prob):
    if prob.dim == 1:
        idx, x = collocation_1d(prob.n, prob.s, prob.T, prob.domain)
        return idx, x[:, None]
    return collocation_2d(prob.n, prob.s, prob.T, prob.domain, prob.n_y, prob.T_y)
