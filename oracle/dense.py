"""Dense least-squares systems, entry by entry.

1D approximation (section 2.3):  A_ij = phi_j(x_i) = phi_per(x_i - c_j).
2D approximation (section 5.2, eq. Aa_is_b_2d): the basis function
    phi_j(x, y) = phi_per(x - cx_m) phi_per(y - cy_n),  j = m*Ny + n
(each axis periodized with its own box half-width T^x, T^y).
(the Gaussian is a product of univariate Gaussians, section 5).
Boundary value problems (section 6): interior rows apply the operator to the
basis, boundary rows evaluate it at boundary points (eq. Ai_2d_bvp and the
A^b block).  The operator is written -(Laplacian + k2) and its rows are
divided by 4 eps^2 (= -Laplacian phi at r = 0) so that their size matches the
approximation rows; section 6.1 does the same in 1D with the factor -2 eps^2.
Boundary rows carry a weight w_b (1 in the paper).  Dirichlet rows are
w_b phi_j(x_b); Neumann rows (section 6.3, the normal derivative at a point
of the boundary) are w_b n . grad phi_j(x_b) / eps, divided by eps so that
their size matches the Dirichlet rows (|phi'| peaks at eps sqrt(2/e)); their
data are scaled the same way.
"""
import numpy as np

from . import grids
from .rbf import phi_per, phi1_per, phi2_per


def basis_1d(x, n, T, eps, deriv=0):
    """Matrix [phi_per^(deriv)(x_i - c_j)]_{i,j}, x of shape (m,), deriv 0, 1 or 2."""
    c = grids.centres(n, T)
    d = np.subtract.outer(np.asarray(x, dtype=np.float64), c)
    return (phi_per, phi1_per, phi2_per)[deriv](d, eps, T)


def _rowkron(a, b):
    """Row-wise Kronecker product: out[i, m*nb + n] = a[i, m] * b[i, n]."""
    return (a[:, :, None] * b[:, None, :]).reshape(a.shape[0], -1)


def interior_rows(prob, pts):
    """Rows of the interior block at points ``pts`` (m, dim)."""
    n, T, eps = prob.n, prob.T, prob.eps
    if prob.dim == 1:
        x = pts[:, 0]
        if prob.op == 0:
            return basis_1d(x, n, T, eps)
        a2 = basis_1d(x, n, T, eps, 2)
        a0 = basis_1d(x, n, T, eps, 0)
        return -(a2 + prob.k2 * a0) / (2.0 * eps * eps)
    ny, Ty = prob.n_y, prob.T_y
    ax0 = basis_1d(pts[:, 0], n, T, eps)
    ay0 = basis_1d(pts[:, 1], ny, Ty, eps)
    if prob.op == 0:
        return _rowkron(ax0, ay0)
    ax2 = basis_1d(pts[:, 0], n, T, eps, 2)
    ay2 = basis_1d(pts[:, 1], ny, Ty, eps, 2)
    lap = _rowkron(ax2, ay0) + _rowkron(ax0, ay2)
    return -(lap + prob.k2 * _rowkron(ax0, ay0)) / (4.0 * eps * eps)


def boundary_rows(prob, bpts, types=None, normals=None):
    """Rows at boundary points ``bpts`` (mb, dim): w_b phi_j (Dirichlet,
    type 0) or w_b n . grad phi_j / eps (Neumann, type 1, unit outward normal
    n).  Types and normals default to the problem's."""
    n, T, eps = prob.n, prob.T, prob.eps
    if bpts.shape[0] == 0:
        return np.zeros((0, prob.N))
    types = prob.btypes() if types is None else types
    normals = prob.bnormals() if normals is None else normals
    neu = (np.asarray(types) != 0)[:, None]
    if prob.dim == 1:
        rows = np.where(neu, normals[:, :1] * basis_1d(bpts[:, 0], n, T, eps, 1) / eps,
                        basis_1d(bpts[:, 0], n, T, eps))
        return prob.bweight * rows
    ax0 = basis_1d(bpts[:, 0], n, T, eps)
    ay0 = basis_1d(bpts[:, 1], prob.n_y, prob.T_y, eps)
    rows = _rowkron(ax0, ay0)
    if np.any(neu):
        ax1 = basis_1d(bpts[:, 0], n, T, eps, 1)
        ay1 = basis_1d(bpts[:, 1], prob.n_y, prob.T_y, eps, 1)
        grad_n = (normals[:, :1] * _rowkron(ax1, ay0) + normals[:, 1:2] * _rowkron(ax0, ay1)) / eps
        rows = np.where(neu, grad_n, rows)
    return prob.bweight * rows


def system_matrix(prob):
    """(A, idx, pts, bpts): the full (M + Mb) x N matrix and its row data."""
    idx, pts = grids.collocation(prob)
    bpts = prob.bpoints()
    A = interior_rows(prob, pts)
    if bpts.shape[0]:
        A = np.vstack([A, boundary_rows(prob, bpts)])
    return A, idx, pts, bpts


def _scale(prob):
    return 2.0 * prob.eps ** 2 if prob.dim == 1 else 4.0 * prob.eps ** 2


def rhs(prob, pts, bpts, which=None):
    """Right-hand sides as columns, (M + Mb, nrhs).

    Approximation: b_i = f(x_i).  BVP, equation -(Lap + k2) u = f with u = g
    (Dirichlet points) or du/dn = h (Neumann points) on the boundary:
    interior rows f / (4 eps^2) (2D) or f / (2 eps^2) (1D), boundary rows
    w_b g or w_b h / eps.
    """
    fs = prob.rhs if which is None else [prob.rhs[i] for i in which]
    cols = []
    for i, f in enumerate(fs):
        v = f(*pts.T)
        if prob.op != 0:
            v = v / _scale(prob)
            j = i if which is None else which[i]
            scale = np.where(prob.btypes() != 0, 1.0 / prob.eps, 1.0)
            v = np.concatenate([v, prob.bweight * scale * prob.bdata(j, bpts)])
        cols.append(v)
    return np.stack(cols, axis=1)
