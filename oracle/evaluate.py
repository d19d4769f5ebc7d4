"""Residuals and evaluation of the approximant.

The approximant is f(x) ~ sum_j a_j phi_j(x) (section 2.1; 2D section 5.1).
Dense evaluation builds the rows phi_j(t) at the test points.  For sizes where
the dense matrix does not fit, ``apply_local`` evaluates the same sums by
direct local summation: the Gaussian is below 1e-20 beyond 6.8/eps, so each
point only sums the centres within that window (periodic distance).  No FFT
is involved, so the result is independent of the GPU path's arithmetic.
"""
import math

import numpy as np

from . import dense
from .rbf import phi, phi1, phi2


def relres(A, x, b):
    r = A @ x - b
    if b.ndim == 1:
        return float(np.linalg.norm(r) / np.linalg.norm(b))
    return np.linalg.norm(r, axis=0) / np.linalg.norm(b, axis=0)


def eval_dense(prob, coef, tpts, chunk=4096):
    """Approximant at test points (rows of the approximation basis)."""
    out = []
    aprob = _as_approx(prob)
    for i in range(0, tpts.shape[0], chunk):
        out.append(dense.interior_rows(aprob, tpts[i:i + chunk]) @ coef)
    return np.concatenate(out, axis=0)


def _as_approx(prob):
    import copy
    p = copy.copy(prob)
    p.op = 0
    return p


def _window_1d(t, n, T, eps, deriv):
    """Centre indices and kernel values for points t, shape (m, 2W+1)."""
    h = 2.0 * T / n
    W = int(math.ceil(6.8 / (eps * h))) + 1
    j0 = np.floor((t + T) / h).astype(np.int64)
    off = np.arange(-W, W + 2)
    j = j0[:, None] + off[None, :]
    d = t[:, None] - (-T + j * h)                # unreduced distance, |d| <= (W+1)h
    jj = np.mod(j, n)
    f = (phi, phi1, phi2)[deriv]
    v = f(d, eps)
    if (W + 1) * h * 2 > 2 * T:
        raise ValueError("window wider than the box; use dense evaluation")
    return jj, v


def apply_local(prob, coef, pts, op=None):
    """Rows of the system at ``pts`` applied to coef (N,) or (N, nrhs).

    op: 0 approximation rows, else the scaled operator rows (as dense.py).
    """
    op = prob.op if op is None else op
    n, T, eps = prob.n, prob.T, prob.eps
    C = coef if coef.ndim == 2 else coef[:, None]
    if prob.dim == 1:
        jx, vx = _window_1d(pts[:, 0], n, T, eps, 0)
        if op == 0:
            out = np.einsum("mw,mwr->mr", vx, C[jx])
        else:
            _, vx2 = _window_1d(pts[:, 0], n, T, eps, 2)
            out = np.einsum("mw,mwr->mr", -(vx2 + prob.k2 * vx) / (2 * eps * eps), C[jx])
        return out if coef.ndim == 2 else out[:, 0]
    ny, Ty = prob.n_y, prob.T_y
    C3 = C.reshape(n, ny, -1)
    jx, vx = _window_1d(pts[:, 0], n, T, eps, 0)
    jy, vy = _window_1d(pts[:, 1], ny, Ty, eps, 0)
    out = np.zeros((pts.shape[0], C.shape[1]))
    if op == 0:
        for a in range(jx.shape[1]):
            out += vx[:, a:a + 1] * np.einsum("mw,mwr->mr", vy, C3[jx[:, a:a + 1], jy])
    else:
        _, vx2 = _window_1d(pts[:, 0], n, T, eps, 2)
        _, vy2 = _window_1d(pts[:, 1], ny, Ty, eps, 2)
        s = -1.0 / (4 * eps * eps)
        for a in range(jx.shape[1]):
            g = C3[jx[:, a:a + 1], jy]             # (m, Wy, r)
            t0 = np.einsum("mw,mwr->mr", vy, g)
            t2 = np.einsum("mw,mwr->mr", vy2, g)
            out += s * (vx2[:, a:a + 1] * t0 + vx[:, a:a + 1] * t2
                        + prob.k2 * vx[:, a:a + 1] * t0)
    return out if coef.ndim == 2 else out[:, 0]


def apply_boundary_local(prob, coef, bpts=None, types=None, normals=None):
    """The boundary rows of dense.boundary_rows applied to coef (N,) or
    (N, nrhs) by local sums: w_b u(x_b) at Dirichlet points, w_b n . grad
    u(x_b) / eps at Neumann points."""
    bpts = prob.bpoints() if bpts is None else bpts
    types = prob.btypes() if types is None else np.asarray(types)
    normals = prob.bnormals() if normals is None else normals
    n, T, eps = prob.n, prob.T, prob.eps
    C = coef if coef.ndim == 2 else coef[:, None]
    neu = (types != 0)[:, None]
    if prob.dim == 1:
        jx, vx = _window_1d(bpts[:, 0], n, T, eps, 0)
        _, vx1 = _window_1d(bpts[:, 0], n, T, eps, 1)
        val = np.einsum("mw,mwr->mr", vx, C[jx])
        dn = normals[:, :1] * np.einsum("mw,mwr->mr", vx1, C[jx]) / eps
    else:
        ny, Ty = prob.n_y, prob.T_y
        C3 = C.reshape(n, ny, -1)
        jx, vx = _window_1d(bpts[:, 0], n, T, eps, 0)
        jy, vy = _window_1d(bpts[:, 1], ny, Ty, eps, 0)
        _, vx1 = _window_1d(bpts[:, 0], n, T, eps, 1)
        _, vy1 = _window_1d(bpts[:, 1], ny, Ty, eps, 1)
        val = np.zeros((bpts.shape[0], C.shape[1]))
        dx = np.zeros_like(val)
        dy = np.zeros_like(val)
        for a in range(jx.shape[1]):
            g = C3[jx[:, a:a + 1], jy]
            t0 = np.einsum("mw,mwr->mr", vy, g)
            t1 = np.einsum("mw,mwr->mr", vy1, g)
            val += vx[:, a:a + 1] * t0
            dx += vx1[:, a:a + 1] * t0
            dy += vx[:, a:a + 1] * t1
        dn = (normals[:, :1] * dx + normals[:, 1:2] * dy) / eps
    out = prob.bweight * np.where(neu, dn, val)
    return out if coef.ndim == 2 else out[:, 0]
