"""The periodic solver and the incomplete generalised inverse Z* (sections 3.1,
3.2, 5.1, 5.2, 6.1, 6.2), built from explicit matrices.

Section 3.1: the L x N periodic matrix A^c (eq. matrix_entries) is permuted by
Pi into s stacked circulant N x N blocks (eq. circulant_system_pi).  With the
unitary DFT matrix F_kl = exp(2 pi i (k-1)(l-1)/N)/sqrt(N) and P the
block-diagonal matrix with F* on its diagonal (eq. P),
    B = P Pi A^c F
is block-column diagonal with diagonals d_1..d_s, and its pseudo-inverse
(eq. B_pinv) has diagonal blocks conj(d_i) / sum_j |d_j|^2.  Section 3.2
defines Z* = F B^+ P E with E the zero-padding extension.  In 2D everything
is a Kronecker product over the axes (eq. circulant_system_2d, B_pinv_2d);
for boundary value problems B is a sum of Kronecker products and
B^+ = (B*B)^{-1} B* with B*B diagonal (section 6.2), and Z* gets zero columns
for the boundary rows.

Regularisation (the paper inverts sum_j |d_j|^2 exactly): weights whose
denominator is at or below tauZ * max are set to zero.  This matters where
the symbol vanishes (the zero mode of the Laplacian) and is inactive
otherwise.  Collocation rows are kept in natural grid order, so E here is
Pi^T composed with zero padding in natural order.
"""
import numpy as np

from . import dense, grids


def dft_matrix(n):
    k = np.arange(n)
    return np.exp(2j * np.pi * np.outer(k, k) / n) / np.sqrt(n)


def pi_perm(n, s):
    """Row order of Pi A^c: block r holds rows r, r+s, r+2s, ... (0-based)."""
    return np.array([r + s * j for r in range(s) for j in range(n)])


def periodic_matrix(prob):
    """A^c (or A^ic for BVPs): the interior operator at every fine-grid point."""
    xt = grids.fine_grid(prob.n, prob.s, prob.T)
    if prob.dim == 1:
        return dense.interior_rows(prob, xt[:, None])
    yt = grids.fine_grid(prob.n_y, prob.s, prob.T_y)
    X, Y = np.meshgrid(xt, yt, indexing="ij")
    return dense.interior_rows(prob, np.stack([X.ravel(), Y.ravel()], axis=1))


def _pi_full(prob):
    p1 = pi_perm(prob.n, prob.s)
    if prob.dim == 1:
        return p1
    p2 = pi_perm(prob.n_y, prob.s)
    Ly = prob.n_y * prob.s
    return (p1[:, None] * Ly + p2[None, :]).ravel()


def _F_full(prob):
    F1 = dft_matrix(prob.n)
    return F1 if prob.dim == 1 else np.kron(F1, dft_matrix(prob.n_y))


def _P_full(prob):
    P1 = np.kron(np.eye(prob.s), dft_matrix(prob.n).conj().T)
    if prob.dim == 1:
        return P1
    return np.kron(P1, np.kron(np.eye(prob.s), dft_matrix(prob.n_y).conj().T))


def _block_rows(prob):
    """Row order that makes the diagonal blocks of B contiguous.

    In 1D the rows of P Pi A^c F already come in s blocks of N.  In 2D the
    Kronecker product interleaves them: block (rx, ry) = D^x_rx (x) D^y_ry
    sits at rows (rx n_x + kx) s n_y + ry n_y + ky.  Listing, for each block,
    its rows in (kx, ky) order groups them.
    """
    n, s = prob.n, prob.s
    if prob.dim == 1:
        return np.arange(s * n)
    ny = prob.n_y
    kx, ky = np.meshgrid(np.arange(n), np.arange(ny), indexing="ij")
    return np.concatenate([((rx * n + kx) * (s * ny) + ry * ny + ky).ravel()
                           for rx in range(s) for ry in range(s)])


def block_diagonal_form(prob):
    """B = P Pi A^c F with rows grouped into s^dim diagonal N x N blocks."""
    Ac = periodic_matrix(prob)
    B = _P_full(prob) @ Ac[_pi_full(prob)] @ _F_full(prob)
    return B[_block_rows(prob)]


def diagonals(B, N):
    """Diagonals d_i of the stacked N x N blocks of B, shape (blocks, N)."""
    nb = B.shape[0] // N
    return np.stack([np.diag(B[i * N:(i + 1) * N]) for i in range(nb)])


def bpinv(d, tauZ):
    """B^+ from the diagonals: block i is diag(conj(d_i) / sum_j |d_j|^2)."""
    D = np.sum(np.abs(d) ** 2, axis=0)
    w = np.where(D > tauZ * D.max(), 1.0 / np.where(D > 0, D, 1.0), 0.0)
    return np.hstack([np.diag(np.conj(di) * w) for di in d])


def zstar(prob, idx, tauZ=1e-12, nb=0):
    """Z* = F B^+ P E as a real N x (M + nb) matrix, built literally.

    Intended for small grids (2D: n up to about 16).  Returns (Z, imag_max)
    where imag_max is the largest imaginary part discarded.
    """
    N = prob.N
    B = block_diagonal_form(prob)
    Bp = bpinv(diagonals(B, N), tauZ)
    L = prob.N * prob.s ** prob.dim
    E = np.zeros((L, idx.size))
    E[idx, np.arange(idx.size)] = 1.0
    PE = _P_full(prob) @ E[_pi_full(prob)]
    Zc = _F_full(prob) @ Bp @ PE[_block_rows(prob)]
    Z = np.real(Zc)
    if nb:
        Z = np.hstack([Z, np.zeros((N, nb))])
    return Z, float(np.max(np.abs(np.imag(Zc)))) if Zc.size else 0.0


def symbol_weights(prob, tauZ=1e-12):
    """Regularised 1 / diag(B*B) on the coefficient Fourier grid.

    By Lemma 4.2 the diagonal d_i of block i of B is the DFT of the first
    column of the circulant block A^c_i, i.e. of the operator's kernel
    sampled on the i-th shifted grid; diag(B*B) = sum_i |d_i|^2.  In 2D the
    blocks are indexed by the pair of shifts and the DFT is 2D.
    """
    Ac = periodic_matrix(prob)
    col = Ac[:, 0]                              # kernel of centre c_0 on the fine grid
    s, n = prob.s, prob.n
    if prob.dim == 1:
        D = sum(np.abs(np.fft.fft(col[r::s])) ** 2 for r in range(s))
    else:
        g = col.reshape(s * n, s * prob.n_y)
        D = sum(np.abs(np.fft.fft2(g[rx::s, ry::s])) ** 2
                for rx in range(s) for ry in range(s)).ravel()
    return np.where(D > tauZ * D.max(), 1.0 / np.where(D > 0, D, 1.0), 0.0), D


def zstar_normal(prob, idx, tauZ=1e-12, nb=0):
    """Z* written as F diag(w) F* A^cT E: since P is unitary and Pi a
    permutation, F B^+ P E = F (B*B)^{-1} F* (Pi A^c)^T Pi E, and F (.) F* of a
    diagonal is the circulant with that symbol, applied here with FFTs.  The
    same operator as ``zstar``, for moderate grids without forming the
    sN x sN matrix P."""
    Ac = periodic_matrix(prob)
    w, _ = symbol_weights(prob, tauZ)
    N = prob.N
    G = Ac[idx].T                                # N x M  (A^cT E)
    if prob.dim == 1:
        Z = np.real(np.fft.ifft(w[:, None] * np.fft.fft(G, axis=0), axis=0))
    else:
        n, ny = prob.n, prob.n_y
        G3 = G.reshape(n, ny, -1)
        Z = np.real(np.fft.ifft2(w.reshape(n, ny)[:, :, None] *
                                 np.fft.fft2(G3, axes=(0, 1)), axes=(0, 1)))
        Z = Z.reshape(N, -1)
    if nb:
        Z = np.hstack([Z, np.zeros((N, nb))])
    return Z
