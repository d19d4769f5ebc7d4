"""The periodic problems (sections 3.1 and 5.1): the domain is the whole box,
so A is the periodic matrix A^c and Z* is its exact pseudo-inverse wherever
the regularisation keeps the weight (Z* A^c = I, section 4.1).  Checked at
full size against the closed-form symbol of the kernel (Lemma 4.3, from the
oracle), and the AZ solve of the paper's periodic experiments (section 3.3,
Fig. 3.1; section 5.4) against the oracle and the accuracy the paper states.
"""
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle import dense, evaluate, lstsq, spectra

from gpu_util import announce, require_gpu

pytestmark = pytest.mark.gpu
U = 2.0 ** -53


def _mods():
    require_gpu()
    from paper_2308_14490_amd import azrbf, problems
    return azrbf, problems


def _symbol_1d(n, s, T, eps):
    """sum_r |d_r|^2 over the s shifted grids, closed form (Lemma 4.3)."""
    return sum(np.abs(spectra.diag_closed_form(n, s, T, eps, r)) ** 2 for r in range(s))


@pytest.mark.parametrize("dim,n,nvec", [(1, 65536, 8), (2, 256, 4)])
def test_zstar_inverts_the_periodic_matrix_full_size(dim, n, nvec):
    """Z* (A X) = X on the kept Fourier modes.  In 1D at eps*h = 0.5 nothing
    is zeroed; in 2D the symbol is the product of the axes' and its smallest
    entries fall below 1e-12 of the largest, so the identity holds for the
    modes the regularisation keeps: X projected onto them by a DFT.  Rounding
    of the FFTs (u log2 N) is amplified by at most ||A^c|| ||Z*||."""
    azrbf, problems = _mods()
    prob = W.Problem("box", dim, n, 2, 1.0, 0.5, W.box(1.0, dim), [])
    p = problems.plan_for(prob)
    announce("box identity", dim, n, "M", p.M)
    assert p.M == (2 * n) ** dim
    D1 = _symbol_1d(n, 2, 1.0, prob.eps)
    D = D1 if dim == 1 else np.outer(D1, D1).ravel()
    keep = D > 1e-12 * D.max()
    normA, normZ = math.sqrt(D.max()), 1.0 / math.sqrt(D[keep].min())
    rng = np.random.default_rng(5)
    X = rng.standard_normal((nvec, prob.N))
    if not keep.all():
        Xf = np.fft.fft2(X.reshape(nvec, n, n)) * keep.reshape(n, n)
        X = np.real(np.fft.ifft2(Xf)).reshape(nvec, -1)
    Xd = torch.from_numpy(X).cuda()
    Y = azrbf.apply_A(p, Xd)
    Z = azrbf.apply_Zstar(p, Y).cpu().numpy()
    err = np.max(np.abs(Z - X)) / np.max(np.abs(X))
    tol = 20 * U * math.log2(prob.N) * normA * normZ
    announce("zeroed", int((~keep).sum()), "err", err, "tol", tol)
    assert err < tol
    p.destroy()


def _periodic_case(dim, n, s, tau0, f):
    eh = W.shape_parameter_eh(tau0)
    return W.Problem(f"periodic{dim}d", dim, n, s, 1.0, eh, W.box(1.0, dim), [f], k=32 if dim == 1 else 0)


@pytest.mark.parametrize("n,s", [(256, 2), (1024, 2), (256, 3), (1024, 3)])
def test_periodic_1d_solve_matches_oracle_and_paper(n, s):
    """f = sin([N/5] pi x) on the periodic box, T = 1, tau0 = 1e-10: the first
    experiment of section 3.3 (s = 3, Fig. 3.1), and the same at s = 2.  The
    paper reports a maximum error below 1e-12 and a coefficient norm
    ||a|| / sqrt(N) of about 5 (checked within a factor 1.5 at s = 3)."""
    azrbf, problems = _mods()
    kk = math.floor(n / 5)
    prob = _periodic_case(1, n, s, 1e-10, lambda x: np.sin(kk * np.pi * x))
    p = problems.plan_for(prob)
    B = problems.rhs_for(p, prob)
    X, rel = azrbf.solve(p, B)
    torch.cuda.synchronize()
    Xg = X.cpu().numpy().T
    A, idx, pts, bpts = dense.system_matrix(prob)
    Bo = dense.rhs(prob, pts, bpts)
    Xo, _ = lstsq.tsvd_solve(A, Bo, 1e-12)
    tp = W.test_points(prob)
    f = prob.rhs[0](tp[:, 0])
    eg = np.abs(evaluate.eval_dense(prob, Xg, tp)[:, 0] - f).max()
    eo = np.abs(evaluate.eval_dense(prob, Xo, tp)[:, 0] - f).max()
    rg, ro = evaluate.relres(A, Xg, Bo), evaluate.relres(A, Xo, Bo)
    cn = np.linalg.norm(Xg) / math.sqrt(n)
    announce("periodic 1D", n, "s", s, "rank", p.info()["rank"], "relres", rg, ro, "maxerr", eg, eo, "||a||/sqrt(N)", cn)
    assert np.all(rg <= 10 * ro + 1e-15)
    assert eg <= 10 * eo + 1e-15 and eg < 1e-12
    if s == 3:
        assert 5.0 / 1.5 < cn < 5.0 * 1.5
    p.destroy()


def test_periodic_2d_solve_matches_oracle_and_paper():
    """f = sin([N/10] pi (x + y)) on the periodic square, s = 2, tau0 = 1e-5
    (the first experiment of section 5.4): maximum error around 1e-12."""
    azrbf, problems = _mods()
    n = 32
    kk = math.floor(n / 10)
    prob = _periodic_case(2, n, 2, 1e-5, lambda x, y: np.sin(kk * np.pi * (x + y)))
    p = problems.plan_for(prob)
    B = problems.rhs_for(p, prob)
    X, rel = azrbf.solve(p, B)
    torch.cuda.synchronize()
    Xg = X.cpu().numpy().T
    A, idx, pts, bpts = dense.system_matrix(prob)
    Bo = dense.rhs(prob, pts, bpts)
    Xo, _ = lstsq.tsvd_solve(A, Bo, 1e-12)
    tp = W.test_points(prob, m2d=61)
    f = prob.rhs[0](tp[:, 0], tp[:, 1])
    eg = np.abs(evaluate.eval_dense(prob, Xg, tp)[:, 0] - f).max()
    eo = np.abs(evaluate.eval_dense(prob, Xo, tp)[:, 0] - f).max()
    rg, ro = evaluate.relres(A, Xg, Bo), evaluate.relres(A, Xo, Bo)
    announce("periodic 2D", n, "k", p.info()["k"], "rank", p.info()["rank"], "relres", rg, ro, "maxerr", eg, eo)
    assert np.all(rg <= 10 * ro + 1e-15)
    assert eg <= 10 * eo + 1e-15 and eg < 1e-11
    p.destroy()


def test_zstar_inverts_the_periodic_matrix_anisotropic():
    """Z* A^c = I on the kept modes of the anisotropic box [-1.4, 1.4] x
    [-0.7, 0.7] with 256 x 128 centres."""
    azrbf, problems = _mods()
    nx, ny = 256, 128
    prob = W.Problem("box-aniso", 2, nx, 2, 1.4, 0.5, W.box(1.4, 2, 0.7), [], ny=ny, Ty=0.7)
    p = problems.plan_for(prob)
    assert p.M == 4 * nx * ny
    Dx = _symbol_1d(nx, 2, 1.4, prob.eps)
    Dy = _symbol_1d(ny, 2, 0.7, prob.eps)
    D = np.outer(Dx, Dy).ravel()
    keep = D > 1e-12 * D.max()
    normA, normZ = math.sqrt(D.max()), 1.0 / math.sqrt(D[keep].min())
    rng = np.random.default_rng(6)
    X = rng.standard_normal((3, prob.N))
    Xf = np.fft.fft2(X.reshape(3, nx, ny)) * keep.reshape(nx, ny)
    X = np.real(np.fft.ifft2(Xf)).reshape(3, -1)
    Z = azrbf.apply_Zstar(p, azrbf.apply_A(p, torch.from_numpy(X).cuda())).cpu().numpy()
    err = np.max(np.abs(Z - X)) / np.max(np.abs(X))
    tol = 20 * U * math.log2(prob.N) * normA * normZ
    announce("aniso box identity", "zeroed", int((~keep).sum()), "err", err, "tol", tol)
    assert err < tol
    p.destroy()
