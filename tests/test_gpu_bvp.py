"""Boundary value problems solved end to end on the GPU (section 6): the
Helmholtz ODE of the section 6.1 example and the 2D Helmholtz problem on the
unit disk of section 6.3, plus manufactured solutions with a nonzero source
term.  Parity with the oracle on the residual and the maximum error of u
(both within 10x), and the accuracy the paper states (1D: max error below
1e-8, Fig. 6.1).  The right-hand sides are assembled by the library from the
raw data f and g (azrbf_rhs) and must equal the oracle's."""
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle import dense, evaluate, lstsq

from gpu_util import announce, require_gpu

pytestmark = pytest.mark.gpu


def _mods():
    require_gpu()
    from paper_2308_14490_amd import azrbf, problems
    return azrbf, problems


def _run(prob, m2d=120):
    azrbf, problems = _mods()
    p = problems.plan_for(prob)
    B = problems.rhs_for(p, prob)
    A, idx, pts, bpts = dense.system_matrix(prob)
    Bo = dense.rhs(prob, pts, bpts)
    assert p.M == idx.size and p.Mb == bpts.shape[0]
    assert np.max(np.abs(B.cpu().numpy().T - Bo)) <= 1e-15 * np.abs(Bo).max()
    X, rel = azrbf.solve(p, B)
    torch.cuda.synchronize()
    Xg = X.cpu().numpy().T
    Xo, _ = lstsq.tsvd_solve(A, Bo, 1e-12)
    tp = W.test_points(prob, m2d=m2d)
    u = np.stack([g(*tp.T) for g in prob.exact], axis=1)
    eg = np.max(np.abs(evaluate.eval_dense(prob, Xg, tp) - u), axis=0)
    eo = np.max(np.abs(evaluate.eval_dense(prob, Xo, tp) - u), axis=0)
    rg, ro = evaluate.relres(A, Xg, Bo), evaluate.relres(A, Xo, Bo)
    info = p.info()
    announce(prob.name, prob.n, "M", p.M, "Mb", p.Mb, "k", info["k"], "rank", info["rank"],
             "relres", rg, ro, "maxerr", eg, eo)
    assert np.allclose(rel.cpu().numpy(), rg, rtol=1e-3, atol=1e-16)
    assert np.all(rg <= 10 * ro + 1e-15)
    assert np.all(eg <= 10 * eo + 1e-15)
    p.destroy()
    return eg


def _ode(n, f=None, u=None):
    """u'' + k^2 u = 0 on [-1, 1], k = n/5, u(+-1) = sin(+-n/5), T = 1.5,
    s = 2, tau0 = 1e-10 (section 6.1 example; Fig. 6.1)."""
    kk = n / 5.0
    u = u or (lambda x: np.sin(kk * x))
    f = f or (lambda x: 0.0 * x)
    return W.Problem(f"ode{n}", 1, n, 2, 1.5, W.shape_parameter_eh(1e-10), W.interval(-1.0, 1.0), [f],
                     op=W.HELMHOLTZ, k2=kk * kk, bnd=[u], nb=2, exact=[u])


@pytest.mark.parametrize("n", [64, 128, 256])
def test_helmholtz_ode_paper_example(n):
    eg = _run(_ode(n))
    assert np.all(eg < 1e-8)


def test_helmholtz_ode_nonzero_source():
    """u = sin(kx) + x^2 with f = -(u'' + k^2 u) = -(2 + k^2 x^2)."""
    n = 128
    kk = n / 5.0
    eg = _run(_ode(n, f=lambda x: -(2.0 + kk * kk * x * x), u=lambda x: np.sin(kk * x) + x * x))
    assert np.all(eg < 1e-8)


def _disk_helmholtz(n, k2=13.0, f=None, u=None, dom=None, nb=100, T=1.5, tau0=1e-5):
    """Lap u + k0^2 u = 0 on the unit disk with u = sin(2x + 3y), k0^2 = 13,
    T = 1.5, s = 2, tau0 = 1e-5 and 100 equispaced boundary points (section
    6.3, Fig. 6.2)."""
    u = u or (lambda x, y: np.sin(2 * x + 3 * y))
    f = f or (lambda x, y: 0.0 * x)
    return W.Problem(f"helm2d{n}", 2, n, 2, T, W.shape_parameter_eh(tau0), dom or W.disk(1.0), [f],
                     op=W.HELMHOLTZ, k2=k2, bnd=[u], nb=nb, exact=[u])


@pytest.mark.parametrize("n", [32, 64])
def test_helmholtz_2d_unit_disk_paper_example(n):
    _run(_disk_helmholtz(n))


def test_helmholtz_2d_star_nonzero_source():
    """u = sin 2x cos 3y on the star 0.7 + 0.1 cos 5t, k2 = 5, f = 8 u, weak
    Dirichlet rows at the round(4 length / h) boundary points."""
    base = W.config_c4(32)

    def u(x, y):
        return np.sin(2 * x) * np.cos(3 * y)
    prob = W.Problem("star-helm", 2, 32, 2, 1.0, 0.5, base.domain, [lambda x, y: 8.0 * u(x, y)],
                     op=W.HELMHOLTZ, k2=5.0, bnd=[u], nb=base.nb, exact=[u])
    eg = _run(prob)
    assert np.all(eg < 1e-4)


# ---------------------------------------------------------------- Neumann rows (section 6.3)

@pytest.mark.parametrize("n", [32, 64])
def test_mixed_neumann_dirichlet_flower(n):
    """Section 6.3's last setting with manufactured data: the multiply
    connected flower, Helmholtz k^2 = 4, Neumann rows on the outer curve
    (200 points) and Dirichlet rows on the circle cut out (100 points).
    Right-hand sides, residual and error as the oracle's."""
    eg = _run(W.config_flower(n, manufactured=True))
    if n == 64:
        assert np.all(eg < 1e-5)


def test_helmholtz_ode_neumann_left_end():
    """u = sin(kx) + x^2 with u'(-1) imposed by a Neumann row (outward normal
    -1) and u(1) by a Dirichlet row."""
    n = 128
    kk = n / 5.0
    prob = _ode(n, f=lambda x: -(2.0 + kk * kk * x * x), u=lambda x: np.sin(kk * x) + x * x)
    prob.bc_outer = "ND"
    prob.bnd_n = [lambda x, nx: (kk * np.cos(kk * x) + 2 * x) * nx]
    eg = _run(prob)
    assert np.all(eg < 1e-8)


def test_neumann_rows_match_the_oracle_element_by_element():
    """apply_A's boundary rows at Neumann and Dirichlet points against the
    oracle's dense rows (flower, n = 32, eight vectors)."""
    azrbf, problems = _mods()
    prob = W.config_flower(32, manufactured=True)
    p = problems.plan_for(prob)
    A, idx, pts, bpts = dense.system_matrix(prob)
    Xc = np.random.default_rng(11).standard_normal((8, prob.N))
    Y = azrbf.apply_A(p, torch.from_numpy(Xc).cuda())
    torch.cuda.synchronize()
    got = Y.cpu().numpy().T
    want = A @ Xc.T
    M = idx.size
    scale = np.abs(want).max()
    announce("flower rows", "interior", np.abs(got[:M] - want[:M]).max(), "boundary",
             np.abs(got[M:] - want[M:]).max(), "scale", scale)
    assert np.abs(got[M:] - want[M:]).max() <= 1e-13 * scale
    assert np.abs(got[:M] - want[:M]).max() <= 1e-12 * scale
    p.destroy()
