"""GPU parity of the structured operators A and Z* and of the sketch generator
against the CPU oracle (dense matrices built entry by entry).

Tolerances follow from FFT rounding: a radix-2^q transform of length N has
relative error about u log2 N (u = 2^-53), so A X agrees to 20 u log2 N of its
size; Z* divides by the symbol, which amplifies that by at most
||A^c|| ||Z*||, so Z* R agrees to 20 u log2 N ||A^c|| ||Z*||.
"""
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle import dense, grids, periodic, philox

from gpu_util import announce, engine_path, oracle_norms, rel_err, require_gpu, to_dev

pytestmark = pytest.mark.gpu
U = 2.0 ** -53


def _az():
    require_gpu()
    from paper_2308_14490_amd import azrbf, problems
    return azrbf, problems


def _grid(prob):
    """Rounding of the grid itself.  With s n a power of two (per axis) every
    fine-grid point and centre is a binary fraction and x_i - c_j is exact on
    both sides.  Otherwise (s = 3, or n = 100) the points -T + i 2T/(s n) are
    rounded: the oracle's x_i - c_j carries an error up to about 2uT, and the
    library samples the kernel at (i - s j) h_L with h_L rounded, so entries
    of the two matrices differ by up to |phi'| 4uT <= 0.86 eps 4uT.  Relative
    to the largest product entry (order one) this adds 8 eps T u."""
    axes = prob.axes()
    if all(((prob.s * n) & (prob.s * n - 1)) == 0 for n, _ in axes):
        return 0.0
    return 8.0 * prob.eps * max(T for _, T in axes) * U


def _tol_A(N, prob=None):
    return 20 * U * math.log2(N) + 1e-16 + (_grid(prob) if prob is not None else 0.0)


def _tol_Z(N, plan, prob):
    normA, normZ = oracle_norms(prob)
    return (20 * U * math.log2(N) + _grid(prob)) * normA * normZ


def _case(prob, nvec, ld_pad, engine, seed=0):
    azrbf, problems = _az()
    announce(prob.name, prob.dim, prob.n, prob.s, "nvec", nvec, "pad", ld_pad, "engine", engine)
    if engine:
        with engine_path():
            p = problems.plan_for(prob)
    else:
        p = problems.plan_for(prob)
    A, idx, pts, bpts = dense.system_matrix(prob)
    assert p.M == idx.size and p.Mb == bpts.shape[0]
    assert np.array_equal(p.points(), pts)
    rng = np.random.default_rng(seed)
    X = rng.standard_normal((nvec, prob.N))
    Xd = to_dev(np.pad(X, ((0, 0), (0, ld_pad))))[:, :prob.N]
    Y = azrbf.apply_A(p, Xd)
    want = X @ A.T
    assert rel_err(Y, want) < _tol_A(prob.N, prob), rel_err(Y, want)
    # alpha/beta form
    Y0 = rng.standard_normal((nvec, p.Mt))
    Yd = to_dev(Y0)
    azrbf.apply_A(p, Xd, Yd, alpha=-0.5, beta=2.0)
    assert rel_err(Yd, 2.0 * Y0 - 0.5 * want) < 4 * _tol_A(prob.N, prob)
    # Z*
    Zo = periodic.zstar_normal(prob, idx, 1e-12, nb=bpts.shape[0])
    R = rng.standard_normal((nvec, p.Mt))
    Z = azrbf.apply_Zstar(p, to_dev(R))
    wz = R @ Zo.T
    assert rel_err(Z, wz) < _tol_Z(prob.N, p, prob), (rel_err(Z, wz), _tol_Z(prob.N, p, prob))
    Z0 = rng.standard_normal((nvec, prob.N))
    Zd = to_dev(Z0)
    azrbf.apply_Zstar(p, to_dev(R), Zd, alpha=1.0, beta=1.0)
    assert rel_err(Zd, Z0 + wz) < 2 * _tol_Z(prob.N, p, prob)
    # A Z* (one spectral pass between the operators) and the residual form r - A Z* r
    waz = wz @ A.T
    Rd = to_dev(R)
    AZ = azrbf.apply_AZstar(p, Rd)
    assert rel_err(AZ, waz) < _tol_Z(prob.N, p, prob), (rel_err(AZ, waz), _tol_Z(prob.N, p, prob))
    azrbf.apply_AZstar(p, Rd, Rd, alpha=-1.0, beta=1.0)            # in place
    # (r - A Z* r can be far smaller than r, e.g. without oversampling: error relative to r)
    err = np.max(np.abs(Rd.cpu().numpy() - (R - waz))) / np.max(np.abs(R))
    assert err < 2 * _tol_Z(prob.N, p, prob), err
    p.destroy()


@pytest.mark.parametrize("n,s,nvec", [(16, 2, 1), (64, 1, 3), (256, 2, 4), (256, 3, 3), (256, 4, 2), (1024, 2, 5),
                                      (4096, 2, 2), (4096, 3, 2)])
def test_apply_1d_fused(n, s, nvec):
    prob = W.config_c1a(n)
    prob.s = s
    prob.name = f"1d-fused-s{s}"
    _case(prob, nvec, ld_pad=3 if nvec > 1 else 0, engine=False)


def test_apply_1d_saturated_shape_parameter():
    _case(W.config_c1(256), 3, 0, engine=False)


@pytest.mark.parametrize("n,s,nvec", [(256, 2, 3), (1024, 2, 2), (2048, 1, 1), (2048, 3, 3), (4096, 4, 3)])
def test_apply_1d_four_step(n, s, nvec):
    prob = W.config_c1a(n)
    prob.s = s
    prob.name = f"1d-4step-s{s}"
    _case(prob, nvec, ld_pad=1, engine=True)


@pytest.mark.parametrize("n,nvec", [(16, 1), (32, 3), (64, 2)])
def test_apply_2d_disk(n, nvec):
    _case(W.config_c3a(n), nvec, ld_pad=2, engine=False)


@pytest.mark.parametrize("n,nvec", [(16, 2), (32, 3)])
def test_apply_2d_poisson_star(n, nvec):
    _case(W.config_c4(n), nvec, ld_pad=0, engine=False)


@pytest.mark.parametrize("n,s,nvec", [(16, 3, 2), (32, 3, 3), (16, 4, 1)])
def test_apply_2d_disk_other_oversampling(n, s, nvec):
    """2D with s = 3 (nine phases, three per line in the row passes) and s = 4."""
    prob = W.config_c3a(n)
    prob.s = s
    prob.name = f"disk-s{s}"
    _case(prob, nvec, ld_pad=1, engine=False)


@pytest.mark.parametrize("n,nvec", [(16, 2), (32, 3)])
def test_apply_2d_flower_mixed_boundary(n, nvec):
    """The multiply connected flower of section 6.3: Neumann rows on the
    outer curve, Dirichlet rows on the hole, Helmholtz k^2 = 4."""
    _case(W.config_flower(n, manufactured=True), nvec, ld_pad=1, engine=False)


def test_apply_1d_neumann_rows():
    prob = W.Problem("ode-nd", 1, 256, 2, 1.5, W.shape_parameter_eh(1e-10), W.interval(-1.0, 1.0),
                     [lambda x: 0 * x], op=W.HELMHOLTZ, k2=(256 / 5.0) ** 2, bnd=[lambda x: 0 * x],
                     bnd_n=[lambda x, nx: 0 * x], nb=2, bc_outer="ND")
    _case(prob, 2, ld_pad=0, engine=False)


def test_apply_2d_poisson_star_s3():
    prob = W.config_c4(16)
    prob.s = 3
    prob.name = "star-s3"
    _case(prob, 2, ld_pad=0, engine=False)


def test_apply_1d_bvp_with_boundary_rows():
    n = 128
    prob = W.Problem("ode", 1, n, 2, 1.5, 0.5, W.interval(-1.0, 1.0), [lambda x: 0 * x],
                     op=W.HELMHOLTZ, k2=(n / 5.0) ** 2, bnd=[lambda x: np.sin(n * x / 5)], nb=2)
    _case(prob, 3, 0, engine=False)


def test_gaussian_sketch_matches_oracle():
    azrbf, _ = _az()
    for rows, cols, seed in [(10, 3, 42), (1027, 5, (5 << 32) | 77)]:
        announce("gaussian", rows, cols, seed)
        got = azrbf.gaussian(seed, rows, cols).cpu().numpy().T
        want = philox.gaussian_sketch(rows, cols, seed)
        assert np.max(np.abs(got - want)) < 1e-14 * np.max(np.abs(want))


def test_empty_and_zero_vector_calls():
    azrbf, problems = _az()
    p = problems.plan_for(W.config_c1a(64))
    import torch
    X = torch.zeros((0, p.N), dtype=torch.float64, device="cuda")
    Y = azrbf.apply_A(p, X)
    assert Y.shape == (0, p.Mt)
    Z = azrbf.apply_Zstar(p, torch.zeros((2, p.Mt), dtype=torch.float64, device="cuda"))
    assert float(Z.abs().max()) == 0.0
    p.destroy()


def test_autotune_keeps_results_bitwise():
    """Tile shapes regroup independent line transforms: A X is the same bit for bit."""
    require_gpu()
    from paper_2308_14490_amd import azrbf, problems
    prob = W.family_1d(16384, 2)
    announce("autotune", prob.n)
    p = problems.plan_for(prob)
    X = azrbf.gaussian(3, p.N, 24)
    Y0 = azrbf.apply_A(p, X)
    Z0 = azrbf.apply_Zstar(p, Y0)
    rep = azrbf.autotune(p, 24)
    assert rep["engine"] and rep["ms"] > 0 and len(rep["trials"]) >= 4
    Y1 = azrbf.apply_A(p, X)
    Z1 = azrbf.apply_Zstar(p, Y1)
    torch.cuda.synchronize()
    assert torch.equal(Y0, Y1) and torch.equal(Z0, Z1)
    assert rep["key"] in azrbf.tune_table()
    p.destroy()


@pytest.mark.parametrize("nx,ny,nvec", [(32, 16, 3), (16, 32, 2), (64, 32, 2)])
def test_apply_2d_anisotropic_ellipse(nx, ny, nvec):
    """Section 5.1's anisotropic box: the ellipse x^2 + 4 y^2 <= 1 in
    [-1.4, 1.4] x [-0.7, 0.7] with nx x ny centres (equal spacing when
    ny = nx / 2, else different spacing per axis)."""
    _case(W.config_ellipse(nx, ny), nvec, ld_pad=1, engine=False)


def test_apply_2d_anisotropic_poisson():
    """-Lap on the same ellipse with weak Dirichlet rows at 120 points."""
    base = W.config_ellipse(32, 16)

    def u(x, y):
        return np.sin(2 * x) * np.cos(3 * y)
    prob = W.Problem("ellipse-poisson", 2, 32, 2, 1.4, base.eh, base.domain, [lambda x, y: 13 * u(x, y)],
                     op=W.POISSON, bnd=[u], nb=120, exact=[u], ny=16, Ty=0.7)
    _case(prob, 2, ld_pad=0, engine=False)
