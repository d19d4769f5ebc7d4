"""GPU tests of the grouped solve (azrbf_solve_batched): many 1D problems of
uneven sizes, oversampling factors, shape parameters, intervals, sketch
widths and refinement counts in one call, with repeated plans, a ragged
number of right-hand sides (past one 16-column block) and entries that take
the per-plan path (a four-step transform, a 2D disk).

Coefficients of a frame are not unique, and the grouped dense products sum in
another order than the per-plan solve, so grouped entries are compared on the
residual ||A x - b|| / ||b|| (the library's, recomputed on the CPU with the
oracle's dense A, and the oracle's truncated-SVD residual) and on the fitted
values on the fine test set; entries on the per-plan path must equal
azrbf_solve bit for bit."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import dense, evaluate, lstsq

from gpu_util import announce, require_gpu

pytestmark = pytest.mark.gpu

# (n, s, eps*h, interval, k, refine, right-hand sides); every sketch width is
# at least 1.45 times the numerical rank of A - A Z* A (20 to 42 here)
_SPECS = [
    (256, 2, 0.5, (-0.5, 0.5), 32, 1, 3),
    (1024, 2, 0.5, (-0.5, 0.5), 32, 1, 17),
    (2048, 3, 0.5, (-0.6, 0.4), 64, 1, 5),
    (512, 4, 0.5, (-0.45, 0.55), 32, 0, 2),
    (8192, 2, 0.5, (-0.5, 0.5), 32, 1, 20),
    (4096, 3, 0.5, (-0.3, 0.7), 32, 2, 1),
    (128, 2, 0.4, (-0.5, 0.5), 64, 1, 4),
]


def _mods():
    require_gpu()
    from paper_2308_14490_amd import azrbf, problems
    return azrbf, problems


def _problem(i, spec, seed0):
    n, s, eh, (lo, hi), k, refine, nrhs = spec
    prob = W.Problem(f"b{i}-n{n}", 1, n, s, 1.0, eh, W.interval(lo, hi),
                     [W.trig_sum_1d(seed0 + j) for j in range(nrhs)], k=k)
    return prob, refine


def _cpu_relres(prob, X, B):
    """||A x - b|| / ||b|| per column with the oracle's dense A (X: nrhs x N),
    and the floor under which the library's and this residual may differ.
    With s a power of two both sides sample the same binary grid; otherwise
    the fine-grid points carry a rounding of about eps T u that the two sides
    make differently, so the matrices differ by that much per entry (as in the
    one-plan solve tests)."""
    A, idx, pts, bpts = dense.system_matrix(prob)
    Xn = X.cpu().numpy().T
    Bn = B.cpu().numpy().T
    floor = 1e-16 if prob.s & (prob.s - 1) == 0 else 1e-12
    return evaluate.relres(A, Xn, Bn), A, Bn, floor


def _fitted(prob, X):
    tp = W.test_points(prob)
    return evaluate.eval_dense(prob, X.cpu().numpy().T, tp)


def _build(seed0=500):
    azrbf, problems = _mods()
    probs = [_problem(i, sp, seed0 + 100 * i) for i, sp in enumerate(_SPECS)]
    plans_a = [problems.plan_for(p, refine=r) for p, r in probs]
    plans_b = [problems.plan_for(p, refine=r) for p, r in probs]
    Bs = [problems.rhs_for(pl, p) for pl, (p, _) in zip(plans_a, probs)]
    return azrbf, problems, probs, plans_a, plans_b, Bs


def test_grouped_solve_matches_per_plan_solves_and_oracle():
    azrbf, problems, probs, plans_a, plans_b, Bs = _build()
    announce("grouped solve", [p.name for p, _ in probs])
    single = [azrbf.solve(pl, B) for pl, B in zip(plans_a, Bs)]
    # entries: every plan once, plan 1 again with its columns reversed, and an
    # entry with no right-hand sides
    ent_plans = plans_b + [plans_b[1], plans_b[0]]
    ent_B = Bs + [Bs[1].flip(0).contiguous(), Bs[0][:0]]
    Xs, rels = azrbf.solve_batched(ent_plans, ent_B)      # factors inside
    rev = azrbf.solve(plans_a[1], ent_B[len(probs)])
    torch.cuda.synchronize()
    for i, ((p, _), (Xp, rp), Xb, rb) in enumerate(zip(probs, single, Xs, rels)):
        rp, rb = rp.cpu().numpy(), rb.cpu().numpy()
        announce(p.name, "relres per-plan", rp.max(), "grouped", rb.max())
        # same residual level as the per-plan solve, and at most 1e-10
        assert np.all(rb <= 10 * rp + 1e-15) and np.all(rp <= 10 * rb + 1e-15), p.name
        assert np.all(rb <= 1e-10), p.name
        # the library's residual is the residual of the returned coefficients
        rc, A, Bn, floor = _cpu_relres(p, Xb, Bs[i])
        assert np.all(np.abs(rb - rc) <= 1e-3 * rc + floor), (p.name, rb, rc, floor)
        # the fitted values agree to within the residual level
        fb, fp = _fitted(p, Xb), _fitted(p, Xp)
        scale = np.max(np.abs(fp), axis=0)
        assert np.all(np.max(np.abs(fb - fp), axis=0) <= 1e-9 * scale + 1e-12), p.name
        if p.n <= 1024:
            Xo, _ = lstsq.tsvd_solve(A, Bn, 1e-12)
            ro = evaluate.relres(A, Xo, Bn)
            announce(p.name, "oracle relres", ro.max())
            assert np.all(rc <= 10 * ro + 1e-15), p.name
    # the repeated plan's second entry
    rb2 = rels[len(probs)].cpu().numpy()
    rp2 = rev[1].cpu().numpy()
    assert np.all(rb2 <= 10 * rp2 + 1e-15) and np.all(rb2 <= 1e-10)
    fb, fp = _fitted(probs[1][0], Xs[len(probs)]), _fitted(probs[1][0], rev[0])
    assert np.max(np.abs(fb - fp)) <= 1e-9 * np.max(np.abs(fp)) + 1e-12
    assert Xs[-1].shape[0] == 0
    for pl in plans_a + plans_b:
        pl.destroy()


def test_grouped_solve_second_call_reuses_staging():
    """Two more calls on the factored plans, the second with fewer entries
    and fewer right-hand sides: each equals a fresh grouped call's result on
    the same inputs bit for bit (the staging buffers carry nothing over), also
    after the staging buffers have been released."""
    azrbf, problems, probs, plans_a, plans_b, Bs = _build(seed0=900)
    Xs1, r1 = azrbf.solve_batched(plans_b, Bs)
    sub = [0, 2, 4]
    Bsub = [Bs[i][: max(1, Bs[i].shape[0] // 2)].contiguous() for i in sub]
    Xs2, r2 = azrbf.solve_batched([plans_b[i] for i in sub], Bsub)
    Xs3, r3 = azrbf.solve_batched([plans_a[i] for i in sub], Bsub)     # factors plans_a inside
    torch.cuda.synchronize()
    for a, b in zip(Xs2, Xs3):
        assert torch.equal(a, b)
    for a, b in zip(r2, r3):
        assert torch.equal(a, b)
    for r in r1 + r2:
        assert float(r.max()) <= 1e-10
    # the staging buffers freed in between: the next call allocates them again
    azrbf.release_cached_memory()
    Xs4, r4 = azrbf.solve_batched([plans_b[i] for i in sub], Bsub)
    torch.cuda.synchronize()
    for a, b in zip(Xs2, Xs4):
        assert torch.equal(a, b)
    for pl in plans_a + plans_b:
        pl.destroy()


def test_grouped_solve_with_entries_on_the_per_plan_path():
    """A four-step 1D plan (N = 16384) and a 2D disk (n = 16) in the same call
    as grouped entries: they are solved as by azrbf_solve, bit for bit."""
    azrbf, problems = _mods()
    probs = [W.family_1d(16384, 2, seed0=41, name="big"), W.config_c3a(16),
             W.family_1d(1024, 3, seed0=51, name="small")]
    pa = [problems.plan_for(p) for p in probs]
    pb = [problems.plan_for(p) for p in probs]
    Bs = [problems.rhs_for(pl, p) for pl, p in zip(pa, probs)]
    single = [azrbf.solve(pl, B) for pl, B in zip(pa, Bs)]
    Xs, rels = azrbf.solve_batched(pb, Bs)
    torch.cuda.synchronize()
    for i in (0, 1):
        assert torch.equal(single[i][0], Xs[i]), probs[i].name
        assert torch.equal(single[i][1], rels[i]), probs[i].name
    assert float(rels[2].max()) <= 1e-10
    for pl in pa + pb:
        pl.destroy()


def test_grouped_factor_equals_per_plan_factor():
    """Unfactored plans of a grouped call are factored together (one launch
    per step for all of them) with the per-plan kernels in the same order per
    plan: Q, R, the singular values and the retained rank equal those of
    azrbf_factor bit for bit, and so do the solutions on either factor."""
    azrbf, problems, probs, plans_a, plans_b, Bs = _build(seed0=1300)
    for pl in plans_a:
        azrbf.factor(pl)
    azrbf.solve_batched(plans_b, [B[:1].contiguous() for B in Bs])    # factors plans_b in one grouped call
    torch.cuda.synchronize()
    for (p, _), pa, pb, B in zip(probs, plans_a, plans_b, Bs):
        for which in ("Q", "R", "sigma"):
            assert torch.equal(azrbf.get_factor(pa, which), azrbf.get_factor(pb, which)), (p.name, which)
        assert pa.info()["rank"] == pb.info()["rank"], p.name
        Xa, ra = azrbf.solve(pa, B)
        Xb, rb = azrbf.solve(pb, B)
        torch.cuda.synchronize()
        assert torch.equal(Xa, Xb) and torch.equal(ra, rb), p.name
    for pl in plans_a + plans_b:
        pl.destroy()


def test_grouped_call_edge_cases():
    """No qualifying entry (a four-step plan only), only empty entries, and a
    single entry: each as by azrbf_solve."""
    azrbf, problems = _mods()
    big = W.family_1d(16384, 2, seed0=61, name="big-only")
    small = W.family_1d(512, 3, seed0=71, name="small-only")
    pa, pb = problems.plan_for(big), problems.plan_for(big)
    qa, qb = problems.plan_for(small), problems.plan_for(small)
    Bb, Bs = problems.rhs_for(pa, big), problems.rhs_for(qa, small)
    Xa, ra = azrbf.solve(pa, Bb)
    Xb, rb = azrbf.solve_batched([pb], [Bb])
    Ya, sa = azrbf.solve(qa, Bs)
    Yb, sb = azrbf.solve_batched([qb], [Bs])
    Xe, re_ = azrbf.solve_batched([pb, qb], [Bb[:0], Bs[:0]])
    torch.cuda.synchronize()
    assert torch.equal(Xa, Xb[0]) and torch.equal(ra, rb[0])
    # the single small entry goes through the grouped kernels: same residual level
    assert float(sb[0].max()) <= 1e-10 and float(sa.max()) <= 1e-10
    assert torch.all(sb[0].cpu() <= 10 * sa.cpu() + 1e-15)
    assert Xe[0].shape[0] == 0 and Xe[1].shape[0] == 0
    for p in (pa, pb, qa, qb):
        p.destroy()
