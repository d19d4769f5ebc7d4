"""Plans and right-hand sides for workload descriptions (``workloads.Problem``).

The collocation mask comes from the plan's own fine grid (eq. set_Xtilde)
and the domain's membership test; right-hand sides are the workload's
functions sampled at the plan's collocation points (and, for boundary value
problems, the boundary data: values at Dirichlet points, normal derivatives
at Neumann points), assembled into the
system's right-hand side by the library.
"""
import numpy as np
import torch

from . import azrbf


def default_refine(prob):
    """Refinement passes: one, or two for 2D boundary value problems (on the
    256 x 256 Poisson star the second pass takes the residual from 1.7e-12
    to 9.7e-13)."""
    return 2 if prob.op != 0 and prob.dim == 2 else 1


def plan_for(prob, refine=None, tau=1e-12, tauZ=1e-12, k=None, stream=None):
    refine = default_refine(prob) if refine is None else refine
    mask = azrbf.make_mask(prob.dim, prob.n, prob.s, prob.T, prob.domain.contains, prob.ny, prob.Ty)
    bpts = prob.bpoints() if prob.nb else None
    neu = prob.has_neumann
    return azrbf.Plan(prob.dim, prob.n, prob.s, prob.T, mask, eps=prob.eps,
                      op=azrbf.OP_APPROX if prob.op == 0 else azrbf.OP_BVP, k2=prob.k2,
                      bpts=bpts, bweight=prob.bweight, tau=tau, tauZ=tauZ,
                      k=prob.k if k is None else k, refine=refine, seed=prob.seed, stream=stream,
                      ny=prob.ny or 0, Ty=prob.Ty or 0.0,
                      btype=prob.btypes() if neu else None, bnormal=prob.bnormals() if neu else None)


def footprint_for(prob, max_rhs, mask=None, refine=None, tau=1e-12, tauZ=1e-12):
    """Device bytes a plan for ``prob`` needs with ``max_rhs`` right-hand sides
    per solve (azrbf_footprint_bytes)."""
    import ctypes
    if mask is None:
        mask = azrbf.make_mask(prob.dim, prob.n, prob.s, prob.T, prob.domain.contains, prob.ny, prob.Ty)
    m = np.ascontiguousarray(mask, dtype=np.uint8).ravel()
    bp = np.ascontiguousarray(prob.bpoints(), dtype=np.float64).reshape(-1) if prob.nb else None
    pr = azrbf._Problem()
    pr.dim, pr.n, pr.s, pr.T = prob.dim, prob.n, prob.s, float(prob.T)
    pr.eps, pr.tau0, pr.op, pr.k2 = float(prob.eps), 0.0, 0 if prob.op == 0 else 1, float(prob.k2)
    pr.mask = m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    pr.nb = prob.nb
    pr.bpts = bp.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if prob.nb else None
    pr.bweight, pr.tau, pr.tauZ = float(prob.bweight), float(tau), float(tauZ)
    refine = default_refine(prob) if refine is None else refine
    pr.k, pr.refine, pr.seed = int(prob.k), int(refine), int(prob.seed)
    pr.ny, pr.Ty = int(prob.ny or 0), float(prob.Ty or 0.0)
    return azrbf.footprint_bytes(pr, max_rhs)


def rhs_for(plan, prob, which=None, device=None):
    """Right-hand sides as a (nrhs, M + Mb) float64 tensor on ``device``: the
    workload's functions sampled at the plan's collocation points (and its
    boundary data: values at Dirichlet points, normal derivatives at Neumann
    points), assembled by the library
    (azrbf_rhs), which applies the boundary value problems' row
    normalisation."""
    pts = plan.points()
    idx = list(range(len(prob.rhs))) if which is None else list(which)
    dev = device or torch.device("cuda", torch.cuda.current_device())
    F = np.stack([prob.rhs[i](*pts.T) for i in idx], axis=0)
    Fd = torch.from_numpy(np.ascontiguousarray(F)).to(dev)
    Gd = None
    if plan.Mb:
        bp = prob.bpoints()
        G = np.stack([prob.bdata(i, bp) for i in idx], axis=0)
        Gd = torch.from_numpy(np.ascontiguousarray(G)).to(dev)
    return azrbf.rhs(plan, Fd, Gd)
