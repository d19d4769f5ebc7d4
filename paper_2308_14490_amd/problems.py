"""Plans and right-hand sides for workload descriptions (``workloads.Problem``).

The collocation mask comes from the plan's own fine grid (eq. set_Xtilde)
and the domain's membership test; right-hand sides are the workload's
functions sampled at the plan's collocation points (for boundary value
problems the interior data are divided by 2 eps^2 in 1D and 4 eps^2 in 2D,
matching the operator rows, and boundary rows carry the weighted Dirichlet
data).
"""
import numpy as np
import torch

from . import azrbf


def plan_for(prob, refine=1, tau=1e-12, tauZ=1e-12, k=None, stream=None):
    mask = azrbf.make_mask(prob.dim, prob.n, prob.s, prob.T, prob.domain.contains)
    bpts = prob.bpoints() if prob.nb else None
    return azrbf.Plan(prob.dim, prob.n, prob.s, prob.T, mask, eps=prob.eps,
                      op=azrbf.OP_APPROX if prob.op == 0 else azrbf.OP_BVP, k2=prob.k2,
                      bpts=bpts, bweight=prob.bweight, tau=tau, tauZ=tauZ,
                      k=prob.k if k is None else k, refine=refine, seed=prob.seed, stream=stream)


def footprint_for(prob, max_rhs, mask=None, refine=1, tau=1e-12, tauZ=1e-12):
    """Device bytes a plan for ``prob`` needs with ``max_rhs`` right-hand sides
    per solve (azrbf_footprint_bytes)."""
    import ctypes
    if mask is None:
        mask = azrbf.make_mask(prob.dim, prob.n, prob.s, prob.T, prob.domain.contains)
    m = np.ascontiguousarray(mask, dtype=np.uint8).ravel()
    bp = np.ascontiguousarray(prob.bpoints(), dtype=np.float64).reshape(-1) if prob.nb else None
    pr = azrbf._Problem()
    pr.dim, pr.n, pr.s, pr.T = prob.dim, prob.n, prob.s, float(prob.T)
    pr.eps, pr.tau0, pr.op, pr.k2 = float(prob.eps), 0.0, 0 if prob.op == 0 else 1, float(prob.k2)
    pr.mask = m.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
    pr.nb = prob.nb
    pr.bpts = bp.ctypes.data_as(ctypes.POINTER(ctypes.c_double)) if prob.nb else None
    pr.bweight, pr.tau, pr.tauZ = float(prob.bweight), float(tau), float(tauZ)
    pr.k, pr.refine, pr.seed = int(prob.k), int(refine), int(prob.seed)
    return azrbf.footprint_bytes(pr, max_rhs)


def rhs_for(plan, prob, which=None, device=None):
    """Right-hand sides as a (nrhs, M + Mb) float64 tensor on ``device``."""
    pts = plan.points()
    fs = prob.rhs if which is None else [prob.rhs[i] for i in which]
    idx = range(len(prob.rhs)) if which is None else which
    rows = []
    eps = plan.info()["eps"]
    for i, f in zip(idx, fs):
        v = f(*pts.T)
        if prob.op != 0:
            v = v / ((2.0 if prob.dim == 1 else 4.0) * eps * eps)
            g = prob.bnd[i]
            bp = prob.bpoints()
            v = np.concatenate([v, prob.bweight * g(*bp.T)])
        rows.append(v)
    B = np.stack(rows, axis=0)
    dev = device or torch.device("cuda", torch.cuda.current_device())
    return torch.from_numpy(np.ascontiguousarray(B)).to(dev)
