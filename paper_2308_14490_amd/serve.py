"""Continuous-batching server for AZ least-squares solves on one GPU.

A request carries a problem (domain, grid, operator) and one or more
right-hand sides.  The factor of step 1 of the AZ algorithm (Algorithm 1,
section 3.2.3) depends on the operator only, so the server keeps factored
plans resident in HBM, keyed by the operator: spectra, index list, the sketch
Omega, the explicit Q of the sketch and the truncated pseudo-inverse of R.
Later requests with the same operator only run the solve.

Scheduling is iteration-level ("ticks"):
  * a tick admits, in arrival order, requests that have arrived, while the
    bytes of the plans they need (resident ones plus new ones, with their solve
    workspace) fit the memory budget; resident plans that the tick does not
    use are evicted, least recently used first, to make room;
  * the admitted requests are grouped by operator: the right-hand sides of a
    group are concatenated and solved in one call, so they share every
    launch; different groups run concurrently (``azrbf_solve_many`` spreads
    them over the library's internal streams);
  * requests that arrive while a tick is on the GPU wait for the next tick.

Every solve of a request, alone or in a tick, runs the same kernels on the
same plan arithmetic; only the sketch seed of a shared plan (the first
request's) and the pairing of right-hand sides in the FFTs differ, so results
agree within rounding and the residual test.

The scheduling logic talks to a backend (``GpuBackend`` here; tests also use
a host-only fake), so it can be checked without a GPU.
"""
import collections
import dataclasses
import hashlib
import time

import numpy as np


@dataclasses.dataclass
class Result:
    rid: int
    nrhs: int
    arrival: float
    admitted: float
    done: float
    relres: np.ndarray
    X: object = None          # (nrhs, N) coefficients (backend tensor) if kept
    key: str = ""

    @property
    def latency(self):
        return self.done - self.arrival


def operator_key(prob, mask, k=0, tau=1e-12, tauZ=1e-12, refine=1):
    """Identity of the operator: everything the factor depends on except the
    sketch seed (any Gaussian sketch of the same width serves)."""
    h = hashlib.sha1()
    h.update(repr((prob.dim, prob.n, prob.s, float(prob.T), float(prob.eps), int(prob.op), float(prob.k2),
                   float(prob.bweight), int(prob.k or k), tau, tauZ, refine)).encode())
    h.update(np.ascontiguousarray(mask, dtype=np.uint8).tobytes())
    if prob.nb:
        h.update(np.ascontiguousarray(prob.bpoints(), dtype=np.float64).tobytes())
    return h.hexdigest()


class GpuBackend:
    """Plans, right-hand sides and batched solves on the current HIP device."""

    def __init__(self, refine=1, keep_x=False):
        import torch
        from . import azrbf, problems
        self.torch, self.azrbf, self.problems = torch, azrbf, problems
        self.refine = refine
        self.keep_x = keep_x
        self.dev = torch.device("cuda", torch.cuda.current_device())
        self._masks = {}

    def mask(self, prob):
        mk = id(prob)
        if mk not in self._masks:
            self._masks[mk] = self.azrbf.make_mask(prob.dim, prob.n, prob.s, prob.T, prob.domain.contains)
        return self._masks[mk]

    def key(self, prob):
        return operator_key(prob, self.mask(prob), refine=self.refine)

    def footprint(self, prob, nrhs):
        return self.problems.footprint_for(prob, nrhs, mask=self.mask(prob))

    def create(self, prob):
        return self.problems.plan_for(prob, refine=self.refine)

    def nbytes(self, plan):
        return plan.info()["device_bytes"]

    def rhs(self, plan, prob):
        return self.problems.rhs_for(plan, prob, device=self.dev)

    def solve_groups(self, groups):
        """groups: list of (plan, [B tensors]).  Returns per group the list of
        (X, relres) slices in the same order, after the device finished."""
        torch = self.torch
        plans, Bs, sizes = [], [], []
        for plan, blist in groups:
            plans.append(plan)
            Bs.append(torch.cat(blist, 0).contiguous() if len(blist) > 1 else blist[0])
            sizes.append([b.shape[0] for b in blist])
        Xs, rels = self.azrbf.solve_many(plans, Bs)
        torch.cuda.synchronize()
        out = []
        for X, r, sz in zip(Xs, rels, sizes):
            rr = r.cpu().numpy()
            parts, o = [], 0
            for n in sz:
                parts.append((X[o:o + n] if self.keep_x else None, rr[o:o + n]))
                o += n
            out.append(parts)
        return out

    def destroy(self, plan):
        plan.destroy()

    def now(self):
        return time.perf_counter()

    def sleep_until(self, t):
        d = t - time.perf_counter()
        if d > 0:
            time.sleep(d)


class Server:
    """Continuous batching with a factor cache and admission by memory."""

    def __init__(self, backend, budget_bytes, max_batch=64):
        self.be = backend
        self.budget = int(budget_bytes)
        self.max_batch = max_batch
        self.cache = collections.OrderedDict()   # key -> (plan, bytes), LRU order
        self.ticks = []                          # (t_start, t_end, n_requests, n_groups, n_new_plans)
        self.evictions = 0
        self.created = 0

    def resident_bytes(self):
        return sum(b for _, b in self.cache.values())

    def _evict(self, need, keep):
        """Evict unused plans (LRU first) until need bytes fit; False if not possible."""
        for key in list(self.cache):
            if self.resident_bytes() + need <= self.budget:
                return True
            if key in keep:
                continue
            plan, _ = self.cache.pop(key)
            self.be.destroy(plan)
            self.evictions += 1
        return self.resident_bytes() + need <= self.budget

    def _admit(self, queue):
        """Takes requests from the head of the queue while their plans fit."""
        batch, groups, new_bytes = [], {}, 0
        while queue and len(batch) < self.max_batch:
            req = queue[0]
            key = self.be.key(req.problem)
            nrhs = len(req.problem.rhs)
            extra = 0 if (key in self.cache or key in groups) else self.be.footprint(req.problem, max(nrhs, 1))
            keep = set(groups) | {key}
            if not self._evict(new_bytes + extra, keep):
                if batch:
                    break                      # waits for the next tick
                if extra > self.budget:
                    raise MemoryError(f"request {req.rid} needs {extra} bytes, budget {self.budget}")
            batch.append(req)
            groups.setdefault(key, []).append(req)
            new_bytes += extra
            queue.popleft()
        return batch, groups

    def run(self, requests, start=None):
        """Serves requests (objects with rid, arrival, problem) in real time.
        Arrival times are seconds from the start of the run."""
        be = self.be
        pending = collections.deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        queue = collections.deque()
        results = {}
        t0 = be.now() if start is None else start
        while pending or queue:
            now = be.now() - t0
            while pending and pending[0].arrival <= now:
                queue.append(pending.popleft())
            if not queue:
                be.sleep_until(t0 + pending[0].arrival)
                continue
            t_admit = be.now() - t0
            batch, groups = self._admit(queue)
            new = 0
            order = []
            for key, reqs in groups.items():
                if key not in self.cache:
                    plan = be.create(reqs[0].problem)
                    self.cache[key] = (plan, 0)
                    self.created += 1
                    new += 1
                self.cache.move_to_end(key)
                order.append((key, reqs))
            work = []
            for key, reqs in order:
                plan = self.cache[key][0]
                work.append((plan, [be.rhs(plan, r.problem) for r in reqs]))
            outs = be.solve_groups(work)
            t_done = be.now() - t0
            for (key, reqs), parts in zip(order, outs):
                plan = self.cache[key][0]
                self.cache[key] = (plan, be.nbytes(plan))
                for r, (X, rel) in zip(reqs, parts):
                    results[r.rid] = Result(r.rid, len(r.problem.rhs), r.arrival, t_admit, t_done,
                                            np.asarray(rel), X, key)
            self.ticks.append((t_admit, t_done, len(batch), len(order), new))
        return results

    def close(self):
        for plan, _ in self.cache.values():
            self.be.destroy(plan)
        self.cache.clear()


def run_plain(backend, requests, start=None):
    """FIFO, one request at a time, no plan reuse: plan, factor, solve, free."""
    be = backend
    results = {}
    t0 = be.now() if start is None else start
    for r in sorted(requests, key=lambda r: (r.arrival, r.rid)):
        be.sleep_until(t0 + r.arrival)
        ta = be.now() - t0
        plan = be.create(r.problem)
        out = be.solve_groups([(plan, [be.rhs(plan, r.problem)])])
        X, rel = out[0][0]
        td = be.now() - t0
        be.destroy(plan)
        results[r.rid] = Result(r.rid, len(r.problem.rhs), r.arrival, ta, td, np.asarray(rel), X)
    return results


def summarize(results, good=1e-10):
    """Latency percentiles and good-solve throughput of a run."""
    res = list(results.values())
    if not res:
        return {}
    lat = np.array([r.latency for r in res])
    span = max(r.done for r in res) - min(r.arrival for r in res)
    solved = sum(int(np.sum(r.relres <= good)) for r in res)
    total = sum(r.nrhs for r in res)
    return {"requests": len(res), "rhs": total, "rhs_good": solved,
            "makespan_s": span, "solves_per_s": solved / span if span > 0 else float("inf"),
            "p50_ms": float(np.percentile(lat, 50) * 1e3), "p99_ms": float(np.percentile(lat, 99) * 1e3),
            "max_relres": float(max(float(np.max(r.relres)) for r in res))}
