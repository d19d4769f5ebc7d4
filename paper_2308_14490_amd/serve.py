"""Continuous-batching server for AZ least-squares solves on one GPU.

A request carries a problem (domain, grid, operator) and one or more
right-hand sides.  The factor of step 1 of the AZ algorithm (Algorithm 1,
section 3.2.3) depends on the operator only, so the server keeps factored
plans resident in HBM, keyed by the operator: spectra, index list, the sketch
Omega, the explicit Q of the sketch and the truncated pseudo-inverse of R.
Later requests with the same operator only run the solve.

Scheduling is continuous: the run loop never waits for the GPU as a whole.
  * Arrived requests queue in arrival order.  Each pass of the loop admits,
    in that order, the requests whose operator is not already on the GPU and
    whose memory fits the budget: the resident plans, the reservations of the
    groups in flight and the new group's needs (a new plan's whole footprint,
    or a resident plan's workspace growth for the group's right-hand sides).
    Idle resident plans are evicted, least recently used first, to make room.
    A request whose operator is busy waits for that group; requests of other
    operators behind it go ahead.
  * The admitted requests are grouped by operator; a group's right-hand sides
    are concatenated and solved in one call (they share every launch).  Each
    group is handed to the backend at once and runs on its own stream, beside
    the groups already in flight (a 1D solve does not wait for a 2D
    factorisation that started before it).
  * Groups of one admission pass whose plans are resident small 1D plans
    (single-kernel transform, no boundary rows) go to the GPU together in one
    grouped solve (azrbf_solve_batched): seven launches per refinement pass
    for all of them instead of about twenty per group.
  * Completion is polled through per-group events; a finished group's
    results are recorded and its plan becomes idle and resident.

Every solve of a request, alone or in a group, runs the same kernels on the
same plan arithmetic; only the sketch seed of a shared plan (the first
request's) and the pairing of right-hand sides in the FFTs differ, so results
agree within rounding and the residual test.

The scheduling logic talks to a backend (``GpuBackend`` here; tests also use
a host-only fake with a simulated clock), so it can be checked without a GPU.
"""
import collections
import concurrent.futures
import dataclasses
import hashlib
import threading
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
                   float(prob.bweight), int(prob.k or k), tau, tauZ, refine,
                   getattr(prob, "ny", None), getattr(prob, "Ty", None))).encode())
    h.update(np.ascontiguousarray(mask, dtype=np.uint8).tobytes())
    if prob.nb:
        h.update(np.ascontiguousarray(prob.bpoints(), dtype=np.float64).tobytes())
        if prob.has_neumann:
            h.update(prob.btypes().tobytes())
            h.update(np.ascontiguousarray(prob.bnormals(), dtype=np.float64).tobytes())
    return h.hexdigest()


class _GpuGroup:
    """A group in flight: the worker's future, then the completion event."""

    def __init__(self, future, keep_x):
        self.future = future
        self.keep_x = keep_x

    def done(self):
        if not self.future.done():
            return False
        if self.future.exception() is not None:
            return True
        return self.future.result()[4].query()

    def result(self):
        """(plan, [(X or None, relres)] per request) once done()."""
        plan, X, rel, sizes, ev = self.future.result()
        ev.synchronize()
        rr = rel.cpu().numpy()
        parts, o = [], 0
        for n in sizes:
            parts.append((X[o:o + n] if self.keep_x else None, rr[o:o + n]))
            o += n
        return plan, parts


class _Member:
    """One group of a grouped solve: shares the grouped call's handle."""

    def __init__(self, shared, i):
        self.shared, self.i = shared, i

    def done(self):
        return self.shared.done()

    def result(self):
        return self.shared.result()[self.i]


class _GpuBatch:
    """Several groups solved in one grouped call: the worker's future, then
    the completion event."""

    def __init__(self, future, keep_x):
        self.future = future
        self.keep_x = keep_x
        self._res = None

    def done(self):
        if not self.future.done():
            return False
        if self.future.exception() is not None:
            return True
        return self.future.result()[1].query()

    def result(self):
        if self._res is None:
            items, ev = self.future.result()
            ev.synchronize()
            self._res = []
            for plan, X, rel, sizes in items:
                rr = rel.cpu().numpy()
                parts, o = [], 0
                for n in sizes:
                    parts.append((X[o:o + n] if self.keep_x else None, rr[o:o + n]))
                    o += n
                self._res.append((plan, parts))
        return self._res


class GpuBackend:
    """Plans, right-hand sides and solves on the current HIP device.  Each
    group is queued by a worker thread on that thread's own stream (default
    priority), so a group whose factorisation waits on the host inside the
    library does not hold up the others or the run loop."""

    def __init__(self, refine=None, keep_x=False, streams=4):
        import torch
        from . import azrbf, problems
        self.torch, self.azrbf, self.problems = torch, azrbf, problems
        self.refine = refine
        self.keep_x = keep_x
        self.dev = torch.device("cuda", torch.cuda.current_device())
        self._masks = {}
        self._pool = concurrent.futures.ThreadPoolExecutor(max_workers=streams)
        self._local = threading.local()

    def mask(self, prob):
        mk = id(prob)
        if mk not in self._masks:
            self._masks[mk] = self.azrbf.make_mask(prob.dim, prob.n, prob.s, prob.T, prob.domain.contains,
                                                   prob.ny, prob.Ty)
        return self._masks[mk]

    def _refine(self, prob):
        return self.problems.default_refine(prob) if self.refine is None else self.refine

    def key(self, prob):
        return operator_key(prob, self.mask(prob), refine=self._refine(prob))

    def footprint(self, prob, nrhs):
        return self.problems.footprint_for(prob, nrhs, mask=self.mask(prob), refine=self._refine(prob))

    def nbytes(self, plan):
        return plan.info()["device_bytes"]

    def _stream(self):
        st = getattr(self._local, "stream", None)
        if st is None:
            self.torch.cuda.set_device(self.dev)
            st = self._local.stream = self.torch.cuda.Stream(device=self.dev)
        return st

    def _work(self, plan, probs):
        torch = self.torch
        st = self._stream()
        with torch.cuda.stream(st):
            if plan is None:
                plan = self.problems.plan_for(probs[0], refine=self._refine(probs[0]), stream=st)
            Bs = [self.problems.rhs_for(plan, p, device=self.dev) for p in probs]
            B = torch.cat(Bs, 0).contiguous() if len(Bs) > 1 else Bs[0]
            X, rel = self.azrbf.solve(plan, B, stream=st)
            ev = torch.cuda.Event()
            ev.record(st)
        return plan, X, rel, [b.shape[0] for b in Bs], ev

    def launch(self, plan, probs):
        """Queues the solve of the problems' right-hand sides (one operator;
        plan None: make it first).  Returns a handle with done()/result()."""
        return _GpuGroup(self._pool.submit(self._work, plan, probs), self.keep_x)

    def batchable(self, plan):
        """Whether a resident plan's groups share the grouped solve's
        launches (1D on the single-kernel transform, no boundary rows, sketch
        width <= 64)."""
        return (plan.dim == 1 and plan.N <= 8192 and (plan.N & (plan.N - 1)) == 0 and plan.Mb == 0
                and plan.k <= 64)

    def _work_batch(self, items):
        torch = self.torch
        st = self._stream()
        with torch.cuda.stream(st):
            plans, Bs, sizes = [], [], []
            for plan, probs in items:
                bl = [self.problems.rhs_for(plan, p, device=self.dev) for p in probs]
                plans.append(plan)
                Bs.append(torch.cat(bl, 0).contiguous() if len(bl) > 1 else bl[0])
                sizes.append([b.shape[0] for b in bl])
            Xs, rels = self.azrbf.solve_batched(plans, Bs, stream=st)
            ev = torch.cuda.Event()
            ev.record(st)
        return [(pl, X, r, sz) for pl, X, r, sz in zip(plans, Xs, rels, sizes)], ev

    def launch_batch(self, items):
        """Queues one grouped solve of several groups [(resident plan,
        problems)]; returns one handle per group."""
        shared = _GpuBatch(self._pool.submit(self._work_batch, items), self.keep_x)
        return [_Member(shared, i) for i in range(len(items))]

    def destroy(self, plan):
        plan.destroy()

    def now(self):
        return time.perf_counter()

    def wait(self, until):
        """Sleeps until the time `until` (perf_counter) or briefly while groups
        are in flight (the loop polls their events)."""
        d = min(until - time.perf_counter(), 2e-4)
        if d > 0:
            time.sleep(d)

    def close(self):
        self._pool.shutdown(wait=True)


@dataclasses.dataclass
class _Flight:
    key: str
    reqs: list
    handle: object
    t_admit: float
    new: bool
    reserve: int


class Server:
    """Continuous batching with a factor cache and admission by memory."""

    def __init__(self, backend, budget_bytes, max_batch=64):
        self.be = backend
        self.budget = int(budget_bytes)
        self.max_batch = max_batch
        self.cache = collections.OrderedDict()   # key -> (plan, bytes), LRU order; idle or busy
        self.flights = {}                        # key -> _Flight (its plan is busy)
        self.ticks = []                          # per launched group: (t_admit, t_done, n_requests, new plan)
        self.evictions = 0
        self.created = 0
        self.batched_calls = 0                   # grouped solves launched
        self.peak_committed = 0

    def resident_bytes(self):
        return sum(b for _, b in self.cache.values())

    def committed_bytes(self):
        """Resident plans plus the reservations of the groups in flight."""
        return self.resident_bytes() + sum(f.reserve for f in self.flights.values())

    def _fit(self, need, keep):
        """Evict idle plans (LRU first, none in keep) until need more bytes fit
        beside the committed ones."""
        for key in list(self.cache):
            if self.committed_bytes() + need <= self.budget:
                return True
            if key in keep or key in self.flights:
                continue
            plan, _ = self.cache.pop(key)
            self.be.destroy(plan)
            self.evictions += 1
        return self.committed_bytes() + need <= self.budget

    def _admit(self, queue):
        """Requests from the queue, in order, grouped by operator: {key:
        (requests, bytes to reserve)}.  Busy operators are skipped; admission
        stops at the first request that does not fit."""
        groups = {}
        count = 0
        for req in list(queue):
            if count >= self.max_batch:
                break
            key = self.be.key(req.problem)
            if key in self.flights:
                continue
            reqs, reserve = groups.get(key, ([], 0))
            nrhs = sum(len(r.problem.rhs) for r in reqs) + len(req.problem.rhs)
            full = self.be.footprint(req.problem, max(nrhs, 1))
            resident = self.cache[key][1] if key in self.cache else 0
            want = max(full - resident, 0)
            keep = set(groups) | {key}
            admitted = sum(g[1] for g in groups.values())   # reserved by this pass so far
            if not self._fit(admitted + want - reserve, keep):
                if not groups and not self.flights and want > self.budget - self.resident_bytes():
                    if full > self.budget:
                        raise MemoryError(f"request {req.rid} needs {full} bytes, budget {self.budget}")
                break
            groups[key] = (reqs + [req], want)
            queue.remove(req)
            count += 1
        return groups

    def run(self, requests, start=None, progress=None):
        """Serves requests (objects with rid, arrival, problem) in real time.
        Arrival times are seconds from the start of the run.  progress(done,
        total), if given, is called as results come in."""
        be = self.be
        pending = collections.deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        queue = []
        results = {}
        t0 = be.now() if start is None else start
        while pending or queue or self.flights:
            now = be.now() - t0
            while pending and pending[0].arrival <= now:
                queue.append(pending.popleft())
            progressed = False
            for key, fl in list(self.flights.items()):
                if not fl.handle.done():
                    continue
                plan, parts = fl.handle.result()
                t_done = be.now() - t0
                del self.flights[key]
                self.cache[key] = (plan, be.nbytes(plan))
                self.cache.move_to_end(key)
                for r, (X, rel) in zip(fl.reqs, parts):
                    results[r.rid] = Result(r.rid, len(r.problem.rhs), r.arrival, fl.t_admit, t_done,
                                            np.asarray(rel), X, key)
                self.ticks.append((fl.t_admit, t_done, len(fl.reqs), fl.new))
                progressed = True
                if progress:
                    progress(len(results), len(requests))
            if queue:
                t_admit = be.now() - t0
                batch = []        # resident groups that share one grouped solve
                for key, (reqs, reserve) in self._admit(queue).items():
                    new = key not in self.cache
                    if new:
                        self.created += 1
                    else:
                        self.cache.move_to_end(key)
                    plan = None if new else self.cache[key][0]
                    if plan is not None and hasattr(be, "launch_batch") and be.batchable(plan):
                        batch.append((key, reqs, reserve, plan))
                        continue
                    handle = be.launch(plan, [r.problem for r in reqs])
                    self.flights[key] = _Flight(key, reqs, handle, t_admit, new, reserve)
                    progressed = True
                if len(batch) == 1:
                    key, reqs, reserve, plan = batch[0]
                    self.flights[key] = _Flight(key, reqs, be.launch(plan, [r.problem for r in reqs]), t_admit,
                                                False, reserve)
                    progressed = True
                elif batch:
                    handles = be.launch_batch([(plan, [r.problem for r in reqs]) for _, reqs, _, plan in batch])
                    for (key, reqs, reserve, _), h in zip(batch, handles):
                        self.flights[key] = _Flight(key, reqs, h, t_admit, False, reserve)
                    self.batched_calls += 1
                    progressed = True
                self.peak_committed = max(self.peak_committed, self.committed_bytes())
            if progressed:
                continue
            if queue and not self.flights:
                raise MemoryError("queued requests do not fit the budget")
            be.wait(t0 + pending[0].arrival if pending else float("inf"))
        return results

    def close(self):
        for plan, _ in self.cache.values():
            self.be.destroy(plan)
        self.cache.clear()


def run_plain(backend, requests, start=None, progress=None):
    """FIFO, one request at a time, no plan reuse: plan, factor, solve, free."""
    be = backend
    results = {}
    t0 = be.now() if start is None else start
    for r in sorted(requests, key=lambda r: (r.arrival, r.rid)):
        while be.now() < t0 + r.arrival:
            be.wait(t0 + r.arrival)
        ta = be.now() - t0
        h = be.launch(None, [r.problem])
        while not h.done():
            be.wait(float("inf"))
        plan, parts = h.result()
        X, rel = parts[0]
        td = be.now() - t0
        be.destroy(plan)
        results[r.rid] = Result(r.rid, len(r.problem.rhs), r.arrival, ta, td, np.asarray(rel), X)
        if progress:
            progress(len(results), len(requests))
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
