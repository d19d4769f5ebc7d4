"""Host-side tests of the continuous-batching scheduler (no GPU): a fake
backend with a simulated clock records what the server asks for.  Groups in
flight overlap: each finishes at its own time (a new plan's factorisation,
then the solve), like work on separate streams."""
import dataclasses

import numpy as np
import pytest

from paper_2308_14490_amd import serve


@dataclasses.dataclass
class FakeProblem:
    op_id: str
    nbytes: int
    rhs: list
    factor_s: float = 1.0
    rhs_bytes: int = 0          # workspace per right-hand side


@dataclasses.dataclass
class FakeRequest:
    rid: int
    arrival: float
    problem: FakeProblem


class FakePlan:
    def __init__(self, prob):
        self.key, self.nbytes, self.alive, self.prob = prob.op_id, prob.nbytes, True, prob


class FakeHandle:
    def __init__(self, be, plan, probs, finish):
        self.be, self.plan, self.probs, self.finish = be, plan, probs, finish

    def done(self):
        return self.be.t >= self.finish

    def result(self):
        assert self.done()
        self.be.live_handles.remove(self)
        return self.plan, [(None, np.full(len(p.rhs), 1e-15)) for p in self.probs]


class FakeBackend:
    """A new plan costs its problem's factor_s, a solve 0.1 s; the device
    bytes of a plan grow with the largest group it has solved."""

    def __init__(self, budget=1e18):
        self.t = 0.0
        self._budget = budget
        self.created, self.destroyed, self.launches = [], [], []
        self.live, self.live_handles = {}, []
        self.peak_bytes = 0

    def key(self, prob):
        return prob.op_id

    def footprint(self, prob, nrhs):
        return prob.nbytes + prob.rhs_bytes * nrhs

    def nbytes(self, plan):
        return plan.nbytes

    def _account(self):
        b = sum(p.nbytes for p in self.live.values())
        self.peak_bytes = max(self.peak_bytes, b)
        assert b <= self._budget, (b, self._budget)

    def launch(self, plan, probs):
        for p in probs:
            assert p.op_id == probs[0].op_id
        cost = 0.1
        if plan is None:
            plan = FakePlan(probs[0])
            self.created.append(plan.key)
            self.live[id(plan)] = plan
            cost += probs[0].factor_s
        assert plan.alive
        nrhs = sum(len(p.rhs) for p in probs)
        plan.nbytes = max(plan.nbytes, probs[0].nbytes + probs[0].rhs_bytes * nrhs)
        self._account()
        self.launches.append((plan.key, nrhs, self.t))
        h = FakeHandle(self, plan, probs, self.t + cost)
        self.live_handles.append(h)
        return h

    def destroy(self, plan):
        plan.alive = False
        self.destroyed.append(plan.key)
        del self.live[id(plan)]

    def now(self):
        return self.t

    def wait(self, until):
        nxt = min([h.finish for h in self.live_handles] + [until])
        assert nxt < float("inf"), "waiting with nothing to wait for"
        self.t = max(self.t, nxt)


def _server(budget):
    be = FakeBackend(budget)
    return be, serve.Server(be, budget)


def test_groups_requests_by_operator_and_reuses_factors():
    be, srv = _server(100)
    reqs = [FakeRequest(i, 0.0, FakeProblem("A" if i % 2 else "B", 10, [1.0] * (i + 1))) for i in range(6)]
    res = srv.run(reqs)
    assert sorted(res) == list(range(6))
    assert be.created == ["B", "A"]                    # one factor per operator
    assert [(k, n) for k, n, _ in be.launches] == [("B", 1 + 3 + 5), ("A", 2 + 4 + 6)]
    assert all(r.nrhs == i + 1 for i, r in sorted(res.items()))
    assert all(len(r.relres) == r.nrhs for r in res.values())


def test_request_for_a_busy_operator_waits_for_its_group():
    be, srv = _server(100)
    reqs = [FakeRequest(0, 0.0, FakeProblem("A", 10, [1.0])),
            FakeRequest(1, 0.5, FakeProblem("A", 10, [1.0])),      # arrives during the first factor
            FakeRequest(2, 5.0, FakeProblem("A", 10, [1.0]))]
    res = srv.run(reqs)
    assert [n for _, n, _ in be.launches] == [1, 1, 1]
    assert res[1].admitted >= res[0].done                   # the plan was busy until then
    assert res[2].admitted >= 5.0
    assert be.created == ["A"]                               # the factor stayed resident
    assert res[2].done - res[2].arrival == pytest.approx(0.1)


def test_fast_request_overtakes_a_running_factorisation():
    """A cheap operator arriving while an expensive factorisation runs is
    launched at once and finishes first (continuous batching)."""
    be, srv = _server(100)
    reqs = [FakeRequest(0, 0.0, FakeProblem("2D", 10, [1.0], factor_s=2.0)),
            FakeRequest(1, 0.2, FakeProblem("1D", 10, [1.0, 2.0], factor_s=0.05))]
    res = srv.run(reqs)
    assert res[1].admitted == pytest.approx(0.2)
    assert res[1].done < res[0].done
    assert res[1].done == pytest.approx(0.35)
    assert res[0].done == pytest.approx(2.1)


def test_memory_budget_evicts_least_recently_used():
    be, srv = _server(25)
    seq = ["A", "B", "A", "C", "A", "B"]
    reqs = [FakeRequest(i, 10.0 * i, FakeProblem(k, 10, [1.0])) for i, k in enumerate(seq)]
    res = srv.run(reqs)
    assert len(res) == len(seq)
    # A, B resident; C needs room: B (least recently used) goes; A stays
    assert be.created == ["A", "B", "C", "B"]
    assert be.destroyed == ["B", "C"]                       # LRU: B before A, then C before A
    assert srv.resident_bytes() <= 25


def test_admission_stops_at_the_budget_and_resumes():
    be, srv = _server(20)
    reqs = [FakeRequest(i, 0.0, FakeProblem(k, 10, [1.0])) for i, k in enumerate("ABC")]
    res = srv.run(reqs)
    assert len(res) == 3
    assert [t for _, _, t in be.launches] == pytest.approx([0.0, 0.0, 1.1])   # C did not fit beside A and B
    assert res[2].admitted >= res[0].done


def test_same_operator_requests_reserve_their_workspace():
    """Many right-hand sides of one operator in one group: the reservation
    covers the group's concatenated right-hand sides, and a resident plan's
    workspace growth is reserved too, so the device bytes never exceed the
    budget (the fake asserts it at every launch)."""
    be, srv = _server(100)
    reqs = [FakeRequest(i, 0.0, FakeProblem("A", 40, [1.0] * 4, rhs_bytes=2)) for i in range(5)]
    reqs += [FakeRequest(5, 0.0, FakeProblem("B", 30, [1.0], rhs_bytes=2))]
    reqs += [FakeRequest(6 + i, 3.0, FakeProblem("A", 40, [1.0] * 8, rhs_bytes=2)) for i in range(4)]
    res = srv.run(reqs)
    assert len(res) == 10
    assert be.peak_bytes <= 100 and srv.peak_committed <= 100
    # A's first group: 5 x 4 = 20 right-hand sides -> 80 bytes; B (32) does not fit beside it
    assert be.launches[0][:2] == ("A", 20)
    assert ("B", 1) in [(k, n) for k, n, _ in be.launches]
    # the later group of A (32 right-hand sides, 104 bytes) exceeds the budget as one
    # group: it is split across launches that each fit
    assert all(40 + 2 * n <= 100 for k, n, _ in be.launches if k == "A")


def test_request_larger_than_budget_is_rejected():
    be, srv = _server(5)
    with pytest.raises(MemoryError):
        srv.run([FakeRequest(0, 0.0, FakeProblem("A", 10, [1.0]))])


def test_plain_mode_factors_every_request():
    be = FakeBackend()
    reqs = [FakeRequest(i, 0.0, FakeProblem("A", 10, [1.0, 2.0])) for i in range(3)]
    res = serve.run_plain(be, reqs)
    assert be.created == ["A", "A", "A"] and be.destroyed == ["A", "A", "A"]
    assert [r.done for r in sorted(res.values(), key=lambda r: r.rid)] == pytest.approx([1.1, 2.2, 3.3])


def test_summarize():
    res = {i: serve.Result(i, 2, 0.0, 0.0, float(i + 1), np.array([1e-15, 1e-9])) for i in range(100)}
    s = serve.summarize(res)
    assert s["rhs"] == 200 and s["rhs_good"] == 100
    assert s["p50_ms"] == pytest.approx(50.5e3)
    assert s["p99_ms"] == pytest.approx(99.01e3)
    assert s["solves_per_s"] == pytest.approx(1.0)


def test_operator_key_ignores_the_seed_but_not_the_domain():
    import workloads as W
    a = W.family_1d(256, 2)
    b = W.family_1d(256, 2)
    b.seed = a.seed + 1
    m = np.ones(512, np.uint8)
    assert serve.operator_key(a, m) == serve.operator_key(b, m)
    m2 = m.copy()
    m2[0] = 0
    assert serve.operator_key(a, m) != serve.operator_key(a, m2)
    c = W.family_1d(512, 2)
    assert serve.operator_key(a, m) != serve.operator_key(c, m)


class BatchingBackend(FakeBackend):
    """A fake backend with a grouped solve: resident plans whose key starts
    with "s" (small) are batchable; a grouped call costs one solve."""

    def __init__(self, budget=1e18):
        super().__init__(budget)
        self.batches = []

    def batchable(self, plan):
        return plan.key.startswith("s")

    def launch_batch(self, items):
        self.batches.append(sorted(plan.key for plan, _ in items))
        finish = self.t + 0.1
        hs = []
        for plan, probs in items:
            assert plan.alive and self.batchable(plan)
            self.launches.append((plan.key, sum(len(p.rhs) for p in probs), self.t))
            h = FakeHandle(self, plan, probs, finish)
            self.live_handles.append(h)
            hs.append(h)
        return hs


def test_resident_small_groups_of_one_pass_share_a_grouped_solve():
    """First pass: three new operators, each factored on its own.  Second
    pass (all resident): the two small operators' groups go in one grouped
    call, the large one alone; every request gets its results."""
    be = BatchingBackend()
    srv = serve.Server(be, 1e9)
    reqs = [FakeRequest(0, 0.0, FakeProblem("s1", 10, [1.0])),
            FakeRequest(1, 0.0, FakeProblem("s2", 10, [1.0, 2.0])),
            FakeRequest(2, 0.0, FakeProblem("L", 10, [1.0])),
            FakeRequest(3, 5.0, FakeProblem("s1", 10, [1.0, 2.0, 3.0])),
            FakeRequest(4, 5.0, FakeProblem("s2", 10, [1.0])),
            FakeRequest(5, 5.0, FakeProblem("L", 10, [1.0])),
            FakeRequest(6, 5.0, FakeProblem("s2", 10, [1.0]))]
    res = srv.run(reqs)
    assert sorted(res) == list(range(7))
    assert be.created == ["s1", "s2", "L"]
    assert be.batches == [["s1", "s2"]]
    assert srv.batched_calls == 1
    assert all(len(r.relres) == r.nrhs for r in res.values())
    assert res[3].nrhs == 3 and res[4].done == res[3].done
    assert res[6].admitted == res[4].admitted            # same operator, same group
