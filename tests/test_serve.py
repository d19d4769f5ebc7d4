"""Host-side tests of the continuous-batching scheduler (no GPU): a fake
backend with a simulated clock records what the server asks for."""
import collections
import dataclasses

import numpy as np
import pytest

from paper_2308_14490_amd import serve


@dataclasses.dataclass
class FakeProblem:
    op_id: str
    nbytes: int
    rhs: list


@dataclasses.dataclass
class FakeRequest:
    rid: int
    arrival: float
    problem: FakeProblem


class FakePlan:
    def __init__(self, key, nbytes):
        self.key, self.nbytes, self.alive = key, nbytes, True


class FakeBackend:
    """Factor costs 1.0 s, a solve group 0.1 s, all groups of a tick overlap."""

    def __init__(self):
        self.t = 0.0
        self.created, self.destroyed, self.ticks = [], [], []
        self.live = {}

    def key(self, prob):
        return prob.op_id

    def footprint(self, prob, nrhs):
        return prob.nbytes

    def create(self, prob):
        self.t += 1.0
        p = FakePlan(prob.op_id, prob.nbytes)
        self.created.append(prob.op_id)
        self.live[id(p)] = p
        return p

    def nbytes(self, plan):
        return plan.nbytes

    def rhs(self, plan, prob):
        assert plan.alive and plan.key == prob.op_id
        return np.asarray(prob.rhs, dtype=float)

    def solve_groups(self, groups):
        self.t += 0.1
        self.ticks.append([(g[0].key, sum(len(b) for b in g[1])) for g in groups])
        assert sum(p.nbytes for p in self.live.values()) <= self._budget
        return [[(None, np.full(len(b), 1e-15)) for b in blist] for plan, blist in groups]

    def destroy(self, plan):
        plan.alive = False
        self.destroyed.append(plan.key)
        del self.live[id(plan)]

    def now(self):
        return self.t

    def sleep_until(self, t):
        self.t = max(self.t, t)


def _server(budget):
    be = FakeBackend()
    be._budget = budget
    return be, serve.Server(be, budget)


def test_groups_requests_by_operator_and_reuses_factors():
    be, srv = _server(100)
    reqs = [FakeRequest(i, 0.0, FakeProblem("A" if i % 2 else "B", 10, [1.0] * (i + 1))) for i in range(6)]
    res = srv.run(reqs)
    assert sorted(res) == list(range(6))
    assert be.created == ["B", "A"]                    # one factor per operator
    assert be.ticks == [[("B", 1 + 3 + 5), ("A", 2 + 4 + 6)]]
    assert all(r.nrhs == i + 1 for i, r in sorted(res.items()))
    assert all(len(r.relres) == r.nrhs for r in res.values())


def test_requests_arriving_during_a_tick_wait_for_the_next():
    be, srv = _server(100)
    reqs = [FakeRequest(0, 0.0, FakeProblem("A", 10, [1.0])),
            FakeRequest(1, 0.5, FakeProblem("A", 10, [1.0])),      # arrives during the first factor
            FakeRequest(2, 5.0, FakeProblem("A", 10, [1.0]))]
    res = srv.run(reqs)
    assert [len(t) for t in be.ticks] == [1, 1, 1]
    assert res[1].admitted >= res[0].done                   # joined the second tick
    assert res[2].admitted >= 5.0
    assert be.created == ["A"]                               # the factor stayed resident
    assert res[2].done - res[2].arrival == pytest.approx(0.1)


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
    assert [len(t) for t in be.ticks] == [2, 1]             # C did not fit beside A and B
    assert res[2].admitted >= res[0].done


def test_request_larger_than_budget_is_rejected():
    be, srv = _server(5)
    with pytest.raises(MemoryError):
        srv.run([FakeRequest(0, 0.0, FakeProblem("A", 10, [1.0]))])


def test_plain_mode_factors_every_request():
    be = FakeBackend()
    be._budget = 1e9
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
