"""Scheduling policy of the CG-SENSE server, on a virtual clock (no GPU)."""
import numpy as np
import pytest

from paper_2111_02912_amd.serve import (FakeExecutor, Problem, Request, Server, latency_stats,
                                        poisson_arrivals)


def _probs():
    return [Problem(0, (64, 64), 8, 1000, "2d"), Problem(1, (96, 96, 96), 8, 100000, "3d"),
            Problem(2, (48, 48), 4, 800, "2d")]


def _cost(p):
    return {0: 0.001, 1: 0.02, 2: 0.0008}[p.pid]


def test_every_request_completes_with_all_iterations():
    probs = _probs()
    arr = poisson_arrivals(60, 50.0, seed=11)
    reqs = [Request(i, float(t), probs[i % 3], iters=10) for i, t in enumerate(arr)]
    ex = FakeExecutor(_cost)
    done = Server(ex, hbm_budget=1 << 40, lanes=3, chunk=2).run(reqs)
    assert len(done) == 60
    for r in done:
        assert r.completed == r.iters == r.issued == 10
        assert r.t_admit >= r.arrival - 1e-12 and r.t_done > r.t_admit
    st = latency_stats(done)
    assert st["n"] == 60 and st["p99_ms"] >= st["p50_ms"] > 0


def test_admission_is_fifo_and_respects_the_budget():
    probs = _probs()
    need = {0: 100, 1: 1000, 2: 80}
    ex = FakeExecutor(_cost, need=lambda p: need[p.pid])
    reqs = [Request(i, 0.001 * i, probs[i % 3], iters=5) for i in range(30)]
    budget = 2000 + 3 * 1024
    srv = Server(ex, hbm_budget=budget, lanes=2, chunk=1)
    done = srv.run(reqs)
    assert len(done) == 30
    assert srv.admit_order == list(range(30))  # arrival order, no overtaking
    assert srv.peak_bytes <= budget


def test_idle_plans_are_evicted_least_recently_used_first():
    probs = [Problem(i, (32, 32), 2, 500, "2d") for i in range(4)]
    ex = FakeExecutor(lambda p: 0.001, need=lambda p: 1000)
    # one request at a time; the budget holds two plans plus one solver state
    reqs = [Request(i, 1.0 * i, probs[i % 4], iters=2) for i in range(8)]
    srv = Server(ex, hbm_budget=2000 + 1024, lanes=1)
    srv.run(reqs)
    assert srv.peak_bytes <= 2000 + 1024
    assert ex.plans_created == 8  # round-robin over 4 problems with room for 2: never a hit


def test_resident_plan_is_reused():
    p = Problem(0, (64, 64), 8, 1000, "2d")
    ex = FakeExecutor(lambda q: 0.001, need=lambda q: 1000)
    reqs = [Request(i, 0.1 * i, p, iters=3) for i in range(5)]
    Server(ex, hbm_budget=1 << 30).run(reqs)
    assert ex.plans_created == 1 and ex.plan_hits == 4


def test_short_request_is_not_blocked_by_a_long_one():
    """Iteration-level interleaving on one lane: a short solve admitted
    while a long one runs finishes first."""
    long_p = Problem(0, (96, 96, 96), 8, 100000, "3d")
    short_p = Problem(1, (48, 48), 4, 800, "2d")
    ex = FakeExecutor(lambda p: 1.0 if p.pid == 0 else 0.01)
    reqs = [Request(0, 0.0, long_p, iters=10), Request(1, 0.5, short_p, iters=10)]
    done = {r.rid: r for r in Server(ex, hbm_budget=1 << 40, lanes=1, chunk=1, depth=1).run(reqs)}
    assert done[1].t_done < done[0].t_done
    assert done[1].latency < 3.0  # at most a couple of long iterations of waiting


def test_request_that_can_never_fit_fails_alone():
    p = Problem(0, (64, 64), 8, 1000, "2d")
    big = Problem(1, (96, 96, 96), 8, 10 ** 6, "3d")
    ex = FakeExecutor(lambda q: 0.001, need=lambda q: 10 ** 6 if q.pid == 1 else 100)
    reqs = [Request(0, 0.0, p, iters=3), Request(1, 0.001, big, iters=3), Request(2, 0.002, p, iters=3)]
    srv = Server(ex, hbm_budget=100000)
    done = {r.rid: r for r in srv.run(reqs)}
    assert set(done) == {0, 1, 2}
    assert done[1].error and "budget" in done[1].error and done[1].completed == 0
    assert done[0].error is None and done[2].error is None
    assert done[0].completed == done[2].completed == 3
    assert [r.rid for r in srv.failed] == [1]
    assert latency_stats(list(done.values()))["n"] == 2


@pytest.mark.parametrize("kind", ["poison", "poison_step"])
def test_poison_request_fails_alone(kind):
    """A request whose plan cannot be made (or whose CG step fails after
    one chunk) is retired with an error and releases what it held; every
    other request completes all its iterations and the held bytes return
    to the idle plans."""
    good = [Problem(i, (32, 32), 2, 500, "2d") for i in range(3)]
    bad = Problem(9, (32, 32), 2, 500, "2d", data={kind: True})
    ex = FakeExecutor(lambda q: 0.001, need=lambda q: 1000)
    arr = poisson_arrivals(40, 200.0, seed=5)
    reqs = [Request(i, float(t), bad if i % 7 == 3 else good[i % 3], iters=4) for i, t in enumerate(arr)]
    srv = Server(ex, hbm_budget=1 << 20, lanes=2, chunk=1, depth=2)
    done = {r.rid: r for r in srv.run(reqs)}
    assert len(done) == 40
    for r in reqs:
        d = done[r.rid]
        if r.problem is bad:
            assert d.error is not None
        else:
            assert d.error is None and d.completed == d.iters == 4
    assert len(srv.failed) == sum(1 for r in reqs if r.problem is bad)
    # only idle plans of the good problems are held at the end
    assert ex.held == sum(len(v) for v in ex.idle.values()) * 1000


def test_poisson_arrivals():
    a = poisson_arrivals(20000, 50.0, seed=3)
    gaps = np.diff(np.concatenate([[0.0], a]))
    assert np.all(gaps > 0)
    assert abs(gaps.mean() - 0.02) < 0.02 * 0.03
    assert np.array_equal(a, poisson_arrivals(20000, 50.0, seed=3))


def test_zero_iteration_request():
    p = Problem(0, (16, 16), 1, 100, "2d")
    ex = FakeExecutor(lambda q: 0.001)
    done = Server(ex, hbm_budget=1 << 30).run([Request(0, 0.0, p, iters=0)])
    assert done[0].completed == 0 and done[0].t_done is not None
