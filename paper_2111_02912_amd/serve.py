"""Continuous-batching CG-SENSE server (host-side scheduling policy).

Each request reconstructs one image by CG-SENSE, (E^H E + lambda I) x =
E^H y with a fixed iteration count (Sec. IV-B, T = I), on its own problem
(image shape, trajectory, coil maps, k-space data).  The server:

  * admits requests in arrival order when the bytes they need fit an HBM
    budget (solver state, output image, and the plan unless one is already
    resident for the same problem); idle resident plans are evicted least
    recently used first when memory runs short;
  * keeps plans resident between requests of the same problem, so a
    repeated trajectory skips plan creation and the index pass;
  * interleaves requests at iteration granularity: each lane (a GPU stream)
    issues `chunk` CG iterations at a time, with at most `depth` chunks in
    flight, choosing among its active requests the one with the least
    remaining estimated work (ties: earliest arrival), so a short request
    admitted behind a long solve runs at the next iteration boundary; lanes
    run concurrently on the GPU;
  * retires a request when its last iteration completes (latency = finish
    time - arrival time);
  * fails a request alone when it cannot be served (it can never fit the
    budget, its plan cannot be created, its sample locations are not finite,
    or a library call for it fails): the request is retired with `error` set
    and everything it held is released, while the others go on.

All reconstruction arithmetic is in the HIP library (kbn_cg_*); executors
only place calls and allocate buffers.  ``FakeExecutor`` replaces the GPU by
a virtual clock for tests of the policy.
"""
from __future__ import annotations

import collections
import dataclasses
import math
import time
from typing import Dict, List, Optional

import numpy as np


@dataclasses.dataclass
class Problem:
    pid: int
    N: tuple
    coils: int
    M: int
    kind: str = ""
    data: Optional[dict] = None  # executor inputs: omega, smaps, y (resident device tensors)


@dataclasses.dataclass
class Request:
    rid: int
    arrival: float
    problem: Problem
    iters: int = 10
    t_admit: Optional[float] = None
    t_done: Optional[float] = None
    issued: int = 0
    completed: int = 0
    lane: int = -1
    handle: object = None
    result: object = None
    error: Optional[str] = None

    @property
    def latency(self) -> Optional[float]:
        return None if self.t_done is None else self.t_done - self.arrival


def poisson_arrivals(n: int, rate: float, seed: int, t0: float = 0.0) -> np.ndarray:
    """Arrival times with exponential gaps of mean 1/rate."""
    return t0 + np.cumsum(np.random.default_rng(seed).exponential(1.0 / rate, size=n))


class RequestError(RuntimeError):
    """A request that cannot be served; the server retires it alone."""


def plan_bytes(N, M: int, coils: int) -> int:
    """Device bytes of one CG-SENSE plan: the library's own footprint
    (constants, index-pass buffers for M points, forward and adjoint grid
    workspace for one image of `coils` coils), computed on the host."""
    from .nufft import footprint
    return footprint(N, M, B=1, C=coils)


class FakeExecutor:
    """Virtual-clock stand-in for the GPU: each lane runs its chunks one
    after another, an iteration of a problem costs `iter_cost(problem)`
    seconds and the start (E^H y) half of that."""

    def __init__(self, iter_cost, plan_cost: float = 0.0, need=None):
        self.cost = iter_cost
        self.t = 0.0
        self.plan_cost = plan_cost
        self._need = need or (lambda p: 1 << 20)
        self.lane_free: Dict[int, float] = collections.defaultdict(float)
        self.held = 0
        self.idle: "collections.OrderedDict[int, list]" = collections.OrderedDict()
        self.plans_created = 0
        self.plan_hits = 0
        self.events: List[float] = []

    # executor interface -------------------------------------------------
    def now(self) -> float:
        return self.t

    def iter_cost(self, prob: Problem) -> float:
        return self.cost(prob)

    def plan_size(self, prob: Problem) -> int:
        return self._need(prob)

    def state_size(self, prob: Problem) -> int:
        return 1 << 10

    def has_idle_plan(self, prob: Problem) -> bool:
        return bool(self.idle.get(prob.pid))

    def bytes_held(self) -> int:
        return self.held

    def evict(self, nbytes: int) -> int:
        freed = 0
        for pid in list(self.idle.keys()):
            while self.idle[pid] and freed < nbytes:
                size = self.idle[pid].pop()
                self.held -= size
                freed += size
            if not self.idle[pid]:
                del self.idle[pid]
            if freed >= nbytes:
                break
        return freed

    def admit(self, req: Request, lane: int):
        p = req.problem
        if p.data and p.data.get("poison"):
            raise RequestError(f"problem {p.pid}: plan cannot be created")
        start = max(self.t, self.lane_free[lane])
        if self.has_idle_plan(p):
            size = self.idle[p.pid].pop()
            if not self.idle[p.pid]:
                del self.idle[p.pid]
            self.plan_hits += 1
        else:
            size = self.plan_size(p)
            self.held += size
            start += self.plan_cost
            self.plans_created += 1
        self.held += self.state_size(p)
        self.lane_free[lane] = start + 0.5 * self.iter_cost(p)
        req.handle = {"plan": size}

    def issue(self, req: Request, n: int, lane: int):
        if req.problem.data and req.problem.data.get("poison_step") and req.issued >= 1:
            raise RequestError(f"problem {req.problem.pid}: CG step failed")
        start = max(self.t, self.lane_free[lane])
        end = start + n * self.iter_cost(req.problem)
        self.lane_free[lane] = end
        self.events.append(end)
        return end

    def ready(self, ev) -> bool:
        return self.t >= ev

    def retire(self, req: Request):
        p = req.problem
        self.held -= self.state_size(p)
        self.idle.setdefault(p.pid, []).append(req.handle["plan"])
        self.idle.move_to_end(p.pid)
        req.result = ("done", req.completed)

    def abort(self, req: Request):
        """Release what a failed request holds (its plan is not kept)."""
        if req.handle is not None:
            self.held -= self.state_size(req.problem) + req.handle["plan"]
            req.handle = None

    def wait(self, until: Optional[float]):
        pend = [e for e in self.events if e > self.t]
        nxt = min(pend) if pend else None
        if until is not None and (nxt is None or until < nxt):
            nxt = until
        if nxt is None:
            raise RuntimeError("fake executor would wait forever")
        self.t = max(self.t, nxt)


class GpuExecutor:
    """Runs requests with the HIP library on `lanes` streams of one GPU."""

    def __init__(self, device, lanes: int = 4, lam: float = 1e-3, keep_results: bool = False):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(lanes)]
        self.lam = float(lam)
        self.keep_results = keep_results
        self.idle: "collections.OrderedDict[int, list]" = collections.OrderedDict()
        self.plan_mem: Dict[int, int] = {}
        self.held = 0
        self.plans_created = 0
        self.plan_hits = 0
        self._state_cache: Dict[tuple, int] = {}

    def now(self) -> float:
        return time.perf_counter()

    def iter_cost(self, prob: Problem) -> float:
        """Estimated seconds per CG iteration: the bytes of one forward and
        one adjoint per coil at 3 TB/s plus a fixed launch overhead."""
        D = len(prob.N)
        gsz = math.prod(2 * n for n in prob.N)
        return prob.coils * (2 * (D + 1) * gsz * 8 + 16 * prob.M) / 3e12 + 100e-6

    def plan_size(self, prob: Problem) -> int:
        return plan_bytes(prob.N, prob.M, prob.coils)

    def state_size(self, prob: Problem) -> int:
        npix = math.prod(prob.N)
        return int(256 + 8192 + 4 * 8 * npix + 8 * prob.coils * prob.M + 4096)

    def has_idle_plan(self, prob: Problem) -> bool:
        return bool(self.idle.get(prob.pid))

    def bytes_held(self) -> int:
        return self.held

    def evict(self, nbytes: int) -> int:
        freed = 0
        for pid in list(self.idle.keys()):
            while self.idle[pid] and freed < nbytes:
                plan = self.idle[pid].pop()
                size = self.plan_mem.get(id(plan), 0)
                self._drop_plan(plan)
                freed += size
            if not self.idle[pid]:
                del self.idle[pid]
            if freed >= nbytes:
                break
        return freed

    def admit(self, req: Request, lane: int):
        from ._lib import KbnError
        from .cg import CgSense
        from .nufft import KbNufft
        torch = self.torch
        p = req.problem
        d = p.data
        plan = None
        with torch.cuda.stream(self.streams[lane]):
            try:
                if self.has_idle_plan(p):
                    plan = self.idle[p.pid].pop()
                    if not self.idle[p.pid]:
                        del self.idle[p.pid]
                    self.plan_hits += 1
                else:
                    plan = KbNufft(p.N, device=self.device)
                    self.plan_mem[id(plan)] = self.plan_size(p)
                    self.held += self.plan_mem[id(plan)]
                    self.plans_created += 1
                    plan.set_points(d["omega"])
                    # a new trajectory is checked once (this waits for the
                    # lane's stream); a resident plan was checked when made
                    if plan.check_error() != 0:
                        raise RequestError(f"request {req.rid}: non-finite sample locations")
                solver = CgSense(plan, p.coils).begin(d["y"], d["smaps"])
            except (KbnError, RequestError, RuntimeError, ValueError) as e:
                if plan is not None:
                    self._drop_plan(plan)
                raise RequestError(str(e)) from e
        self.held += self.state_size(p)
        req.handle = (plan, solver)

    def _drop_plan(self, plan):
        size = self.plan_mem.pop(id(plan), 0)
        self.held -= size
        plan.close()

    def abort(self, req: Request):
        """Release what a failed request holds; its plan is closed."""
        if req.handle is not None:
            plan, solver = req.handle
            req.handle = None
            self.held -= self.state_size(req.problem)
            with self.torch.cuda.stream(self.streams[max(req.lane, 0)]):
                self._drop_plan(plan)

    def issue(self, req: Request, n: int, lane: int):
        from ._lib import KbnError
        torch = self.torch
        plan, solver = req.handle
        s = self.streams[lane]
        with torch.cuda.stream(s):
            try:
                solver.step(n, self.lam)
            except KbnError as e:
                raise RequestError(str(e)) from e
            ev = torch.cuda.Event()
            ev.record(s)
        return ev

    def ready(self, ev) -> bool:
        return ev.query()

    def retire(self, req: Request):
        torch = self.torch
        plan, solver = req.handle
        p = req.problem
        with torch.cuda.stream(self.streams[req.lane]):
            rel = solver.scalars()[0, 5:6].clone()
        req.result = {"x": solver.x[0] if self.keep_results else None, "rel": rel}
        req.handle = None
        self.held -= self.state_size(p)
        self.idle.setdefault(p.pid, []).append(plan)
        self.idle.move_to_end(p.pid)

    def wait(self, until: Optional[float]):
        time.sleep(0.0001)

    def close(self):
        for pid in list(self.idle.keys()):
            for plan in self.idle[pid]:
                plan.close()
        self.idle.clear()


class Server:
    def __init__(self, executor, hbm_budget: int, lanes: int = 4, chunk: int = 1, depth: int = 2,
                 max_active: int = 64):
        if lanes < 1 or chunk < 1 or depth < 1 or max_active < 1:
            raise ValueError("lanes, chunk, depth and max_active must be >= 1")
        self.ex = executor
        self.budget = int(hbm_budget)
        self.nlanes = lanes
        self.chunk = chunk
        self.depth = depth
        self.max_active = max_active
        self.peak_bytes = 0
        self.peak_active = 0
        self.admit_order: List[int] = []

    def _need(self, prob: Problem) -> int:
        ex = self.ex
        return ex.state_size(prob) + (0 if ex.has_idle_plan(prob) else ex.plan_size(prob))

    def run(self, requests: List[Request]) -> List[Request]:
        ex = self.ex
        done: List[Request] = []
        self.failed: List[Request] = []
        servable = []
        for r in requests:
            try:
                full = ex.state_size(r.problem) + ex.plan_size(r.problem)
                err = None if full <= self.budget else \
                    f"request {r.rid} needs {full} bytes, more than the budget {self.budget}"
            except (RequestError, RuntimeError, ValueError) as e:  # no plan can be made for it
                err = f"request {r.rid}: {e}"
            if err is not None:
                r.error = err
                r.t_done = r.arrival
                self.failed.append(r)
                done.append(r)
            else:
                servable.append(r)
        pending = collections.deque(sorted(servable, key=lambda r: (r.arrival, r.rid)))
        queue: "collections.deque[Request]" = collections.deque()
        active: List[List[Request]] = [[] for _ in range(self.nlanes)]
        inflight: List[collections.deque] = [collections.deque() for _ in range(self.nlanes)]
        remaining = [0] * self.nlanes  # iterations still to issue per lane (load estimate)
        n_active = 0
        t0 = ex.now()

        def fail(req, err, li=None):
            req.error = str(err)
            req.t_done = ex.now() - t0
            ex.abort(req)
            self.failed.append(req)
            done.append(req)
            if li is not None and req in active[li]:
                active[li].remove(req)
                remaining[li] -= req.iters - req.issued
                return True
            return False

        while pending or queue or n_active:
            t = ex.now() - t0
            progressed = False
            while pending and pending[0].arrival <= t:
                queue.append(pending.popleft())
                progressed = True
            # completions
            for li in range(self.nlanes):
                q = inflight[li]
                while q and ex.ready(q[0][1]):
                    req, _, n = q.popleft()
                    req.completed += n
                    progressed = True
                    if req.completed == req.iters:
                        req.t_done = ex.now() - t0
                        active[li].remove(req)
                        n_active -= 1
                        ex.retire(req)
                        done.append(req)
            # admission, in arrival order
            while queue and n_active < self.max_active:
                req = queue[0]
                need = self._need(req.problem)
                over = ex.bytes_held() + need - self.budget
                if over > 0:
                    ex.evict(over)
                    need = self._need(req.problem)
                    if ex.bytes_held() + need > self.budget:
                        break  # wait for running requests to free memory
                queue.popleft()
                li = min(range(self.nlanes),
                         key=lambda i: (remaining[i] * 1.0, len(active[i]), i))
                req.lane = li
                req.t_admit = ex.now() - t0
                try:
                    ex.admit(req, li)
                except RequestError as e:
                    fail(req, e)
                    progressed = True
                    continue
                if req.iters == 0:
                    req.t_done = ex.now() - t0
                    ex.retire(req)
                    done.append(req)
                else:
                    active[li].append(req)
                    remaining[li] += req.iters
                    n_active += 1
                self.admit_order.append(req.rid)
                self.peak_bytes = max(self.peak_bytes, ex.bytes_held())
                self.peak_active = max(self.peak_active, n_active)
                progressed = True
            # issue: least remaining work first within each lane
            for li in range(self.nlanes):
                act = active[li]
                while len(inflight[li]) < self.depth and act:
                    pick = None
                    best = None
                    for cand in act:
                        if cand.issued < cand.iters:
                            key = ((cand.iters - cand.issued) * ex.iter_cost(cand.problem),
                                   cand.arrival, cand.rid)
                            if best is None or key < best:
                                best, pick = key, cand
                    if pick is None:
                        break
                    n = min(self.chunk, pick.iters - pick.issued)
                    try:
                        ev = ex.issue(pick, n, li)
                    except RequestError as e:
                        # its iterations already in flight are dropped from the lane
                        inflight[li] = collections.deque(x for x in inflight[li] if x[0] is not pick)
                        if fail(pick, e, li):
                            n_active -= 1
                        progressed = True
                        continue
                    pick.issued += n
                    remaining[li] -= n
                    inflight[li].append((pick, ev, n))
                    progressed = True
            if not progressed:
                ex.wait(t0 + pending[0].arrival if pending else None)
        return done


def latency_stats(reqs: List[Request], skip: int = 0) -> dict:
    """Latency percentiles of the served requests (failed ones excluded)."""
    ok = [r for r in sorted(reqs, key=lambda r: r.rid)[skip:] if r.error is None]
    lat = np.array([r.latency for r in ok], dtype=np.float64)
    if lat.size == 0:
        return {"n": 0}
    return {"n": int(lat.size), "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
            "max_ms": float(lat.max() * 1e3)}
