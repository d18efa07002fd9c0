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
    time - arrival time).

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

    @property
    def latency(self) -> Optional[float]:
        return None if self.t_done is None else self.t_done - self.arrival


def poisson_arrivals(n: int, rate: float, seed: int, t0: float = 0.0) -> np.ndarray:
    """Arrival times with exponential gaps of mean 1/rate."""
    return t0 + np.cumsum(np.random.default_rng(seed).exponential(1.0 / rate, size=n))


def plan_bytes(N, M: int, coils: int) -> int:
    """Upper estimate of one plan's device memory for CG-SENSE with `coils`
    coils: grid workspace of the adjoint (two grids, sorted k-space and the
    partial tiles of the spread per coil), sorted point records and the
    spread owner lists."""
    D = len(N)
    K = [2 * n + 16 for n in N]  # oversampled sizes round up to a 7-smooth length
    gsz = math.prod(K)
    ws = coils * (2 * gsz + M + 256 * 16 ** D) * 8
    # per owner-list entry (at most 2^D per sample): list position, sorted and
    # caller-order sample index, tap origins and fractions
    pts = M * (24 * D + 16 + (2 ** D) * (12 + 8 * D))
    return int(ws + pts + (1 << 20))


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
                size = self.plan_mem.pop(id(plan))
                plan.close()
                self.held -= size
                freed += size
            if not self.idle[pid]:
                del self.idle[pid]
            if freed >= nbytes:
                break
        return freed

    def admit(self, req: Request, lane: int):
        from .cg import CgSense
        from .nufft import KbNufft
        torch = self.torch
        p = req.problem
        d = p.data
        with torch.cuda.stream(self.streams[lane]):
            if self.has_idle_plan(p):
                plan = self.idle[p.pid].pop()
                if not self.idle[p.pid]:
                    del self.idle[p.pid]
                self.plan_hits += 1
            else:
                plan = KbNufft(p.N, device=self.device)
                plan.set_points(d["omega"])
                self.plan_mem[id(plan)] = self.plan_size(p)
                self.held += self.plan_mem[id(plan)]
                self.plans_created += 1
            solver = CgSense(plan, p.coils).begin(d["y"], d["smaps"])
        self.held += self.state_size(p)
        req.handle = (plan, solver)

    def issue(self, req: Request, n: int, lane: int):
        torch = self.torch
        plan, solver = req.handle
        s = self.streams[lane]
        with torch.cuda.stream(s):
            solver.step(n, self.lam)
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
        for r in requests:
            full = ex.state_size(r.problem) + ex.plan_size(r.problem)
            if full > self.budget:
                raise ValueError(f"request {r.rid} needs {full} bytes, more than the budget {self.budget}")
        pending = collections.deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        queue: "collections.deque[Request]" = collections.deque()
        active: List[List[Request]] = [[] for _ in range(self.nlanes)]
        inflight: List[collections.deque] = [collections.deque() for _ in range(self.nlanes)]
        remaining = [0] * self.nlanes  # iterations still to issue per lane (load estimate)
        n_active = 0
        t0 = ex.now()
        done: List[Request] = []
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
                ex.admit(req, li)
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
                    ev = ex.issue(pick, n, li)
                    pick.issued += n
                    remaining[li] -= n
                    inflight[li].append((pick, ev, n))
                    progressed = True
            if not progressed:
                ex.wait(t0 + pending[0].arrival if pending else None)
        return done


def latency_stats(reqs: List[Request], skip: int = 0) -> dict:
    lat = np.array([r.latency for r in sorted(reqs, key=lambda r: r.rid)[skip:]], dtype=np.float64)
    if lat.size == 0:
        return {"n": 0}
    return {"n": int(lat.size), "p50_ms": float(np.percentile(lat, 50) * 1e3),
            "p99_ms": float(np.percentile(lat, 99) * 1e3), "mean_ms": float(lat.mean() * 1e3),
            "max_ms": float(lat.max() * 1e3)}
