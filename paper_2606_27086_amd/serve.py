"""Continuous-batching solve server over the slot ABI of libsmx.

Requests are superiorized band+box solves: several slices (right-hand sides)
that share one operator A, each slice with its own bands and starting point,
run for K outer iterations.  The server keeps one *group* per operator: the
operator on the device plus one multi-slot problem (capacity B slots, its own
HIP stream).  Scheduling, all on the host:

* admission by HBM footprint: a group is created only if its device bytes
  (the library's allocation plan, ``smx_footprint``) fit in the budget next
  to the groups already resident; idle groups are evicted when another
  operator needs the room;
* a request is admitted into its group when enough slots are free; its slices
  are loaded into free slots with a budget of K iterations
  (``smx_slot_load``), so each slot stops on the device at exactly K;
* continuous batching: every group with running slots replays chunks of
  iterations (HIP graphs) on its own stream, so the work of different groups
  overlaps on the GPU; after each chunk the group's finished requests are
  collected and waiting requests join at the chunk boundary.

A slot's arithmetic does not depend on the other slots of its group, so every
result is the same whether the request ran alone or in the mix.
"""
from __future__ import annotations

import time
from collections import deque
from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np

from . import Operator, Problem, problem_footprint


@dataclass
class OperatorSpec:
    """The shared part of a family of requests: A and the problem parameters."""

    key: str
    m: int
    n: int
    row_ptr: np.ndarray
    col_idx: np.ndarray
    val: np.ndarray
    params: dict  # Problem keyword arguments other than bands (box, obj, gamma, ...)
    slots: Optional[int] = None  # slots of this operator's group (None: the server's default)

    @property
    def nnz(self) -> int:
        return int(self.row_ptr[-1])


@dataclass
class Request:
    rid: int
    op_key: str
    lower: np.ndarray  # [m, S]
    upper: np.ndarray  # [m, S]
    x0: np.ndarray  # [n, S]
    K: int
    t_arrival: float = 0.0  # seconds from the start of the run
    t_admit: Optional[float] = None
    t_done: Optional[float] = None
    slots: List[int] = field(default_factory=list)
    result: Optional[np.ndarray] = None  # [n, S]

    @property
    def S(self) -> int:
        return int(self.lower.shape[1])


class Group:
    def __init__(self, spec: OperatorSpec, B: int, storage: str, device: str):
        import torch

        self.spec = spec
        self.B = B
        self.stream = torch.cuda.Stream(device=device)  # default priority
        with torch.cuda.stream(self.stream):
            self.op = Operator(spec.m, spec.n, spec.row_ptr, spec.col_idx, spec.val, storage=storage,
                               keep_f32=True, device=device, stream=self.stream)
            if B > 1:  # the row-panel pass 2 serves one-slice problems only
                self.op.release_panels()
            zeros_m = np.zeros((spec.m, B), np.float32)
            self.prob = Problem(self.op, lower=zeros_m, upper=zeros_m, B=B, device=device, stream=self.stream,
                                refine_iters=0, **spec.params)
        # the two passes sum in a fixed order: a request's result does not depend
        # on what shares its group (a one-slot group would otherwise take the
        # fused pass, whose LDS atomics sum in a varying order)
        self.prob.set_fused(False)
        for s in range(B):
            self.prob.slot_disable(s)
        self.free = list(range(B))
        self.requests: List[Request] = []
        self.event = None
        self.running = False
        self.last_used = time.perf_counter()
        self.slice_iters = 0

    def close(self):
        self.prob.close()
        self.op.close()


class Server:
    def __init__(self, specs: Dict[str, OperatorSpec], hbm_budget: int, slots: int = 32, chunk: int = 10,
                 storage: str = "bf16", device: str = "cuda", graph: bool = True, autotune: bool = True):
        self.specs = specs
        self.hbm_budget = int(hbm_budget)
        self.slots = slots
        self.chunk = chunk
        self.storage = storage
        self.device = device
        self.graph = graph
        self.autotune = autotune
        self.groups: Dict[str, Group] = {}
        self.done: List[Request] = []
        self.rejected: List[Request] = []
        self._bytes: Dict[str, int] = {}

    def slots_of(self, spec: OperatorSpec) -> int:
        return int(spec.slots or self.slots)

    # -- footprint ---------------------------------------------------------
    def group_bytes(self, spec: OperatorSpec) -> int:
        """Device bytes of a group, from the library's own allocation plan
        (smx_footprint): its operator (an upper bound) and its B-slot problem.
        The autotuner's temporary copies and captured graphs come on top."""
        b = self._bytes.get(spec.key)
        if b is None:
            ob, pb = problem_footprint(spec.m, spec.n, spec.nnz, self.storage, keep_f32=True, B=self.slots_of(spec),
                                       refine_iters=0, **spec.params)
            b = self._bytes[spec.key] = ob + pb
        return b

    def resident_bytes(self) -> int:
        return sum(self.group_bytes(g.spec) for g in self.groups.values())

    def _group_for(self, key: str) -> Optional[Group]:
        g = self.groups.get(key)
        if g is not None:
            return g
        spec = self.specs[key]
        need = self.group_bytes(spec)
        if need > self.hbm_budget:
            return None
        # evict idle groups (least recently used first) until the new one fits
        while self.resident_bytes() + need > self.hbm_budget:
            idle = [x for x in self.groups.values() if not x.requests and not x.running]
            if not idle:
                return None
            victim = min(idle, key=lambda x: x.last_used)
            victim.close()
            del self.groups[victim.spec.key]
        g = Group(spec, self.slots_of(spec), self.storage, self.device)
        if self.autotune:
            g.prob.autotune(reps=5)
        self.groups[key] = g
        return g

    # -- the loop ----------------------------------------------------------
    def run(self, requests: List[Request], realtime: bool = True, timeout: float = 600.0) -> dict:
        """Serve `requests` (arrival times relative to the start); returns stats."""
        import torch

        arrivals = deque(sorted(requests, key=lambda r: r.t_arrival))
        waiting: deque = deque()
        t0 = time.perf_counter()
        now = lambda: time.perf_counter() - t0  # noqa: E731
        while arrivals or waiting or any(g.requests for g in self.groups.values()):
            if now() > timeout:
                raise TimeoutError("serving did not finish in time")
            t = now()
            while arrivals and (arrivals[0].t_arrival <= t or not realtime):
                waiting.append(arrivals.popleft())
            # admission (FIFO, a request that cannot start yet does not block others)
            still = deque()
            while waiting:
                r = waiting.popleft()
                spec = self.specs[r.op_key]
                if r.S > self.slots_of(spec) or self.group_bytes(spec) > self.hbm_budget:
                    self.rejected.append(r)
                    continue
                g = self._group_for(r.op_key)
                if g is None or g.running or len(g.free) < r.S:
                    still.append(r)
                    continue
                r.slots = [g.free.pop(0) for _ in range(r.S)]
                for j, s in enumerate(r.slots):
                    g.prob.slot_load(s, r.lower[:, j], r.upper[:, j], r.x0[:, j], r.K)
                r.t_admit = now()
                g.requests.append(r)
            waiting = still
            # launch a chunk on every idle group with running slots
            for g in self.groups.values():
                if g.requests and not g.running:
                    with torch.cuda.stream(g.stream):
                        g.prob.run(self.chunk, perturb=True, graph=self.graph)
                        g.event = torch.cuda.Event()
                        g.event.record(g.stream)
                    g.running = True
                    g.last_used = time.perf_counter()
            # collect finished chunks
            progressed = False
            for g in self.groups.values():
                if g.running and g.event.query():
                    g.running = False
                    progressed = True
                    k, live = g.prob.slot_status()
                    for r in list(g.requests):
                        if all(k[s] >= r.K and not live[s] for s in r.slots):
                            r.result = np.stack([g.prob.slot_x_host(s) for s in r.slots], axis=1)
                            r.t_done = now()
                            g.slice_iters += r.K * r.S
                            for s in r.slots:
                                g.prob.slot_disable(s)
                                g.free.append(s)
                            g.requests.remove(r)
                            self.done.append(r)
            if not progressed:
                if arrivals and not waiting and not any(g.running for g in self.groups.values()):
                    time.sleep(max(0.0, min(arrivals[0].t_arrival - now(), 0.01)))
                else:
                    time.sleep(20e-6)
        elapsed = now()
        lat = np.array([r.t_done - r.t_arrival for r in self.done]) if self.done else np.zeros(0)
        slice_iters = sum(r.K * r.S for r in self.done)
        return {
            "requests": len(self.done),
            "rejected": len(self.rejected),
            "elapsed_s": elapsed,
            "slice_iterations": int(slice_iters),
            "slice_it_s": slice_iters / elapsed if elapsed > 0 else 0.0,
            "p50_ms": float(np.percentile(lat, 50) * 1e3) if lat.size else None,
            "p99_ms": float(np.percentile(lat, 99) * 1e3) if lat.size else None,
            "max_ms": float(lat.max() * 1e3) if lat.size else None,
        }

    def close(self):
        for g in self.groups.values():
            g.close()
        self.groups.clear()
