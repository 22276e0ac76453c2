"""Serving loop: continuous batching of force evaluations on one GPU.

Requests (a particle set, an accuracy target and a number of drift steps) are
queued in arrival order and admitted as soon as a slot is free and their
device footprint (fmm_footprint_bytes) fits into the HBM budget next to the
requests already running.  Every slot owns one libfmm context on its own HIP
stream (default priority), so admitted requests run concurrently on the
device.  A request's steps stay on its slot: the first step builds the tree;
every drift step (x += v dt) recycles the tree and uses the previous step's
|a| as the sink scale of the acceptance test (Sec. 5.4.1, tree recycling as
in Sec. 7.1).  Kernels are deterministic and contexts are not shared, so a
request's result does not depend on what else runs beside it.
"""
from __future__ import annotations

import collections
import dataclasses
import threading
import time

import torch

from . import fmm


class Admission:
    """FIFO admission by slots and bytes (no GPU needed).

    Each slot's library context keeps its buffers at the largest size it has
    needed, so the budget counts what every slot holds, idle or not: held[s]
    is the largest footprint slot s has run.  The head request starts on the
    free slot that grows least, once the held bytes after it fit the budget.
    If they fit only without some idle slots' buffers, those slots are listed
    to be emptied first (the caller recreates their contexts).  A request
    larger than the whole budget is refused."""

    def __init__(self, slots: int, budget_bytes: int):
        if slots < 1 or budget_bytes <= 0:
            raise ValueError("need at least one slot and a positive budget")
        self.slots = slots
        self.budget = int(budget_bytes)
        self.held = [0] * slots
        self.free = list(range(slots))
        self.queue: collections.deque = collections.deque()

    @property
    def running(self) -> int:
        return self.slots - len(self.free)

    @property
    def used(self) -> int:
        return sum(self.held)

    def push(self, item, nbytes: int) -> bool:
        if nbytes > self.budget:
            return False
        self.queue.append((item, int(nbytes)))
        return True

    def pop_admissible(self):
        """(item, nbytes, slot, slots to empty first) for the head of the
        queue if it can start now, else None."""
        if not self.queue or not self.free:
            return None
        item, nbytes = self.queue[0]
        # the free slot that needs the least growth; ties to the lower slot
        slot = min(self.free, key=lambda s: (max(0, nbytes - self.held[s]), s))
        need = self.used - self.held[slot] + max(self.held[slot], nbytes)
        empty = []
        for s in sorted((s for s in self.free if s != slot and self.held[s] > 0),
                        key=lambda s: (-self.held[s], s)):
            if need <= self.budget:
                break
            need -= self.held[s]
            empty.append(s)
        if need > self.budget:
            return None
        self.queue.popleft()
        for s in empty:
            self.held[s] = 0
        self.held[slot] = max(self.held[slot], nbytes)
        self.free.remove(slot)
        return item, nbytes, slot, empty

    def release(self, slot: int):
        self.free.append(slot)


@dataclasses.dataclass
class Request:
    pos: torch.Tensor                  # (n, 3) float64 on the device
    mass: torch.Tensor                 # (n,)
    target_err: float = 1e-7
    p: int = -1
    G: float = 1.0
    steps: int = 1                     # force evaluations; steps > 1 drift in between
    vel: torch.Tensor | None = None    # (n, 3) for drift steps
    dt: float = 1e-3
    keep_all: bool = False
    # filled in by the server
    t_submit: float = 0.0
    t_start: float = 0.0
    t_end: float = 0.0
    pot: torch.Tensor | None = None
    acc: torch.Tensor | None = None
    history: list = dataclasses.field(default_factory=list)
    error: Exception | None = None
    done: threading.Event = dataclasses.field(default_factory=threading.Event)
    slot: int = -1

    @property
    def latency(self) -> float:
        return self.t_end - self.t_submit

    def result(self, timeout: float | None = None):
        if not self.done.wait(timeout):
            raise TimeoutError("request not finished")
        if self.error is not None:
            raise self.error
        return self.pot, self.acc


class Server:
    def __init__(self, device: int = 0, slots: int = 4, budget_bytes: int | None = None,
                 leaf_size: int = 0, p2p_factor: float = 0.0, precision: str = "fp64",
                 centre: str = "auto"):
        self.device = device
        if budget_bytes is None:
            free, total = torch.cuda.mem_get_info(device)
            budget_bytes = int(0.6 * free)
        self.adm = Admission(slots, budget_bytes)
        self.cv = threading.Condition()
        self.closed = False
        self.completed: list[Request] = []
        self.max_running = 0
        self._ctx_args = dict(device=device, leaf_size=leaf_size, p2p_factor=p2p_factor,
                              centre=centre, scale_source="previous", timing=True,
                              precision=precision)
        self.streams = []
        self.contexts = []
        with torch.cuda.device(device):
            for s in range(slots):
                self.streams.append(torch.cuda.Stream(device=device))   # default priority
                self.contexts.append(self._context(s))
        self._threads = [threading.Thread(target=self._loop, daemon=True)
                         for _ in range(slots)]
        for t in self._threads:
            t.start()

    def _context(self, slot: int):
        return fmm.Context(stream=self.streams[slot], **self._ctx_args)

    # ------------------------------------------------------------- client
    def submit(self, req: Request) -> Request:
        n = req.pos.shape[0]
        p = req.p if req.p > 0 else max(1, fmm.order_for_error(req.target_err))
        nbytes = fmm.footprint_bytes(n, p)
        req.t_submit = time.perf_counter()
        with self.cv:
            if self.closed:
                raise RuntimeError("server closed")
            if not self.adm.push(req, nbytes):
                req.error = MemoryError(f"request needs {nbytes} B, budget {self.adm.budget} B")
                req.t_end = req.t_submit
                req.done.set()
                return req
            self.cv.notify_all()
        return req

    def close(self):
        with self.cv:
            self.closed = True
            self.cv.notify_all()
        for t in self._threads:
            t.join()
        for c in self.contexts:
            c.close()

    # ------------------------------------------------------------- workers
    def _loop(self):
        while True:
            with self.cv:
                while True:
                    got = self.adm.pop_admissible()
                    if got is not None:
                        break
                    if self.closed and not self.adm.queue:
                        return
                    self.cv.wait()
                req, nbytes, slot, empty = got
                for s in empty:     # idle slots whose buffers must go for this one
                    self.contexts[s].close()
                    self.contexts[s] = self._context(s)
                self.max_running = max(self.max_running, self.adm.running)
            try:
                self._run(slot, req)
            except Exception as e:      # reported to the caller of result()
                req.error = e
            finally:
                req.t_end = time.perf_counter()
                with self.cv:
                    self.adm.release(slot)
                    self.completed.append(req)
                    self.cv.notify_all()
                req.done.set()

    def _run(self, slot: int, req: Request):
        ctx, stream = self.contexts[slot], self.streams[slot]
        req.slot = slot
        req.t_start = time.perf_counter()
        n = req.pos.shape[0]
        with torch.cuda.device(self.device), torch.cuda.stream(stream):
            stream.wait_stream(torch.cuda.default_stream(self.device))
            pos = req.pos.clone()
            pot = torch.empty(n, dtype=torch.float64, device=pos.device)
            acc = torch.empty((n, 3), dtype=torch.float64, device=pos.device)
            for step in range(req.steps):
                if step > 0:
                    if req.vel is None:
                        raise ValueError("drift steps need velocities")
                    pos.add_(req.vel, alpha=req.dt)
                ctx.forces(pos, req.mass, req.G, req.p, req.target_err, pot, acc,
                           refit=step > 0)
                if req.keep_all:
                    req.history.append((pot.clone(), acc.clone(), ctx.stats()))
            req.pot, req.acc = pot, acc
            stream.synchronize()


def latency_summary(reqs) -> dict:
    import numpy as np
    lat = np.sort(np.array([r.latency for r in reqs if r.error is None]))
    if lat.size == 0:
        return {"n": 0}

    def pct(q):
        k = int(np.ceil(q / 100.0 * lat.size)) - 1
        return float(lat[min(max(k, 0), lat.size - 1)])

    return {"n": int(lat.size), "p50_ms": 1e3 * pct(50), "p99_ms": 1e3 * pct(99),
            "max_ms": 1e3 * float(lat[-1]), "mean_ms": 1e3 * float(lat.mean())}
