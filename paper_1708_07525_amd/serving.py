"""Continuous-batching solve loop for many independent porous cavities on one GPU.

Requests (a problem statement, initial fields and a storage precision) arrive over time.
The loop admits a waiting request as soon as its device footprint fits the memory budget
and a slot is free, keeps every admitted cavity resident in HBM, advances all of them
together with one batched launch per precision per time step (replayed from a captured
HIP graph; a cavity with walls through the boundary nodes is stepped by its own launches
beside the batch), checks each cavity's steady-state residual every ``check_every`` steps, and
retires a cavity when it converges or reaches the step cap, freeing its memory for the
next request.  Requests that arrive while others run join the batch at the next chunk
boundary, so their work overlaps on the device.

All numerical work runs in the library's kernels; this module is bookkeeping only.
"""
from __future__ import annotations

import heapq
import time
from dataclasses import dataclass, field

import numpy as np

from . import lbm as _lbm


@dataclass
class Request:
    id: int
    arrival: float                 # seconds after the start of the run
    params: dict
    precision: str = "fp32"
    phi: np.ndarray | None = None
    T: np.ndarray | None = None
    C: np.ndarray | None = None


@dataclass
class Result:
    id: int
    arrival: float
    admitted: float
    finished: float
    steps: int
    converged: bool
    nodes: int
    precision: str
    obs: dict = field(default_factory=dict)
    fields: dict | None = None

    @property
    def latency(self) -> float:
        return self.finished - self.arrival




def converged(ob: dict, tol: float, quiet_speed: float) -> bool:
    """Steady state: the K-step velocity residual is below tol; in a fluid at rest (largest
    speed below quiet_speed) the scalar residuals decide instead."""
    if max(ob["max_ux"], ob["max_uy"]) < quiet_speed:
        return max(ob["r_T"], ob["r_C"]) < tol
    return ob["r_u"] < tol


class Server:
    """budget_bytes: device memory the resident cavities may use; max_slots: batch capacity;
    chunk: steps per graph replay; check_every: steps between residual checks (a multiple of
    chunk); tol, max_steps: stopping rule; autotune_steps > 0: tune the batched launch
    (lbm_batch_autotune) once, on the first resident set.  ``backend`` supplies Solver, Batch and
    footprint_bytes (the GPU library by default; tests of the bookkeeping pass a stand-in)."""

    def __init__(self, budget_bytes: int, max_slots: int = 256, chunk: int = 100, check_every: int = 1000,
                 tol: float = 1e-8, max_steps: int = 100000, keep_fields: bool = False, backend=None,
                 autotune_steps: int = 0):
        self.be = backend if backend is not None else _lbm
        if check_every % chunk:
            raise ValueError("check_every must be a multiple of chunk")
        self.budget = int(budget_bytes)
        self.max_slots = int(max_slots)
        self.chunk = int(chunk)
        self.check_every = int(check_every)
        self.tol = float(tol)
        self.max_steps = int(max_steps)
        self.keep_fields = keep_fields
        self.autotune_steps = int(autotune_steps)
        self.tuned = False
        self.batch = self.be.Batch(max_slots, chunk=chunk)
        self.solo = set()     # ids of resident solvers that the batch does not take
        self.used = 0
        self.active = []      # (solver, request, admitted, bytes, steps)
        self.node_steps = 0

    def _admit(self, req: Request, now: float) -> bool:
        need = self.be.footprint_bytes(req.params, req.precision)
        if len(self.active) >= self.max_slots or self.used + need > self.budget:
            return False
        s = self.be.Solver(req.params, phi=req.phi, T=req.T, C=req.C, precision=req.precision)
        try:
            self.batch.attach(s)
        except RuntimeError as err:
            # a cavity the batch does not take (walls through the nodes with FP16 storage or on
            # a lattice smaller than one two-step tile) is stepped on its own each chunk
            if getattr(err, "status", None) != _lbm.EINVAL:
                raise
            self.solo.add(id(s))
        self.active.append([s, req, now, need, 0])
        self.used += need
        return True

    def _retire(self, i: int, now: float, ob: dict, conv: bool) -> Result:
        s, req, adm, need, steps = self.active.pop(i)
        fields = s.fields() if self.keep_fields else None
        nodes = s.nx * s.ny
        if id(s) in self.solo:
            self.solo.discard(id(s))
        else:
            self.batch.detach(s)
        s.close()
        self.used -= need
        return Result(req.id, req.arrival, adm, now, steps, conv, nodes, req.precision, ob, fields)

    def run(self, requests, clock=time.perf_counter, log=None, progress=None, progress_every=10000):
        """Serve ``requests`` (sorted by arrival or not) to completion; returns the results in
        completion order and a summary.  ``log(result)`` is called as each request retires,
        ``progress(dict)`` every ``progress_every`` batched steps."""
        pending = [(r.arrival, r.id, r) for r in requests]
        heapq.heapify(pending)
        waiting = []
        results = []
        t0 = clock()
        batched_steps = 0
        while pending or waiting or self.active:
            now = clock() - t0
            while pending and pending[0][0] <= now:
                waiting.append(heapq.heappop(pending)[2])
            # admit in arrival order while the head fits (no overtaking by smaller requests)
            while waiting and self._admit(waiting[0], now):
                waiting.pop(0)
            if not self.active:
                if pending:
                    time.sleep(max(0.0, min(pending[0][0] - (clock() - t0), 0.01)))
                continue
            if len(self.solo) < len(self.active):
                if self.autotune_steps and not self.tuned:
                    # launch choices of the batch (tile shape, cache policy per precision and
                    # size class), timed once on the first resident set; states are restored
                    self.batch.autotune(self.autotune_steps)
                    self.tuned = True
                self.batch.step(self.chunk)
            for a in self.active:
                if id(a[0]) in self.solo:
                    a[0].step(self.chunk)
                a[4] += self.chunk
                self.node_steps += a[0].nx * a[0].ny * self.chunk
            batched_steps += self.chunk
            if progress and batched_steps % progress_every == 0:
                progress(dict(t=clock() - t0, batched_steps=batched_steps, active=len(self.active),
                              waiting=len(waiting), done=len(results)))
            # each cavity is checked on its own clock (every check_every of its steps), so a
            # request's trajectory and stopping step do not depend on what else is resident
            now = clock() - t0
            i = 0
            while i < len(self.active):
                s, req, adm, need, steps = self.active[i]
                if steps % self.check_every:
                    i += 1
                    continue
                ob = s.observables()
                U = s.derived()["U"]
                done = converged(ob, self.tol, 1e-12 * max(U, 1e-30))
                if done or ob["nonfinite"] or steps >= self.max_steps:
                    results.append(self._retire(i, now, ob, done))
                    if log:
                        log(results[-1])
                else:
                    i += 1
        wall = clock() - t0
        lat = np.array([r.latency for r in results]) if results else np.zeros(1)
        summary = dict(requests=len(results), wall_s=wall, aggregate_MLUPS=self.node_steps / max(wall, 1e-9) / 1e6,
                       p50_s=float(np.percentile(lat, 50)), p99_s=float(np.percentile(lat, 99)),
                       converged=sum(r.converged for r in results))
        return results, summary

    def close(self):
        for a in list(self.active):
            if id(a[0]) not in self.solo:
                self.batch.detach(a[0])
            a[0].close()
        self.solo.clear()
        self.active = []
        self.batch.close()
