"""Continuous-batching request loop over a gd_pool (argument marshalling and
host bookkeeping only; every step of every integration runs in the HIP
library).

Requests (independent clusters: masses, positions, velocities already on the
device, and an end time) arrive at given times. The loop admits arrived
requests in arrival order whenever a pool slot and room in the device arena
are free (admission by footprint), advances all resident clusters together
with gd_pool_run, and retires clusters as they finish, recording for each its
arrival, admission and completion times.

A request that fails (rejected parameters or inputs, a non-finite force at
admission or later, or a footprint larger than the whole arena) is recorded
as a failed Result with its status, its slot is released, and the other
requests go on.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import torch

from . import gravidy as g


@dataclass
class Request:
    rid: int
    arrival: float  # seconds after the start of serving
    m: torch.Tensor
    x: torch.Tensor
    v: torch.Tensor
    t_end: float


@dataclass
class Result:
    rid: int
    n: int
    arrival: float
    admitted: float
    done: float
    stats: dict | None
    x: torch.Tensor | None = None
    v: torch.Tensor | None = None
    status: str = "GD_OK"  # the library's status name for a failed request
    error: str | None = None

    @property
    def ok(self) -> bool:
        return self.status == "GD_OK"

    @property
    def latency(self) -> float:
        return self.done - self.arrival


@dataclass
class PoolServer:
    params: g.gd_params
    max_clusters: int
    arena_bytes: int
    device: str = "cuda:0"
    keep_state: bool = False
    arena: torch.Tensor = field(init=False)
    pool: object = field(init=False)

    def __post_init__(self):
        self.arena = torch.empty(self.arena_bytes, dtype=torch.uint8, device=self.device)
        self.pool = g.gd_pool_create(self.params, self.max_clusters, self.arena)
        # Arena bytes beyond the pool tables: what the workspaces can use.
        self.heap_bytes = self.arena_bytes - g.gd_pool_arena_bytes(self.max_clusters, [])

    def fits_alone(self, n: int) -> bool:
        """Whether a cluster of n particles fits the empty arena."""
        return g.gd_workspace_bytes(n, self.params) <= self.heap_bytes

    def close(self):
        if self.pool:
            g.gd_pool_destroy(self.pool)
            self.pool = None

    def serve(self, requests: list[Request]) -> list[Result]:
        pending = collections.deque(sorted(requests, key=lambda r: r.arrival))
        waiting: collections.deque = collections.deque()
        running: dict[int, tuple[Request, float]] = {}
        results: list[Result] = []
        t0 = time.perf_counter()

        def failed(r: Request, t_adm: float, e: g.GdError) -> Result:
            return Result(r.rid, r.m.shape[0], r.arrival, t_adm, time.perf_counter() - t0, None,
                          status=g.status_name(e.status), error=str(e))

        while pending or waiting or running:
            now = time.perf_counter() - t0
            while pending and pending[0].arrival <= now:
                waiting.append(pending.popleft())
            while waiting:
                r = waiting[0]
                t_adm = time.perf_counter() - t0
                if not self.fits_alone(r.m.shape[0]):
                    waiting.popleft()
                    results.append(failed(r, t_adm, g.GdError(g.GD_ENOMEM, "cluster larger than the arena")))
                    continue
                try:
                    slot = g.gd_pool_admit(self.pool, r.m, r.x, r.v, r.t_end)
                except g.GdError as e:
                    waiting.popleft()
                    results.append(failed(r, t_adm, e))
                    continue
                if slot is None:
                    break
                waiting.popleft()
                running[slot] = (r, t_adm)
            if running:
                for slot in g.gd_pool_run(self.pool):
                    r, t_adm = running.pop(slot)
                    xo = vo = None
                    if self.keep_state:
                        xo = torch.empty_like(r.x)
                        vo = torch.empty_like(r.v)
                    try:
                        st = g.gd_pool_result(self.pool, slot, xo, vo)
                        res = Result(r.rid, r.m.shape[0], r.arrival, t_adm, time.perf_counter() - t0, st, xo, vo)
                    except g.GdError as e:
                        res = failed(r, t_adm, e)
                    g.gd_pool_release(self.pool, slot)
                    results.append(res)
            elif pending:
                time.sleep(max(0.0, min(1e-3, pending[0].arrival - (time.perf_counter() - t0))))
        return results


def serve_sequential(params: g.gd_params, requests: list[Request], device="cuda:0",
                     keep_state=False) -> list[Result]:
    """The same requests, one after the other, each with its own context
    (gd_init, gd_step_to to its end time): the plain baseline."""
    results = []
    t0 = time.perf_counter()
    for r in sorted(requests, key=lambda r: r.arrival):
        now = time.perf_counter() - t0
        if r.arrival > now:
            time.sleep(r.arrival - now)
        t_adm = time.perf_counter() - t0
        n = r.m.shape[0]
        ws = torch.empty(g.gd_workspace_bytes(n, params), dtype=torch.uint8, device=device)
        ctx = None
        try:
            ctx = g.gd_init(params, r.m, r.x, r.v, ws)
            st = g.gd_step_to(ctx, r.t_end)
            xo = vo = None
            if keep_state:
                xo = torch.empty_like(r.x)
                vo = torch.empty_like(r.v)
                g.gd_get_state(ctx, xo, vo)
            res = Result(r.rid, n, r.arrival, t_adm, time.perf_counter() - t0, st, xo, vo)
        except g.GdError as e:
            res = Result(r.rid, n, r.arrival, t_adm, time.perf_counter() - t0, None,
                         status=g.status_name(e.status), error=str(e))
        finally:
            g.gd_destroy(ctx)
        results.append(res)
    return results
