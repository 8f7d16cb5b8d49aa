"""Continuous-batching server of independent small solves.

Requests (a workload each, with an arrival time) are admitted in arrival
order while a slot of the fused batch and device memory are free.  An
admitted solve keeps its fields and workspace on the device until it has run
all its steps.  Each fused call (rt_step_many) advances every admitted solve
by one step; requests that arrive meanwhile join at the next call, and a
solve that has finished leaves its slot and memory to the next request.
While a call runs on the GPU, the host opens (uploads) the requests that are
next in line, for as long as the call runs, up to a batch's worth and within
the memory budget, so that they join a later call without waiting for their
upload.  Between calls at most `sync_open` requests are opened before the
next call starts (none once the batch is half full and more than that are
waiting: the backlog goes up while the calls run).  Latency is
completion minus arrival.

Host-side scheduling only: every step of every solve runs in the library's
kernels.  The baseline is the same requests run one at a time through rt_step.
"""
from __future__ import annotations

import collections
import dataclasses
import time
from typing import Callable, List, Optional

import numpy as np

from . import rt


@dataclasses.dataclass
class Served:
    rid: int
    arrival_s: float
    admit_s: float
    done_s: float
    steps: int
    crossings: int
    packets: int
    emitted: float
    residual: float                 # max over steps of |emitted - absorbed - escaped - truncated| / emitted
    fields: Optional[np.ndarray]    # rt.FIELDS order, natural cell order, float64

    @property
    def latency_s(self) -> float:
        return self.done_s - self.arrival_s


def workspace_bytes(work, fp64: bool, direct: bool = True) -> int:
    """Device bytes a request holds while admitted (its workspace; fields in
    bricks of 8^3, as the fused tiled march reads them)."""
    d = rt.desc_from_workload(work, fp64=fp64, direct=direct, brick_log2=3 if direct else -1)
    return rt.rt_workspace_bytes(d, max(1, len(work.src_ndot)))


def round_packets(work) -> int:
    """Packets of one sub-step of a request (the most any of its sub-steps has)."""
    return -(-int(work.packets) // int(work.n_sub))


def percentile(values, q: float) -> float:
    return float(np.percentile(np.asarray(values, dtype=np.float64), q)) if len(values) else float("nan")


def admissible(need: int, used: int, n_active: int, max_slots: int, budget: int) -> bool:
    """A request is admitted when a slot is free and its workspace fits."""
    return n_active < max_slots and used + need <= budget


def fits_batch(packets: int, tiles: int, used_packets: int, used_tiles: int, max_packets: int,
               max_tiles: int) -> bool:
    """... and its packets per sub-step and tiles fit what the fused march holds."""
    return used_packets + packets <= max_packets and used_tiles + tiles <= max_tiles


class GpuExecutor:
    """Solves on the current GPU, stepped together by rt_step_many on the
    batch's stream (their fields and workspaces stay on the device).  The
    batch takes its march instance from the first request it opens.  Solves
    are opened on a stream of their own, so that an upload runs beside a
    fused call instead of after it."""

    def __init__(self, max_slots: int, *, fp64: bool, graph: bool, max_round_packets: int, max_tiles: int,
                 device: str = "cuda", **tiles):
        self.fp64 = fp64
        self.device = device
        self.max_slots = max_slots
        self.graph = graph
        self.max_round_packets = max_round_packets
        self.max_tiles = max_tiles
        self.tiles = tiles
        self.batch = None
        self.open_stream = None

    def open(self, work):
        if self.batch is None:
            import torch
            self.batch = rt.Batch(self.max_slots, work, fp64=self.fp64, max_round_packets=self.max_round_packets,
                                  max_tiles=self.max_tiles, graph=self.graph, device=self.device, **self.tiles)
            self.open_stream = torch.cuda.Stream(device=self.device)
        return rt.Solve(work, fp64=self.fp64, direct=True, brick_log2=3, stream=self.open_stream,
                        device=self.device)

    def step(self, solves):
        return self.batch.step(solves, stats=True)       # synchronises

    def launch(self, solves):
        import torch
        self.batch.launch(solves)                        # returns at once
        self.launched = torch.cuda.Event()
        self.launched.record(self.batch.stream)

    def busy(self) -> bool:
        """The last launched call is still running."""
        return not self.launched.query()

    def wait(self):
        return self.batch.wait()

    def fetch(self, solve):
        return solve.fetch()

    def close(self, solve):
        solve.release()

    def release(self):
        if self.batch is not None:
            self.batch.release()


class Server:
    """Admits requests into one fused batch of at most max_slots solves and a
    device-memory budget (bytes of solve workspaces; default half the free
    device memory when the server starts)."""

    def __init__(self, *, max_slots: int = rt.RT_MAX_BATCH, hbm_budget: Optional[int] = None,
                 fp64: bool = False, graph: bool = True, keep_fields: bool = True, device: str = "cuda",
                 executor=None, max_round_packets: int = rt.RT_MAX_BATCH * 100_000,
                 max_tiles: int = rt.RT_MAX_BATCH * 512, sync_open: int = 32, **tiles):
        if not 1 <= max_slots <= rt.RT_MAX_BATCH:
            raise ValueError(f"max_slots must be in 1..{rt.RT_MAX_BATCH}")
        if sync_open < 1:
            raise ValueError("sync_open must be at least 1")
        self.max_slots = max_slots
        self.sync_open = int(sync_open)
        self.fp64 = fp64
        self.keep_fields = keep_fields
        self.max_round_packets = int(max_round_packets)
        self.max_tiles = int(max_tiles)
        if hbm_budget is None:
            import torch
            free, _ = torch.cuda.mem_get_info()
            hbm_budget = free // 2
        self.hbm_budget = int(hbm_budget)
        self.ex = executor if executor is not None else GpuExecutor(
            max_slots, fp64=fp64, graph=graph, max_round_packets=self.max_round_packets, max_tiles=self.max_tiles,
            device=device, **tiles)
        self.calls = 0
        self.call_solves = []          # solves per fused call
        self.peak_bytes = 0            # most workspace bytes admitted at once

    def run(self, requests, *, realtime: bool = True,
            clock: Callable[[], float] = time.perf_counter) -> List[Served]:
        """Serve every request; arrivals follow request.arrival_s from the
        start of the run when realtime, else all are present at once."""
        pending = collections.deque(sorted(requests, key=lambda r: (r.arrival_s, r.rid)))
        need = {r.rid: workspace_bytes(r.work, self.fp64) for r in pending}
        pk = {r.rid: round_packets(r.work) for r in pending}
        tl = {r.rid: rt.tiles_of(r.work.n) for r in pending}
        for r in pending:
            if need[r.rid] > self.hbm_budget:
                raise ValueError(f"request {r.rid} needs {need[r.rid]} bytes, above the budget")
            if pk[r.rid] > self.max_round_packets or tl[r.rid] > self.max_tiles:
                raise ValueError(f"request {r.rid} does not fit the fused march ({pk[r.rid]} packets per "
                                 f"sub-step, {tl[r.rid]} tiles)")
        active = []                    # [request, solve, admit time, steps done, ledgers]
        opened = {}                    # rid -> solve opened ahead of admission (memory held, no slot)
        used = used_pk = used_tl = 0   # used: bytes of admitted and opened-ahead solves
        out: List[Served] = []
        overlap = hasattr(self.ex, "launch")
        t0 = clock()
        try:
            while pending or active:
                now = clock() - t0
                n_sync = 0                 # requests opened now, with the GPU idle
                cap = self.sync_open
                if overlap and 2 * len(active) >= self.max_slots:
                    # with the batch at least half full, a backlog longer than
                    # sync_open goes up while calls run: opening it now would
                    # hold the next call back
                    waiting = 0
                    for r in pending:
                        if realtime and r.arrival_s > now:
                            break
                        waiting += r.rid not in opened
                    if waiting > self.sync_open:
                        cap = 0
                while pending and (not realtime or pending[0].arrival_s <= now):
                    r = pending[0]
                    ahead = r.rid in opened
                    if overlap and not ahead and n_sync >= cap:
                        break              # the rest go up while the next call runs
                    if not (admissible(0 if ahead else need[r.rid], used, len(active), self.max_slots,
                                       self.hbm_budget)
                            and fits_batch(pk[r.rid], tl[r.rid], used_pk, used_tl, self.max_round_packets,
                                           self.max_tiles)):
                        break
                    pending.popleft()
                    if ahead:
                        s = opened.pop(r.rid)
                    else:
                        s = self.ex.open(r.work)
                        n_sync += 1
                        used += need[r.rid]
                    used_pk += pk[r.rid]
                    used_tl += tl[r.rid]
                    self.peak_bytes = max(self.peak_bytes, used)
                    active.append([r, s, clock() - t0, 0, []])
                if not active:
                    wait = pending[0].arrival_s - (clock() - t0)
                    if wait > 0:
                        time.sleep(min(wait, 0.05))
                    continue
                if overlap:
                    self.ex.launch([a[1] for a in active])
                    # the next requests in line go up while the call runs
                    now = clock() - t0
                    for r in pending:
                        if not self.ex.busy() or len(opened) >= self.max_slots or (realtime and r.arrival_s > now):
                            break
                        if r.rid in opened:
                            continue
                        if used + need[r.rid] > self.hbm_budget:
                            break
                        opened[r.rid] = self.ex.open(r.work)
                        used += need[r.rid]
                        self.peak_bytes = max(self.peak_bytes, used)
                    ledgers = self.ex.wait()
                else:
                    ledgers = self.ex.step([a[1] for a in active])
                self.calls += 1
                self.call_solves.append(len(active))
                done_t = clock() - t0
                still = []
                for a, st in zip(active, ledgers):
                    a[3] += 1
                    a[4].append(st)
                    if a[3] < a[0].work.steps:
                        still.append(a)
                        continue
                    r, s = a[0], a[1]
                    fields = self.ex.fetch(s) if self.keep_fields else None
                    self.ex.close(s)
                    used -= need[r.rid]
                    used_pk -= pk[r.rid]
                    used_tl -= tl[r.rid]
                    led = a[4]
                    res = max(abs(x["emitted"] - (x["absorbed"] + x["escaped"] + x["truncated"])) / x["emitted"]
                              if x["emitted"] > 0 else 0.0 for x in led)
                    out.append(Served(r.rid, r.arrival_s, a[2], done_t, a[3], sum(x["crossings"] for x in led),
                                      sum(x["packets"] for x in led), sum(x["emitted"] for x in led), res, fields))
                active = still
        except BaseException:
            # a failed run leaves no solve open behind it
            for a in active:
                self.ex.close(a[1])
            for s in opened.values():
                self.ex.close(s)
            raise
        return sorted(out, key=lambda x: x.rid)

    def release(self):
        self.ex.release()


def run_alone(requests, *, fp64: bool = True, direct: bool = True, keep_fields: bool = True,
              device: str = "cuda", clock: Callable[[], float] = time.perf_counter):
    """The requests one at a time, each with rt_step on its own solve (all
    present at once: no arrival times).  Returns (results, seconds)."""
    import torch
    out = []
    t0 = clock()
    for r in sorted(requests, key=lambda q: q.rid):
        s = rt.Solve(r.work, fp64=fp64, direct=direct, device=device)
        led = [s.step() for _ in range(r.work.steps)]
        fields = s.fetch() if keep_fields else None
        s.release()
        res = max(abs(x["emitted"] - (x["absorbed"] + x["escaped"] + x["truncated"])) / x["emitted"]
                  if x["emitted"] > 0 else 0.0 for x in led)
        t = clock() - t0
        out.append(Served(r.rid, 0.0, 0.0, t, len(led), sum(x["crossings"] for x in led),
                          sum(x["packets"] for x in led), sum(x["emitted"] for x in led), res, fields))
    torch.cuda.synchronize()
    return out, clock() - t0
