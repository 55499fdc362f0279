"""A TF-update server over resident partitioned distance maps.

Requests are (volume id, opacity table).  The server keeps at most
`max_slots` volumes resident within an HBM byte budget: a request for a
non-resident volume admits it (upload + one-time PDM build on the admission
stream), evicting the least recently used idle volumes until the new one fits.
Serving is continuous batching: every tick gathers all queued requests whose
volume is ready (up to `max_batch`) into ONE batched TF-update launch
(pdm_batch_tf_update) on the update stream and returns at once; a tick does
not wait for earlier ticks, so requests that arrive while others are on the
GPU join the next launch and their work overlaps on the device with the
running launches and with admissions.  A request completes when its launch's
event has completed; latency is completion time minus arrival time.

The scheduling logic is independent of the device: `Executor` is the
interface, `GpuExecutor` runs the HIP library, and tests drive the same
`Server` with a CPU executor to force admission, eviction and error paths.
"""
from __future__ import annotations

import collections
import dataclasses
import itertools
import time
from typing import Callable, Dict, List, Optional

import numpy as np


@dataclasses.dataclass
class VolumeSpec:
    """A volume the server can load: where its voxels come from and how it is
    partitioned."""
    vol_id: int
    shape: tuple          # (nz, ny, nx)
    dtype: object         # np.uint8 or np.uint16
    levels: int
    bounds: np.ndarray    # n+1 partition borders
    # returns the voxels on the host: a numpy array, or a pinned torch tensor
    # (uint8, or int16 holding uint16 bits) that admission copies to the
    # device without blocking the serving loop
    load: Callable[[], object]

    @property
    def n(self) -> int:
        return len(self.bounds) - 1

    @property
    def bricks(self) -> int:
        nz, ny, nx = self.shape
        return ((nz + 3) // 4) * ((ny + 3) // 4) * ((nx + 3) // 4)


@dataclasses.dataclass
class Request:
    req_id: int
    vol_id: int
    alpha: np.ndarray
    arrival: float                 # seconds on the server clock
    done: Optional[float] = None   # completion time
    result: object = None          # executor-specific output handle
    error: Optional[str] = None


class Executor:
    """What the server needs from a device."""

    def footprint(self, spec: VolumeSpec) -> int:
        """Bytes a resident volume occupies (PDMs and outputs)."""
        raise NotImplementedError

    def admit(self, spec: VolumeSpec):
        """Start making `spec` resident; returns a handle."""
        raise NotImplementedError

    def ready(self, handle) -> bool:
        raise NotImplementedError

    def evict(self, handle) -> None:
        raise NotImplementedError

    def per_volume_limit(self) -> Optional[int]:
        """Most requests of one volume that may be launched and not yet
        retired at any time, over all launches in flight (None: no limit)."""
        return None

    def launch(self, batch: List[tuple]):
        """batch: list of (handle, alpha, request).  Start one batched update;
        returns a ticket."""
        raise NotImplementedError

    def finished(self, ticket) -> bool:
        raise NotImplementedError


class Server:
    def __init__(self, executor: Executor, catalog: Dict[int, VolumeSpec], budget_bytes: int,
                 max_slots: int = 24, max_batch: int = 48, clock=time.perf_counter,
                 on_complete: Optional[Callable[[Request], None]] = None):
        self.ex = executor
        # called for every request as it is retired, before any later launch
        # is issued (the moment its output is known to hold its result)
        self.on_complete = on_complete
        self.catalog = catalog
        self.budget = int(budget_bytes)
        self.max_slots = int(max_slots)
        self.max_batch = int(max_batch)
        self.clock = clock
        self.t0 = clock()
        self.resident: "collections.OrderedDict[int, object]" = collections.OrderedDict()  # LRU order
        self.used = 0
        self.queue: "collections.deque[Request]" = collections.deque()
        self._skipped: List[Request] = []  # taken off the queue by the running tick
        self.inflight: List[tuple] = []   # (ticket, [requests])
        self.busy: Dict[int, int] = collections.Counter()  # vol_id -> requests in flight
        self.completed: List[Request] = []
        self.rejected: List[Request] = []
        self.stats = collections.Counter()

    def now(self) -> float:
        return self.clock() - self.t0

    # ----------------------------------------------------------- residency
    def _make_room(self, need: int) -> bool:
        """Evict LRU idle volumes until `need` bytes and a slot are free."""
        while (self.used + need > self.budget or len(self.resident) >= self.max_slots):
            victim = next((v for v in self.resident if self.busy[v] == 0
                           and not any(r.vol_id == v
                                       for r in itertools.chain(self.queue, self._skipped))), None)
            if victim is None:
                victim = next((v for v in self.resident if self.busy[v] == 0), None)
            if victim is None:
                return False
            self.ex.evict(self.resident.pop(victim))
            self.used -= self.ex.footprint(self.catalog[victim])
            self.stats["evictions"] += 1
        return True

    def _ensure(self, vol_id: int) -> Optional[object]:
        if vol_id in self.resident:
            self.resident.move_to_end(vol_id)
            return self.resident[vol_id]
        spec = self.catalog[vol_id]
        need = self.ex.footprint(spec)
        if need > self.budget:
            return None
        if not self._make_room(need):
            return "wait"
        h = self.ex.admit(spec)
        self.resident[vol_id] = h
        self.used += need
        self.stats["admissions"] += 1
        return h

    # ------------------------------------------------------------- serving
    def submit(self, req: Request) -> None:
        spec = self.catalog.get(req.vol_id)
        if spec is None:
            req.error = "unknown volume"
        elif np.asarray(req.alpha).shape != (spec.levels,):
            req.error = "opacity table of the wrong length"
        elif self.ex.footprint(spec) > self.budget:
            req.error = "volume larger than the memory budget"
        if req.error:
            self.rejected.append(req)
            return
        self.queue.append(req)

    def _retire(self) -> None:
        still = []
        for ticket, reqs in self.inflight:
            if self.ex.finished(ticket):
                t = self.now()
                for r in reqs:
                    r.done = t
                    self.busy[r.vol_id] -= 1
                    self.completed.append(r)
                    if self.on_complete is not None:
                        self.on_complete(r)
            else:
                still.append((ticket, reqs))
        self.inflight = still

    def tick(self) -> int:
        """Retire finished launches, admit volumes for queued requests, and
        launch one batch of ready requests, taken in arrival order.  The scan
        stops once the batch is full, so a long queue costs no more per tick
        than the requests it skips (volume not ready, or its limit of
        requests in flight reached).  Returns the batch size."""
        self._retire()
        batch, skipped = [], self._skipped
        limit = self.ex.per_volume_limit()
        q = self.queue
        while q and len(batch) < self.max_batch:
            r = q.popleft()
            # at most `limit` requests of a volume launched and not yet
            # retired, counting this batch (busy is raised as requests join
            # it): the executor's per-volume resources (output maps) are
            # never handed to a request while an earlier holder is in flight
            if limit is not None and self.busy[r.vol_id] >= limit:
                skipped.append(r)
                continue
            h = self._ensure(r.vol_id)
            if h is None:
                r.error = "volume larger than the memory budget"
                self.rejected.append(r)
            elif isinstance(h, str) or not self.ex.ready(h):
                skipped.append(r)
            else:
                # counted busy at once, so a later admission in this tick
                # cannot evict this volume
                self.busy[r.vol_id] += 1
                batch.append((h, r.alpha, r))
        q.extendleft(reversed(skipped))
        skipped.clear()
        if batch:
            self.inflight.append((self.ex.launch(batch), [r for _, _, r in batch]))
            self.stats["launches"] += 1
            self.stats["batched_requests"] += len(batch)
        return len(batch)

    def drain(self, timeout: float = 60.0) -> None:
        """Serve until the queue is empty and every launch has completed.
        Polls without sleeping: a sleep's wake-up slack (tens of
        microseconds and more) would add to every request's latency."""
        end = self.now() + timeout
        while (self.queue or self.inflight) and self.now() < end:
            self.tick()

    def run(self, schedule: List[Request], timeout: float = 120.0,
            idle_sleep_s: float = 0.0005) -> None:
        """Feed requests at their arrival times (server clock) and serve
        until all are done.  The loop polls while work is queued or in flight
        and sleeps only when idle with the next arrival more than
        `idle_sleep_s` away (waking that long before it)."""
        schedule = sorted(schedule, key=lambda r: r.arrival)
        i = 0
        end = self.now() + timeout
        while (i < len(schedule) or self.queue or self.inflight) and self.now() < end:
            t = self.now()
            while i < len(schedule) and schedule[i].arrival <= t:
                self.submit(schedule[i])
                i += 1
            self.tick()
            if not self.queue and not self.inflight and i < len(schedule):
                gap = schedule[i].arrival - self.now()
                if gap > 2 * idle_sleep_s:
                    time.sleep(gap - idle_sleep_s)

    def report(self) -> dict:
        lat = np.array([r.done - r.arrival for r in self.completed]) if self.completed else np.zeros(0)
        span = (max(r.done for r in self.completed) - min(r.arrival for r in self.completed)
                if self.completed else 0.0)
        return {
            "completed": len(self.completed),
            "rejected": len(self.rejected),
            "p50_ms": float(np.percentile(lat, 50) * 1e3) if lat.size else None,
            "p99_ms": float(np.percentile(lat, 99) * 1e3) if lat.size else None,
            "mean_ms": float(lat.mean() * 1e3) if lat.size else None,
            "updates_per_s": len(self.completed) / span if span > 0 else None,
            "launches": self.stats["launches"],
            "mean_batch": (self.stats["batched_requests"] / self.stats["launches"]
                           if self.stats["launches"] else None),
            "admissions": self.stats["admissions"],
            "evictions": self.stats["evictions"],
        }


def requests_from(arrivals) -> List[Request]:
    """Requests from (arrival seconds, volume id, opacity table) tuples."""
    return [Request(k, int(v), np.asarray(alpha, np.float32), float(t))
            for k, (t, v, alpha) in enumerate(arrivals)]


class GpuExecutor(Executor):
    """Runs the server on the GPU through the C ABI.  Admission uploads the
    voxels and builds bricks and PDMs (and, with `range_level`, the range
    table) on `admit_stream`; updates run on `update_stream`, one batched
    launch per tick (with `range_level`: the batched update through the
    tables).  Each request gets an output map from a per-volume pool of
    `outputs_per_volume` buffers, used in turn, and at most that many
    requests of a volume are in flight at once (the server's per-volume
    limit), so a buffer is handed out again only after its previous request
    has been retired: a result stays valid from its completion until that
    many later requests of the same volume have been launched."""

    def __init__(self, outputs_per_volume: int = 8, keep_volume: bool = False,
                 range_level: Optional[int] = None):
        import torch
        self.torch = torch
        self.admit_stream = torch.cuda.Stream()
        self.update_stream = torch.cuda.Stream()
        self.outputs = int(outputs_per_volume)
        self.keep_volume = keep_volume
        # with a range level, admission also builds each volume's range table
        # and a tick's batch updates through the tables (fewer maps read than
        # the batched update of the active PDMs)
        self.range_level = range_level

    def footprint(self, spec: VolumeSpec) -> int:
        import paper_2407_21552_amd as pdm
        G = spec.bricks
        s = np.dtype(spec.dtype).itemsize
        vox = int(np.prod(spec.shape)) * s
        table = pdm.range_table_maps(spec.n, self.range_level) * G if self.range_level else 0
        return spec.n * G + table + self.outputs * G + 2 * G * s + (vox if self.keep_volume else 0)

    class Handle:
        pass

    def admit(self, spec: VolumeSpec):
        import paper_2407_21552_amd as pdm
        torch = self.torch
        h = GpuExecutor.Handle()
        h.spec = spec
        h.is_ready = False
        vox = spec.load()
        with torch.cuda.stream(self.admit_stream):
            if isinstance(vox, torch.Tensor):
                # pinned host voxels: an asynchronous copy on the admission
                # stream, ordered before the build on the same stream
                dev = vox.to("cuda", non_blocking=True)
            else:
                dev = pdm.to_device(vox)
            h.vol = pdm.Volume(dev, spec.levels, spec.bounds, voxel_dtype=spec.dtype)
            h.vol.build(self.admit_stream)
            if self.range_level:
                h.vol.build_range_table(self.range_level, self.admit_stream)
            h.outs = [torch.empty_like(h.vol.dist) for _ in range(self.outputs)]
            h.next_out = 0
            h.ready_ev = torch.cuda.Event()
            h.ready_ev.record(self.admit_stream)
        # PDMs and outputs are used on the update stream: keep the allocator
        # from reusing them while launches there may still run
        h.vol.pdms.record_stream(self.update_stream)
        if self.range_level and h.vol.table is not None:
            h.vol.table.record_stream(self.update_stream)
        for o in h.outs:
            o.record_stream(self.update_stream)
        # the server launches a volume's requests only once ready() has seen
        # the build event complete, so the update stream needs no wait here
        # (a wait would hold every later tick behind this build)
        h.drop_volume_after_ready = not self.keep_volume
        return h

    def ready(self, h) -> bool:
        if h.is_ready:  # a built volume stays built: no event query per request
            return True
        ok = h.ready_ev.query()
        if ok:
            h.is_ready = True
            if h.drop_volume_after_ready:
                h.vol.volume = None  # voxels are not needed once the PDMs exist
        return ok

    def evict(self, h) -> None:
        h.vol = None
        h.outs = None

    def per_volume_limit(self) -> Optional[int]:
        return self.outputs

    def launch(self, batch):
        import paper_2407_21552_amd as pdm
        torch = self.torch
        entries = []
        for h, alpha, req in batch:
            out = h.outs[h.next_out]
            h.next_out = (h.next_out + 1) % len(h.outs)
            req.result = out
            entries.append((h.vol.prepared, alpha, out))
        if self.range_level:
            pdm.batch_tf_update_ranges_prepared(entries, self.update_stream)
        else:
            pdm.batch_tf_update_prepared(entries, self.update_stream)
        ev = torch.cuda.Event()
        ev.record(self.update_stream)
        return ev

    def finished(self, ev) -> bool:
        return ev.query()
