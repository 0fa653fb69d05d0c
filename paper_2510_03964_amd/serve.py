"""Serving loop: many foveated-rendering sessions sharing one GPU.

Sessions arrive over time (a Poisson process in the benchmark), each with its
own resolution, slot count k and frame rate.  A session is admitted when its
reservoir store (``fwrs_state_bytes``) fits in the remaining HBM budget and a
slot is free; otherwise it waits in a FIFO queue.  Frame i of an admitted
session is due at admit_time + i / fps.  Continuous batching: whenever fewer
than `max_inflight` ticks are on the GPU, the loop gathers the due frames of
every active session -- up to `max_group` consecutive ones per session, oldest
first -- and submits them together as one batched tick (``fwrs_engine_tick``,
in which a session's several frames run as one group that reads and writes
its reservoir once); frames that come due while the GPU is busy ride along in
the next tick, so batches grow with the load.  Sessions that end release
their memory and the queue is re-examined.  Each frame's latency is completion - due time; the
deadline is one 90 Hz frame (11.1 ms).

The scheduler (`Scheduler`) is pure host logic behind a small executor
interface, so it runs against a fake executor and a virtual clock in the tests;
`BatchedExecutor` and `PlainExecutor` drive the GPU library (one batched launch
per tick, or one launch per frame, on the same stream).
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np

DEADLINE_MS = 1000.0 / 90.0


@dataclass(frozen=True)
class SessionSpec:
    sid: int
    arrival_s: float
    lifetime_s: float
    width: int
    height: int
    k: int
    fps: float

    @property
    def pixels(self) -> int:
        return self.width * self.height


def poisson_sessions(n: int = 32, rate_per_s: float = 1.0, seed: int = 4242, time_scale: float = 1.0,
                     lifetime_s=(10.0, 60.0), sizes=((1920, 1080), (3840, 2160)), ks=(4, 8),
                     fps=(72.0, 90.0, 120.0)) -> list[SessionSpec]:
    """n sessions with exponential inter-arrival times (mean 1 / rate), lifetime ~ U[lifetime_s],
    resolution, k and frame rate drawn uniformly.  time_scale < 1 compresses arrivals and
    lifetimes alike (same concurrency and offered load, shorter run)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    t = 0.0
    out = []
    for sid in range(n):
        t += rng.exponential(1.0 / rate_per_s)
        life = rng.uniform(*lifetime_s)
        w, h = sizes[int(rng.integers(len(sizes)))]
        out.append(SessionSpec(sid, t * time_scale, life * time_scale, int(w), int(h), int(ks[int(rng.integers(len(ks)))]),
                               float(fps[int(rng.integers(len(fps)))])))
    return out


@dataclass
class _Active:
    spec: SessionSpec
    handle: object
    admit_s: float
    end_s: float
    next_frame: int = 0

    def due_s(self, i: int) -> float:
        return self.admit_s + i / self.spec.fps


@dataclass
class FrameRecord:
    sid: int
    index: int
    due_s: float
    submit_s: float
    tick: int
    done_s: float = math.nan


@dataclass
class ServeStats:
    frames: int
    pixel_updates: int
    wall_s: float
    latency_ms: np.ndarray
    deadline_misses: int
    admitted: int
    rejected: int
    max_queue: int
    max_active: int
    ticks: int
    max_batch: int = 0
    max_group: int = 0
    queue_wait_s: list = field(default_factory=list)

    def summary(self) -> dict:
        lat = self.latency_ms
        return {
            "frames": self.frames, "ticks": self.ticks, "pixel_updates": self.pixel_updates,
            "wall_s": self.wall_s, "gpix_per_s": self.pixel_updates / self.wall_s / 1e9 if self.wall_s > 0 else 0.0,
            "latency_ms_p50": float(np.percentile(lat, 50)) if lat.size else None,
            "latency_ms_p99": float(np.percentile(lat, 99)) if lat.size else None,
            "latency_ms_max": float(lat.max()) if lat.size else None,
            "deadline_ms": DEADLINE_MS, "deadline_misses": self.deadline_misses,
            "sessions_admitted": self.admitted, "sessions_never_admitted": self.rejected,
            "max_queue": self.max_queue, "max_active": self.max_active, "max_batch": self.max_batch,
            "max_frames_of_a_session_per_tick": self.max_group,
            "frames_per_tick": self.frames / self.ticks if self.ticks else 0.0,
            "queue_wait_s_max": max(self.queue_wait_s) if self.queue_wait_s else 0.0,
        }


class Scheduler:
    """Admission, batching and latency bookkeeping; the executor does the work.

    Executor interface:
      state_bytes(spec) -> int
      open(spec) -> handle            (allocates the session's reservoir)
      close(handle)
      submit(list[(handle, frame_index)]) -> tick id   (asynchronous; a session's frames
                                                       consecutive and in order)
      poll() -> list[(tick id, completion time in the clock's seconds)]
      drain() -> same as poll, after waiting for all submitted work
      max_batch (optional attribute) -> the most frames one submit may carry
    """

    def __init__(self, executor, budget_bytes: int, max_active: int = 64, max_inflight: int = 2,
                 max_group: int = 1, clock=time.perf_counter, sleep=time.sleep):
        self.ex = executor
        self.budget = int(budget_bytes)
        self.max_active = int(max_active)
        self.max_inflight = int(max_inflight)
        self.max_group = int(max_group)
        if self.max_group < 1:
            raise ValueError("max_group must be at least 1")
        self.clock = clock
        self.sleep = sleep

    def run(self, sessions: list[SessionSpec], until_s: float | None = None) -> ServeStats:
        ex = self.ex
        pending = sorted(sessions, key=lambda s: (s.arrival_s, s.sid))
        for s in pending:
            if ex.state_bytes(s) > self.budget:
                raise ValueError(f"session {s.sid} can never fit the budget")
        queue: list[tuple[float, SessionSpec]] = []
        active: dict[int, _Active] = {}
        used = 0
        records: list[FrameRecord] = []
        tick_frames: dict[int, list[int]] = {}
        queue_wait = []
        stats = dict(admitted=0, max_queue=0, max_active=0, ticks=0, max_batch=0, max_group=0)
        t0 = self.clock()
        now = 0.0
        horizon = until_s if until_s is not None else max((s.arrival_s + s.lifetime_s for s in pending), default=0.0)
        pi = 0

        def finish_completed(done):
            for tick, t_done in done:
                for ri in tick_frames.pop(tick, []):
                    records[ri].done_s = t_done - t0

        while True:
            now = self.clock() - t0
            # arrivals join the queue
            while pi < len(pending) and pending[pi].arrival_s <= now:
                queue.append((pending[pi].arrival_s, pending[pi]))
                pi += 1
            # sessions whose lifetime is over leave and free their memory
            for sid in [sid for sid, a in active.items() if a.end_s <= now]:
                a = active.pop(sid)
                ex.close(a.handle)
                used -= ex.state_bytes(a.spec)
            # admission in arrival order while the budget and the slots allow
            while queue and len(active) < self.max_active:
                arr, spec = queue[0]
                if arr + spec.lifetime_s <= now:       # its lifetime ran out while it waited
                    queue.pop(0)
                    continue
                need = ex.state_bytes(spec)
                if used + need > self.budget:
                    break
                queue.pop(0)
                used += need
                # the session ends at arrival + lifetime; time spent queued is lost to it
                active[spec.sid] = _Active(spec, ex.open(spec), now, arr + spec.lifetime_s)
                queue_wait.append(now - arr)
                stats["admitted"] += 1
            stats["max_queue"] = max(stats["max_queue"], len(queue))
            stats["max_active"] = max(stats["max_active"], len(active))
            # continuous batching: every active session's due frames (at most max_group, oldest
            # first), once the GPU has room for another tick
            batch = []
            if len(tick_frames) < self.max_inflight:
                for a in active.values():
                    m = 0
                    while m < self.max_group and a.due_s(a.next_frame + m) <= now and \
                            a.due_s(a.next_frame + m) < a.end_s:
                        m += 1
                    if m:
                        batch.append([a, m])
                cap = getattr(ex, "max_batch", None)
                if cap is not None and sum(m for _, m in batch) > cap:   # the rest stay due for the next tick
                    batch.sort(key=lambda am: am[0].due_s(am[0].next_frame))
                    left, kept = cap, []
                    for a, m in batch:
                        if left == 0:
                            break
                        kept.append([a, min(m, left)])
                        left -= kept[-1][1]
                    batch = kept
            if batch:
                n_frames = sum(m for _, m in batch)
                stats["max_batch"] = max(stats["max_batch"], n_frames)
                stats["max_group"] = max(stats["max_group"], max(m for _, m in batch))
                tick = ex.submit([(a.handle, a.next_frame + j) for a, m in batch for j in range(m)])
                stats["ticks"] += 1
                idx = []
                for a, m in batch:
                    for j in range(m):
                        i = a.next_frame + j
                        records.append(FrameRecord(a.spec.sid, i, a.due_s(i), now, tick))
                        idx.append(len(records) - 1)
                    a.next_frame += m
                tick_frames[tick] = idx
            finish_completed(ex.poll())
            if pi >= len(pending) and not queue and not active:
                break
            if now > horizon + 1.0:
                break
            if not batch:
                # sleep until the next event: a due frame, an arrival, a departure, a completion
                nxt = [a.due_s(a.next_frame) for a in active.values()]
                nxt += [a.end_s for a in active.values()]
                if pi < len(pending):
                    nxt.append(pending[pi].arrival_s)
                wait = min(nxt) - (self.clock() - t0) if nxt else 0.0
                if tick_frames:
                    wait = min(wait, 50e-6)
                if wait > 0:
                    self.sleep(min(wait, 0.002))
        finish_completed(ex.drain())
        for a in active.values():
            ex.close(a.handle)
        wall = max((r.done_s for r in records), default=0.0) - min((r.due_s for r in records), default=0.0)
        lat = np.array([(r.done_s - r.due_s) * 1e3 for r in records if not math.isnan(r.done_s)])
        pixels = {s.sid: s.pixels for s in sessions}
        px = sum(pixels[r.sid] for r in records)
        self.frames_done = {}
        for r in records:
            self.frames_done[r.sid] = max(self.frames_done.get(r.sid, 0), r.index + 1)
        return ServeStats(frames=len(records), pixel_updates=px, wall_s=wall, latency_ms=lat,
                          deadline_misses=int(np.count_nonzero(lat > DEADLINE_MS)), admitted=stats["admitted"],
                          rejected=len(sessions) - stats["admitted"], max_queue=stats["max_queue"],
                          max_active=stats["max_active"], ticks=stats["ticks"], max_batch=stats["max_batch"],
                          max_group=stats["max_group"], queue_wait_s=queue_wait)


# ---------------------------------------------------------------------------
# GPU executors
# ---------------------------------------------------------------------------
class _GpuExecutor:
    """Shared by both GPU executors: per-session contexts, output buffers and input rings."""

    def __init__(self, frames_by_size: dict, stream=None, seed: int = 0x25103964, tiles: dict | None = None):
        import torch

        from . import fwrs

        self.torch = torch
        self.fwrs = fwrs
        self.frames = frames_by_size          # (w, h) -> list of (colour, level, gx, gy)
        self.stream = stream or torch.cuda.current_stream()
        self.seed = seed
        self.tiles = tiles or {}
        self.pending: list[tuple[int, object]] = []
        self.next_tick = 0
        self.ref = None
        self.ref_host = 0.0
        self.outputs: dict[int, object] = {}

    def state_bytes(self, spec: SessionSpec) -> int:
        return self.fwrs.state_bytes(spec.width, spec.height, spec.k)

    def open(self, spec: SessionSpec):
        fw = self.fwrs
        p = fw.default_params(spec.width, seed=self.seed, stream_id=spec.sid)
        r = fw.Reservoir(spec.width, spec.height, spec.k, p, stream=self.stream)
        if (spec.width, spec.height) in self.tiles:
            r.set_tile(*self.tiles[(spec.width, spec.height)])
        out = self.torch.empty((spec.height, spec.width, 3), dtype=self.torch.float32, device="cuda")
        self.outputs[spec.sid] = out
        return (spec, r, out)

    def close(self, handle) -> None:
        spec, r, _ = handle
        r.close()

    def frame(self, handle, i):
        spec = handle[0]
        ring = self.frames[(spec.width, spec.height)]
        return ring[(i + 7 * spec.sid) % len(ring)]

    def _clock_ref(self):
        if self.ref is None:
            self.ref = self.torch.cuda.Event(enable_timing=True)
            self.ref.record(self.stream)
            self.ref.synchronize()
            self.ref_host = time.perf_counter()

    def _mark(self):
        self._clock_ref()
        ev = self.torch.cuda.Event(enable_timing=True)
        ev.record(self.stream)
        tick = self.next_tick
        self.next_tick += 1
        self.pending.append((tick, ev))
        return tick

    def poll(self):
        done = []
        while self.pending and self.pending[0][1].query():
            tick, ev = self.pending.pop(0)
            done.append((tick, self.ref_host + self.ref.elapsed_time(ev) / 1e3))
        return done

    def drain(self):
        self.torch.cuda.synchronize()
        return self.poll()


class BatchedExecutor(_GpuExecutor):
    """One batched tick for all due frames: one kernel launch for all of them (a session's several
    frames as one group), issued directly or (use_graph) as the replay of a HIP graph (the
    descriptor-table copy and the kernel)."""

    def __init__(self, frames_by_size: dict, max_frames: int = 64, use_graph: bool = True, **kw):
        super().__init__(frames_by_size, **kw)
        self.engine = self.fwrs.Engine(max_frames, stream=self.stream, use_graph=use_graph)
        self.max_batch = int(max_frames)
        for (w, h), t in self.tiles.items():
            self.engine.set_tile(w * h, *t)

    def submit(self, batch):
        entries = []
        for (h, i) in batch:
            c, lev, gx, gy = self.frame(h, i)
            entries.append((h[1], c, lev, gx, gy, h[2]))
        self.engine.tick(entries)
        return self._mark()


class PlainExecutor(_GpuExecutor):
    """One launch per frame (fwrs_push_frame_resolve), in submission order on one stream."""

    def submit(self, batch):
        for (h, i) in batch:
            c, lev, gx, gy = self.frame(h, i)
            h[1].step(c, lev, gx, gy, h[2])
        return self._mark()
