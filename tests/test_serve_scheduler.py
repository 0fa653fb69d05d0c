"""Serving scheduler logic on the CPU: a fake executor with a serial cost model and a virtual
clock stand in for the GPU (admission, budget, queueing, batching, latency accounting)."""
from __future__ import annotations

import math

import numpy as np
import pytest

from paper_2510_03964_amd import serve


class VirtualClock:
    """Advances by `step` on every read (the loop's own overhead) and on sleep()."""

    def __init__(self, step=20e-6):
        self.t = 0.0
        self.step = step

    def __call__(self):
        self.t += self.step
        return self.t

    def sleep(self, dt):
        self.t += dt


class FakeExecutor:
    """A serial device: a tick starts when the previous one ends and costs a fixed time per pixel."""

    def __init__(self, clock, s_per_pixel=1e-11, launch_s=5e-6):
        self.clock = clock
        self.s_per_pixel = s_per_pixel
        self.launch_s = launch_s
        self.busy_until = 0.0
        self.ticks = []            # (tick, done time)
        self.log = []              # (tick, [(sid, frame)])
        self.open_sids = set()
        self.max_open = 0
        self.open_bytes = 0
        self.max_open_bytes = 0

    def state_bytes(self, spec):
        return spec.pixels * (4 + 20 * spec.k)

    def open(self, spec):
        self.open_sids.add(spec.sid)
        self.max_open = max(self.max_open, len(self.open_sids))
        self.open_bytes += self.state_bytes(spec)
        self.max_open_bytes = max(self.max_open_bytes, self.open_bytes)
        return spec

    def close(self, h):
        self.open_sids.discard(h.sid)
        self.open_bytes -= self.state_bytes(h)

    def submit(self, batch):
        now = self.clock.t
        start = max(now, self.busy_until)
        cost = self.launch_s + sum(h.pixels for h, _ in batch) * self.s_per_pixel
        self.busy_until = start + cost
        tick = len(self.log)
        self.ticks.append((tick, self.busy_until))
        self.log.append((tick, [(h.sid, i) for h, i in batch]))
        return tick

    def poll(self):
        out = [(t, d) for (t, d) in self.ticks if d <= self.clock.t]
        self.ticks = [(t, d) for (t, d) in self.ticks if d > self.clock.t]
        return out

    def drain(self):
        out = list(self.ticks)
        self.clock.t = max([self.clock.t] + [d for _, d in out])
        self.ticks = []
        return out


def _small_mix(n=8, scale=0.05):
    return serve.poisson_sessions(n=n, rate_per_s=1.0, seed=7, time_scale=scale, sizes=((64, 32), (128, 64)))


def _run(sessions, budget, s_per_pixel=1e-11, max_active=64):
    clk = VirtualClock()
    ex = FakeExecutor(clk, s_per_pixel)
    st = serve.Scheduler(ex, budget, max_active=max_active, clock=clk, sleep=clk.sleep).run(sessions)
    return st, ex


def test_every_due_frame_is_processed_once_in_order():
    sessions = _small_mix()
    st, ex = _run(sessions, budget=1 << 40)
    seen = {}
    for tick, frames in ex.log:
        sids = [sid for sid, _ in frames]
        assert len(sids) == len(set(sids)), "one frame per session per tick"
        for sid, i in frames:
            assert seen.get(sid, -1) == i - 1, "frames of a session in order, none skipped"
            seen[sid] = i
    for s in sessions:
        expected = math.ceil(s.lifetime_s * s.fps - 1e-9)
        assert abs((seen[s.sid] + 1) - expected) <= 1
    assert st.frames == sum(len(f) for _, f in ex.log)
    assert st.admitted == len(sessions) and st.rejected == 0


def test_latency_is_completion_minus_due_and_meets_deadline_when_fast():
    st, _ = _run(_small_mix(), budget=1 << 40, s_per_pixel=1e-12)
    assert st.latency_ms.size == st.frames and np.all(st.latency_ms >= 0.0)
    summ = st.summary()
    assert summ["latency_ms_p99"] < serve.DEADLINE_MS
    assert summ["deadline_misses"] == 0


def test_overload_shows_up_as_deadline_misses():
    st, _ = _run(_small_mix(), budget=1 << 40, s_per_pixel=2e-6)
    assert st.deadline_misses > 0
    assert st.summary()["latency_ms_p99"] > serve.DEADLINE_MS


def test_budget_queues_sessions_and_bounds_resident_memory():
    sessions = _small_mix(n=10, scale=0.02)
    per = max(s.pixels * (4 + 20 * s.k) for s in sessions)
    budget = 2 * per
    st, ex = _run(sessions, budget=budget)
    assert ex.max_open_bytes <= budget
    assert ex.open_bytes == 0, "every session released its memory"
    assert st.max_queue >= 1
    assert max(st.queue_wait_s) > 0.0
    assert st.admitted + st.rejected == len(sessions)


def test_max_active_slots_bound_concurrency():
    st, ex = _run(_small_mix(n=10, scale=0.05), budget=1 << 40, max_active=3)
    assert ex.max_open <= 3 and st.max_active <= 3


def test_session_that_can_never_fit_is_refused():
    sessions = _small_mix(n=2)
    with pytest.raises(ValueError):
        _run(sessions, budget=16)


def test_poisson_sessions_follow_the_recipe():
    s = serve.poisson_sessions(n=2000, rate_per_s=1.0, seed=3)
    gaps = np.diff([0.0] + [x.arrival_s for x in s])
    assert abs(gaps.mean() - 1.0) < 0.08
    life = np.array([x.lifetime_s for x in s])
    assert life.min() >= 10.0 and life.max() <= 60.0 and abs(life.mean() - 35.0) < 1.5
    assert {(x.width, x.height) for x in s} == {(1920, 1080), (3840, 2160)}
    assert {x.k for x in s} == {4, 8} and {x.fps for x in s} == {72.0, 90.0, 120.0}
    t = serve.poisson_sessions(n=5, seed=3, time_scale=0.25)
    u = serve.poisson_sessions(n=5, seed=3)
    assert all(abs(a.arrival_s - 0.25 * b.arrival_s) < 1e-12 for a, b in zip(t, u))


def test_batches_grow_when_the_device_is_busy():
    """Back-pressure: with at most two ticks in flight, frames that come due while the device is
    busy are submitted together."""
    light, _ = _run(_small_mix(), budget=1 << 40, s_per_pixel=1e-12)
    heavy, _ = _run(_small_mix(), budget=1 << 40, s_per_pixel=1e-6)
    assert heavy.frames / heavy.ticks > light.frames / light.ticks
    assert heavy.max_batch > 1


def test_ticks_never_exceed_the_executors_batch_limit():
    """An executor that takes at most `max_batch` frames per submit: the rest of the due frames go into the
    next tick, and every frame is still processed once, in order."""
    sessions = _small_mix(n=12, scale=0.02)
    clk = VirtualClock()
    uncapped = FakeExecutor(clk, 1e-6)                       # a busy device: batches grow past the limit
    serve.Scheduler(uncapped, 1 << 40, max_active=12, clock=clk, sleep=clk.sleep).run(sessions)
    assert max(len(f) for _, f in uncapped.log) > 3
    clk = VirtualClock()
    ex = FakeExecutor(clk, 1e-6)
    ex.max_batch = 3
    st = serve.Scheduler(ex, 1 << 40, max_active=12, clock=clk, sleep=clk.sleep).run(sessions)
    assert max(len(f) for _, f in ex.log) <= 3
    assert st.max_batch <= 3
    seen = {}
    for _, frames in ex.log:
        for sid, i in frames:
            assert seen.get(sid, -1) == i - 1
            seen[sid] = i
    assert st.frames == sum(len(f) for _, f in ex.log) and st.admitted == len(sessions)


def _check_order(log, max_group):
    """Every session's frames once, in order; in a tick a session's frames are consecutive and at
    most max_group of them."""
    seen = {}
    most = 0
    for _, frames in log:
        per = {}
        for sid, i in frames:
            assert seen.get(sid, -1) == i - 1, "frames of a session in order, none skipped"
            seen[sid] = i
            per[sid] = per.get(sid, 0) + 1
        most = max([most] + list(per.values()))
        assert all(v <= max_group for v in per.values())
    return seen, most


def test_groups_take_a_sessions_due_frames_together():
    """max_group > 1: when the device falls behind, a tick takes up to max_group of a session's due
    frames (consecutive, oldest first), and still every frame once, in order."""
    sessions = _small_mix(n=8, scale=0.05)
    clk = VirtualClock()
    ex = FakeExecutor(clk, 2e-6)
    st = serve.Scheduler(ex, 1 << 40, max_active=8, max_group=4, clock=clk, sleep=clk.sleep).run(sessions)
    _, most = _check_order(ex.log, 4)
    assert most == 4, "a busy device makes sessions fall behind: groups fill up"
    assert st.frames == sum(len(f) for _, f in ex.log) and st.admitted == len(sessions)
    # the same sessions on a fast device: no frame waits, so no groups form
    clk = VirtualClock()
    fast = FakeExecutor(clk, 1e-13)
    serve.Scheduler(fast, 1 << 40, max_active=8, max_group=4, clock=clk, sleep=clk.sleep).run(sessions)
    assert _check_order(fast.log, 4)[1] == 1


def test_groups_respect_the_executors_batch_limit():
    sessions = _small_mix(n=12, scale=0.02)
    clk = VirtualClock()
    ex = FakeExecutor(clk, 1e-6)
    ex.max_batch = 5
    st = serve.Scheduler(ex, 1 << 40, max_active=12, max_group=3, clock=clk, sleep=clk.sleep).run(sessions)
    assert max(len(f) for _, f in ex.log) <= 5 and st.max_batch <= 5
    _check_order(ex.log, 3)
    assert st.frames == sum(len(f) for _, f in ex.log) and st.admitted == len(sessions)
    with pytest.raises(ValueError):
        serve.Scheduler(ex, 1 << 40, max_group=0)
