"""The serving loop on the GPU: every session's output after the frames it was served equals the
output of the same session run alone with plain launches, bit for bit, in the batched and the
plain executor alike."""
from __future__ import annotations

import pytest
import torch

from paper_2510_03964_amd import fwrs, serve, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fwrs.load()
    return torch.device("cuda:0")


def _rings(dev, sizes, n=8):
    rings = {}
    for (w, h) in sizes:
        spec = synth.StreamSpec(w, h, 4, n, 0.1 * w, 0.25 * w, 2.0, 3, 5.0, stream_id=w)
        src = synth.FrameSource(spec, device=dev)
        rings[(w, h)] = [src.frame(t) for t in range(n)]
    torch.cuda.synchronize()
    return rings


@pytest.mark.parametrize("executor,max_group", [("batched", 1), ("plain", 1), ("batched", 6), ("plain", 6)])
def test_each_session_alone_equals_in_the_mix(dev, executor, max_group):
    """max_group 6 with frame rates above what the loop keeps up with: ticks carry several frames
    of a session (one group in the batched executor), and the outputs are still those of the
    session run alone."""
    sizes = ((128, 64), (96, 48))
    fps = (150.0, 240.0) if max_group == 1 else (20000.0, 30000.0)
    sessions = serve.poisson_sessions(n=6, rate_per_s=20.0, seed=11, lifetime_s=(0.15, 0.4), sizes=sizes,
                                      ks=(2, 3, 4, 8), fps=fps)
    if max_group > 1:
        sessions = [serve.SessionSpec(s.sid, s.arrival_s, s.lifetime_s / 4, s.width, s.height, s.k, s.fps)
                    for s in sessions]
    rings = _rings(dev, sizes)
    stream = torch.cuda.current_stream()
    ex = (serve.BatchedExecutor(rings, max_frames=64, stream=stream) if executor == "batched"
          else serve.PlainExecutor(rings, stream=stream))
    sched = serve.Scheduler(ex, budget_bytes=1 << 30, max_active=8, max_group=max_group)
    st = sched.run(sessions)
    if max_group > 1:
        assert st.max_group > 1, "no tick carried several frames of a session"
    assert st.frames == sum(sched.frames_done.values()) and st.frames > 0
    assert st.latency_ms.size == st.frames
    for s in sessions:
        n = sched.frames_done.get(s.sid, 0)
        assert n > 0
        p = fwrs.default_params(s.width, seed=synth.PHILOX_SEED, stream_id=s.sid)
        alone = fwrs.Reservoir(s.width, s.height, s.k, p, stream=stream)
        out = torch.empty((s.height, s.width, 3), device=dev)
        ring = rings[(s.width, s.height)]
        for i in range(n):
            alone.step(*ring[(i + 7 * s.sid) % len(ring)], out)
        torch.cuda.synchronize()
        assert torch.equal(out, ex.outputs[s.sid]), f"session {s.sid} differs after {n} frames"
        alone.close()


def test_small_budget_queues_sessions_on_the_gpu(dev):
    sizes = ((128, 64),)
    sessions = serve.poisson_sessions(n=5, rate_per_s=50.0, seed=5, lifetime_s=(0.1, 0.2), sizes=sizes, ks=(4,),
                                      fps=(200.0,))
    rings = _rings(dev, sizes)
    ex = serve.BatchedExecutor(rings, max_frames=8)
    one = fwrs.state_bytes(128, 64, 4)
    st = serve.Scheduler(ex, budget_bytes=2 * one, max_active=8).run(sessions)
    assert st.max_active <= 2 and st.max_queue >= 1
    assert st.admitted + st.rejected == len(sessions)


@pytest.mark.parametrize("max_group", [1, 4])
def test_full_size_sessions_alone_equal_in_the_mix(dev, max_group):
    """Sessions of the serving workload's sizes (1080p and 4K, k in {4, 8}) through batched ticks:
    each one's output equals the same session run alone with plain launches.  max_group 4 with frame
    rates above what the GPU serves: the ticks carry groups of a session's overdue frames."""
    sizes = ((1920, 1080), (3840, 2160))
    fps = (90.0, 120.0) if max_group == 1 else (3000.0, 4000.0)
    life = (0.04, 0.08) if max_group == 1 else (0.02, 0.04)
    sessions = serve.poisson_sessions(n=4, rate_per_s=40.0, seed=21, lifetime_s=life, sizes=sizes,
                                      ks=(4, 8), fps=fps)
    rings = _rings(dev, sizes, n=4)
    stream = torch.cuda.current_stream()
    ex = serve.BatchedExecutor(rings, max_frames=8 * max_group, stream=stream)
    sched = serve.Scheduler(ex, budget_bytes=64 * 10**9, max_active=8, max_group=max_group)
    st = sched.run(sessions)
    assert st.frames > 0 and st.admitted == len(sessions)
    if max_group > 1:
        assert st.max_group > 1, "no tick carried several frames of a session"
    for s in sessions:
        n = sched.frames_done.get(s.sid, 0)
        assert n > 0
        p = fwrs.default_params(s.width, seed=synth.PHILOX_SEED, stream_id=s.sid)
        alone = fwrs.Reservoir(s.width, s.height, s.k, p, stream=stream)
        out = torch.empty((s.height, s.width, 3), device=dev)
        ring = rings[(s.width, s.height)]
        for i in range(n):
            alone.step(*ring[(i + 7 * s.sid) % len(ring)], out)
        torch.cuda.synchronize()
        assert torch.equal(out, ex.outputs[s.sid]), f"session {s.sid} differs after {n} frames"
        alone.close()
