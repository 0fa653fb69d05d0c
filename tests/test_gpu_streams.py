"""Work on one context spread over several HIP streams: plain pushes on the context's stream, batched ticks on
an engine's stream, fused foveated pushes against a foveator on a third stream, and a stream change midway.
The library orders these by events; every output and state plane must equal the same sequence run on one
stream, bit for bit."""
from __future__ import annotations

import numpy as np
import pytest
import torch

from paper_2510_03964_amd import fwrs, synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fwrs.load()
    return torch.device("cuda:0")


def _run(dev, spec, frames, full, gaze, streams, use_graph):
    """The sequence: frame t is a plain push (t % 3 == 0), a tick (t % 3 == 1) or a fused foveated push
    (t % 3 == 2); the context moves to `streams['late']` at the midpoint.  Returns the final output and
    state, after every stream has drained."""
    p = fwrs.default_params(spec.width, fovea_radius_px=spec.fovea_radius_px, seed=synth.PHILOX_SEED,
                            stream_id=spec.stream_id)
    res = fwrs.Reservoir(spec.width, spec.height, spec.k, p, stream=streams["ctx"])
    eng = fwrs.Engine(2, stream=streams["engine"], use_graph=use_graph)
    fov = fwrs.Foveator(spec.width, spec.height, spec.fovea_radius_px, spec.ring_radius_px, fwrs.FOV_MIP,
                        stream=streams["fov"])
    col = torch.empty((spec.height, spec.width, 3), device=dev)
    lev = torch.empty((spec.height, spec.width), dtype=torch.uint8, device=dev)
    outs = [torch.zeros((spec.height, spec.width, 3), device=dev) for _ in range(3)]
    torch.cuda.synchronize()
    n = len(frames)
    for t in range(n):
        if t == n // 2:
            res.set_stream(streams["late"])
        o = outs[t % 3]
        if t % 3 == 0:
            res.step(*frames[t], o)
        elif t % 3 == 1:
            eng.tick([(res, *frames[t], o)])
        else:
            gx, gy = float(gaze[t, 0]), float(gaze[t, 1])
            fov.foveate(full, gx, gy, col, lev)            # the foveator's own stream, same level images
            res.step_foveated(fov, full, gx, gy, o)
    last = outs[(n - 1) % 3]
    fov.close()                                            # waits only for the foveator's stream
    eng.close()
    res.sync()
    torch.cuda.synchronize()
    out = last.clone()
    st = res.download()
    res.close()
    return out, st


@pytest.mark.parametrize("use_graph", [False, True])
def test_streams_ordered_by_events(dev, use_graph):
    spec = synth.StreamSpec(320, 192, 4, 24, 20.0, 50.0, 2.0, 6, 4.0, stream_id=9)
    src = synth.FrameSource(spec, device=dev)
    frames = [src.frame(t) for t in range(spec.frames)]
    full = synth.MovingSource(spec, device=dev, n_frames=1).render(0)[0]
    gaze = synth.gaze_trace(spec, spec.frames)
    torch.cuda.synchronize()
    one = torch.cuda.current_stream()
    ref_out, ref_st = _run(dev, spec, frames, full, gaze, {"ctx": one, "engine": one, "fov": one, "late": one},
                           use_graph)
    streams = {name: torch.cuda.Stream() for name in ("ctx", "engine", "fov", "late")}
    out, st = _run(dev, spec, frames, full, gaze, streams, use_graph)
    assert torch.equal(out, ref_out)
    for name in ("wsum", "cnt", "idx"):
        np.testing.assert_array_equal(getattr(st, name), getattr(ref_st, name), err_msg=name)
    for name in ("wt", "col"):
        np.testing.assert_array_equal(getattr(st, name).view(np.uint32), getattr(ref_st, name).view(np.uint32),
                                      err_msg=name)
