"""Parity of the reprojecting pass (moving camera, Sec. 4.3) with the oracle, through the C ABI.

Same bar as the static path: every state plane bit-exact (slot weights, colours, frame indices,
per-pixel counts, weight sums), the resolve within 1e-5 of the oracle's binary64 resolve, and the
flush count equal to the oracle's."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
from paper_2510_03964_amd import fwrs, synth

import edge_colours

pytestmark = pytest.mark.gpu
COLOR_TOL = 1e-5
TOL = 0.1


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fwrs.load()
    return torch.device("cuda:0")


def _params(spec, bias):
    p = fwrs.default_params(spec.width, fovea_radius_px=spec.fovea_radius_px, seed=synth.PHILOX_SEED,
                            stream_id=spec.stream_id, bias_mode=bias, flags=fwrs.FLAG_REPROJECT)
    q = oracle.default_params(spec.width, fovea_radius_px=spec.fovea_radius_px, seed=synth.PHILOX_SEED,
                              stream_id=spec.stream_id, bias_mode=bias)
    return p, q


def _compare(res, orc, out, where):
    st, so = res.download(), orc.state()
    for name in ("cnt", "idx"):
        np.testing.assert_array_equal(getattr(st, name), getattr(so, name), err_msg=f"{name} {where}")
    for name in ("wsum", "wt", "col", "wslot"):
        np.testing.assert_array_equal(getattr(st, name).view(np.uint32), getattr(so, name).view(np.uint32),
                                      err_msg=f"{name} {where}")
    if out is not None:
        err = np.abs(out.cpu().numpy().astype(np.float64) - orc.resolve()).max()
        assert err <= COLOR_TOL, f"resolve differs by {err} {where}"
    assert res.flushes() == orc.flushes, where


def _run(dev, spec, n, bias=fwrs.BIAS_BERNOULLI, frames=None, every=1, tile=None, resolve=True):
    p, q = _params(spec, bias)
    res = fwrs.Reservoir(spec.width, spec.height, spec.k, p, stream=torch.cuda.current_stream())
    if tile:
        res.set_tile(*tile)
    orc = oracle.Oracle(spec.width, spec.height, spec.k, q)
    out = torch.full((spec.height, spec.width, 3), -1.0, device=dev) if resolve else None
    src = None if frames is not None else synth.MovingSource(spec, device=dev, n_frames=n)
    for t in range(n):
        c, lev, mv, d, gx, gy = frames[t] if frames is not None else src.frame(t)
        res.step_reproject(c, lev, mv, d, gx, gy, TOL, out)
        orc.push_reproject(c.cpu().numpy(), lev.cpu().numpy(), mv.cpu().numpy(), d.cpu().numpy(), gx, gy, TOL)
        if (t + 1) % every == 0 or t == n - 1:
            res.sync()
            _compare(res, orc, out, f"frame {t} {spec.width}x{spec.height} k={spec.k} bias={bias}")
    assert res.frame_index == n
    return res, orc, out


@pytest.mark.parametrize("bias", [fwrs.BIAS_BERNOULLI, fwrs.BIAS_NONE, fwrs.BIAS_FULL, fwrs.AES,
                                  fwrs.BIAS_MEMORYLESS])
def test_moving_workload_every_frame(dev, bias):
    """Panning camera and a moving occluder: 192x108, k = 4, 16 frames, every frame compared."""
    spec = synth.StreamSpec(192, 108, 4, 16, 9.6, 24.0, 1.0, 6, 3.0, stream_id=3)
    res, orc, _ = _run(dev, spec, 16, bias=bias)
    assert orc.flushes > spec.pixels          # the disc's edges flushed after the first frame
    v = res.state_view()
    assert v.cnt and v.depth


@pytest.mark.parametrize("w,h,k,frames", [
    (1, 1, 1, 3), (3, 2, 16, 3), (13, 7, 3, 4), (100, 37, 5, 4), (64, 64, 8, 4), (255, 3, 2, 3), (96, 40, 1, 3),
])
@pytest.mark.parametrize("bias", [fwrs.BIAS_BERNOULLI, fwrs.BIAS_FULL, fwrs.AES])
def test_sizes_and_slot_counts(dev, w, h, k, frames, bias):
    spec = synth.StreamSpec(w, h, k, frames, max(1.0, 0.1 * w), max(2.5, 0.25 * w), 0.2 * w + 0.5, 2,
                            0.3 * w + 1, stream_id=k)
    _run(dev, spec, frames, bias=bias)


@pytest.mark.parametrize("tile", [(8, 8), (16, 16), (256, 1)])
def test_tile_shape_never_changes_results(dev, tile):
    spec = synth.StreamSpec(160, 90, 4, 5, 8.0, 20.0, 1.0, 3, 3.0)
    _run(dev, spec, 5, tile=tile)


def _still_frames(dev, spec, n, motions):
    """A static-scene sequence with given per-frame constant motion vectors (None: zero)."""
    src = synth.FrameSource(spec, device=dev, n_frames=n)
    out = []
    for t in range(n):
        c, lev, gx, gy = src.frame(t)
        mv = torch.zeros((spec.height, spec.width, 2), device=dev)
        if motions[t] is not None:
            mv[..., 0], mv[..., 1] = motions[t]
        out.append((c, lev, mv.contiguous(), torch.full((spec.height, spec.width), 5.0, device=dev), gx, gy))
    return out


def test_integer_subpixel_and_invalid_motion(dev):
    spec = synth.StreamSpec(120, 70, 4, 9, 8.0, 20.0, 1.0, 3, 3.0)
    motions = [None, None, (3.0, -2.0), (0.5, 0.0), (0.5 + 2 ** -10, 0.0), (-0.5, 0.0), (float("nan"), 0.0),
               None, (1e30, 1e30)]
    _run(dev, spec, 9, frames=_still_frames(dev, spec, 9, motions))


@pytest.mark.parametrize("k", [4, 8, 3])
def test_eq7_repeated_and_edge_colours(dev, k):
    """Eq. 7 through the reprojecting pass with a still camera, on colours that repeat across frames
    and edge values (signed zeros, a denormal, 2^24 and its neighbour below, +-3e7, +-1e30 whose Lab
    is not finite); a sub-pixel pan on frame 4 moves every sample.  State planes bit-exact each
    frame (the resolve of such colours is compared by the plain-pass test)."""
    w, h, n = 96, 40, 8
    still = edge_colours.palette_frames(w, h, n, dev, seed=20 + k)
    frames = []
    for t, (c, lev, gx, gy) in enumerate(still):
        mv = torch.zeros((h, w, 2), device=dev)
        if t == 4:
            mv[..., 0] = 0.5
        frames.append((c, lev, mv.contiguous(), torch.full((h, w), 5.0, device=dev), gx, gy))
    spec = synth.StreamSpec(w, h, k, n, 8.0, 20.0, 1.0, 2, 3.0, stream_id=k)
    _run(dev, spec, n, bias=fwrs.BIAS_FULL, frames=frames, resolve=False)


def test_update_only_then_resolve(dev):
    spec = synth.StreamSpec(128, 72, 4, 6, 8.0, 20.0, 1.0, 3, 3.0)
    src = synth.MovingSource(spec, device=dev, n_frames=6)
    frames = [src.frame(t) for t in range(6)]
    res_a, _, out_a = _run(dev, spec, 6, frames=frames, every=6)
    res_b, orc_b, _ = _run(dev, spec, 6, frames=frames, every=6, resolve=False)
    out_b = torch.empty_like(out_a)
    res_b.resolve(out_b)
    res_b.sync()
    assert torch.equal(out_a, out_b)


def test_reset_flushes_the_next_frame(dev):
    spec = synth.StreamSpec(96, 64, 4, 6, 8.0, 20.0, 1.0, 3, 3.0)
    src = synth.MovingSource(spec, device=dev, n_frames=6)
    p, q = _params(spec, fwrs.BIAS_BERNOULLI)
    res = fwrs.Reservoir(spec.width, spec.height, spec.k, p, stream=torch.cuda.current_stream())
    out = torch.empty((spec.height, spec.width, 3), device=dev)
    for t in range(3):
        res.step_reproject(*src.frame(t), TOL, out)
    res.reset()
    assert res.frame_index == 0 and res.flushes() == 0
    orc = oracle.Oracle(spec.width, spec.height, spec.k, q)
    for t in range(3, 6):
        c, lev, mv, d, gx, gy = src.frame(t)
        res.step_reproject(c, lev, mv, d, gx, gy, TOL, out)
        orc.push_reproject(c.cpu().numpy(), lev.cpu().numpy(), mv.cpu().numpy(), d.cpu().numpy(), gx, gy, TOL)
    res.sync()
    _compare(res, orc, out, "after reset")


@pytest.mark.parametrize("bias", [fwrs.BIAS_FULL, fwrs.AES])
def test_caller_arena(dev, bias):
    """A caller arena full of garbage is cleared to the empty state (A-ES keys to -infinity)."""
    spec = synth.StreamSpec(96, 64, 8, 4, 8.0, 20.0, 1.0, 3, 3.0)
    p, q = _params(spec, bias)
    need = fwrs.state_bytes(spec.width, spec.height, spec.k, p)
    with pytest.raises(fwrs.FwrsError):
        fwrs.Reservoir(spec.width, spec.height, spec.k, p, stream=torch.cuda.current_stream(),
                       arena=torch.empty(need - 256, dtype=torch.uint8, device=dev))
    arena = torch.full((need,), 0x5A, dtype=torch.uint8, device=dev)
    res = fwrs.Reservoir(spec.width, spec.height, spec.k, p, stream=torch.cuda.current_stream(), arena=arena)
    orc = oracle.Oracle(spec.width, spec.height, spec.k, q)
    src = synth.MovingSource(spec, device=dev, n_frames=4)
    out = torch.empty((spec.height, spec.width, 3), device=dev)
    for t in range(4):
        c, lev, mv, d, gx, gy = src.frame(t)
        res.step_reproject(c, lev, mv, d, gx, gy, TOL, out)
        orc.push_reproject(c.cpu().numpy(), lev.cpu().numpy(), mv.cpu().numpy(), d.cpu().numpy(), gx, gy, TOL)
    res.sync()
    _compare(res, orc, out, "caller arena")


def test_entry_points_check_the_context_kind(dev):
    spec = synth.StreamSpec(64, 32, 4, 2, 8.0, 20.0, 1.0, 3, 3.0)
    src = synth.MovingSource(spec, device=dev, n_frames=2)
    c, lev, mv, d, gx, gy = src.frame(0)
    out = torch.empty((spec.height, spec.width, 3), device=dev)
    plain = fwrs.Reservoir(spec.width, spec.height, spec.k, stream=torch.cuda.current_stream())
    with pytest.raises(fwrs.FwrsError) as e:
        plain.step_reproject(c, lev, mv, d, gx, gy, TOL, out)
    assert e.value.status == fwrs.E_STATE
    p, _ = _params(spec, fwrs.BIAS_BERNOULLI)
    rep = fwrs.Reservoir(spec.width, spec.height, spec.k, p, stream=torch.cuda.current_stream())
    for call in (lambda: rep.step(c, lev, gx, gy, out), lambda: rep.push(c, lev, gx, gy)):
        with pytest.raises(fwrs.FwrsError) as e:
            call()
        assert e.value.status == fwrs.E_STATE
    eng = fwrs.Engine(2, stream=torch.cuda.current_stream())
    with pytest.raises(fwrs.FwrsError) as e:
        eng.tick([(rep, c, lev, gx, gy, out)])
    assert e.value.status == fwrs.E_STATE
    eng.close()
    with pytest.raises(fwrs.FwrsError) as e:
        rep.step_reproject(c, lev, mv, d, gx, gy, -1.0, out)
    assert e.value.status == fwrs.E_ARG
    buf = torch.empty(spec.pixels * 2 + 1, device=dev)
    with pytest.raises(fwrs.FwrsError) as e:                     # motion not 8-byte aligned
        rep.step_reproject(c, lev, buf[1:].view(spec.height, spec.width, 2), d, gx, gy, TOL, out)
    assert e.value.status == fwrs.E_ARG
    assert rep.frame_index == 0
    rep.step_reproject(c, lev, mv, d, gx, gy, TOL, out)
    assert rep.frame_index == 1


def test_4k_moving_frames(dev):
    """3840x2160, k = 4, the benchmarked launch configuration: three frames of the moving
    workload, every state plane compared over the whole image."""
    spec = synth.spec_4k()
    _run(dev, spec, 3, every=3)
