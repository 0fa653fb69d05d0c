"""Parity of the HIP path (through the C ABI) with the CPU oracle, element by element.

Bar: slot frame indices, counts, weights, weight sums and kept colours are
bit-exact (they are decided or copied values); the resolved colour is within
1e-5 of the oracle's binary64 resolve (a binary32 weighted mean of at most 16
values in [0, 1] rounds to within a few 1e-7).
"""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
from paper_2510_03964_amd import fwrs, synth

import edge_colours

pytestmark = pytest.mark.gpu
COLOR_TOL = 1e-5


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fwrs.load()
    return torch.device("cuda:0")


def _params(spec, bias=fwrs.BIAS_BERNOULLI, seed=synth.PHILOX_SEED):
    p = fwrs.default_params(spec.width, fovea_radius_px=spec.fovea_radius_px, seed=seed,
                            stream_id=spec.stream_id, bias_mode=bias)
    q = oracle.default_params(spec.width, fovea_radius_px=spec.fovea_radius_px, seed=seed,
                              stream_id=spec.stream_id, bias_mode=bias)
    return p, q


def _compare_state(st, so, where=""):
    np.testing.assert_array_equal(st.cnt, so.cnt, err_msg=f"cnt {where}")
    np.testing.assert_array_equal(st.idx, so.idx, err_msg=f"idx {where}")
    np.testing.assert_array_equal(st.wsum.view(np.uint32), so.wsum.view(np.uint32), err_msg=f"wsum {where}")
    np.testing.assert_array_equal(st.wt.view(np.uint32), so.wt.view(np.uint32), err_msg=f"wt {where}")
    np.testing.assert_array_equal(st.col.view(np.uint32), so.col.view(np.uint32), err_msg=f"col {where}")
    np.testing.assert_array_equal(st.wslot.view(np.uint32), so.wslot.view(np.uint32), err_msg=f"wslot {where}")


def _compare_out(out, ref, where=""):
    err = np.abs(out.astype(np.float64) - ref).max() if out.size else 0.0
    assert err <= COLOR_TOL, f"resolve differs by {err} {where}"
    return err


def _keeps_plane(bias):
    return bias in (fwrs.BIAS_NONE, fwrs.BIAS_BERNOULLI, fwrs.BIAS_MEMORYLESS)


def _run_pair(dev, spec, n_frames, mode="fused", tile=None, bias=fwrs.BIAS_BERNOULLI, every=1, src=None,
              res_from=None):
    """mode: "fused" (push + resolve in one call), "split" (push, then resolve) or
    "incremental" (first frame fused, then only the changed pixels are rewritten).
    res_from: the frame from which fused passes use the resolve plane (None: the library's default)."""
    p, q = _params(spec, bias)
    src = src or synth.FrameSource(spec, device=dev, n_frames=n_frames)
    res = fwrs.Reservoir(spec.width, spec.height, spec.k, p, stream=torch.cuda.current_stream())
    if tile is not None:
        res.set_tile(*tile)
    if res_from is not None and _keeps_plane(bias):
        res.set_resolve_plane_from(res_from)
    orc = oracle.Oracle(spec.width, spec.height, spec.k, q)
    out = torch.full((spec.height, spec.width, 3), -1.0, dtype=torch.float32, device=dev)
    for t in range(n_frames):
        c, lev, gx, gy = src.frame(t)
        if mode == "fused" or (mode == "incremental" and t == 0):
            res.step(c, lev, gx, gy, out)
        elif mode == "incremental":
            res.step_incremental(c, lev, gx, gy, out)
        else:
            res.push(c, lev, gx, gy)
            res.resolve(out)
        orc.push(c.cpu().numpy(), lev.cpu().numpy(), gx, gy)
        if (t + 1) % every == 0 or t == n_frames - 1:
            res.sync()
            _compare_state(res.download(), orc.state(), f"frame {t} {spec.width}x{spec.height} k={spec.k}")
            _compare_out(out.cpu().numpy(), orc.resolve(), f"frame {t}")
    assert res.frame_index == n_frames
    return res, orc, out


@pytest.mark.parametrize("res_from", [None, 0, 1, 30])
def test_small_workload_every_frame(dev, res_from):
    """256x256, k = 4, 60 frames of the synthetic gaze trace, fused update + resolve; the resolve
    plane used from the library's default frame, from the first, second and thirtieth frame."""
    spec = synth.spec_small()
    res, orc, _ = _run_pair(dev, spec, spec.frames, res_from=res_from)
    takes, changed, updates = res.stats()
    assert updates == spec.frames * spec.pixels
    assert 0 < changed <= takes


def test_push_then_resolve_is_bit_identical_to_fused(dev):
    spec = synth.spec_small()
    _, _, out_a = _run_pair(dev, spec, 12, mode="fused", every=12)
    _, _, out_b = _run_pair(dev, spec, 12, mode="split", every=12)
    assert torch.equal(out_a, out_b)


@pytest.mark.parametrize("k", [4, 1, 3, 8])
def test_incremental_resolve_matches_oracle_and_full_resolve(dev, k):
    """Writing only the changed pixels leaves out bit-identical to the full resolve."""
    spec = synth.StreamSpec(256, 256, k, 30, 32.0, 80.0, 2.0, 10, 6.0)
    _, _, out_inc = _run_pair(dev, spec, 30, mode="incremental", every=3)
    _, _, out_full = _run_pair(dev, spec, 30, mode="fused", every=30)
    assert torch.equal(out_inc, out_full)


def test_incremental_resolve_checks_its_precondition(dev):
    spec = synth.StreamSpec(64, 32, 4, 4, 8.0, 20.0, 2.0, 2, 5.0)
    src = synth.FrameSource(spec, device=dev)
    res = fwrs.Reservoir(spec.width, spec.height, spec.k, stream=torch.cuda.current_stream())
    out = torch.empty((spec.height, spec.width, 3), device=dev)
    other = torch.empty_like(out)
    with pytest.raises(fwrs.FwrsError) as e:          # nothing resolved yet
        res.step_incremental(*src.frame(0), out)
    assert e.value.status == fwrs.E_STATE
    res.step(*src.frame(0), out)
    with pytest.raises(fwrs.FwrsError):               # a different buffer
        res.step_incremental(*src.frame(1), other)
    res.step_incremental(*src.frame(1), out)
    res.push(*src.frame(2))
    with pytest.raises(fwrs.FwrsError):               # an update without resolve since
        res.step_incremental(*src.frame(3), out)
    res.resolve(out)
    res.step_incremental(*src.frame(3), out)
    res.reset()
    with pytest.raises(fwrs.FwrsError):
        res.step_incremental(*src.frame(0), out)
    assert res.frame_index == 0


@pytest.mark.parametrize("w,h,k,frames", [
    (1, 1, 1, 5), (3, 2, 16, 4), (13, 7, 3, 6), (100, 37, 5, 4), (64, 64, 8, 5), (255, 3, 2, 5),
    (96, 40, 7, 4), (128, 33, 12, 3), (1367, 769, 4, 3),
])
@pytest.mark.parametrize("res_from", [None, 1])
def test_sizes_and_slot_counts(dev, w, h, k, frames, res_from):
    """Ragged widths (scalar path), every specialised and generic slot count, tiny images; from
    frame 1 on, unchanged pixels through the resolve plane."""
    spec = synth.StreamSpec(w, h, k, frames, max(1.0, 0.1 * w), max(2.5, 0.25 * w), 0.2 * w + 0.5, 2, 0.3 * w + 1,
                            stream_id=k)
    _run_pair(dev, spec, frames, res_from=res_from)


@pytest.mark.parametrize("tile", [(8, 8), (16, 16), (32, 8), (64, 4), (256, 1), (16, 4), (8, 16), (128, 2)])
def test_tile_shape_never_changes_results(dev, tile):
    spec = synth.StreamSpec(200, 120, 4, 5, 20.0, 50.0, 3.0, 2, 9.0)
    _run_pair(dev, spec, 5, tile=tile, res_from=2)


@pytest.mark.parametrize("res_from", [None, 1])
def test_bias_none_mode(dev, res_from):
    spec = synth.StreamSpec(160, 96, 4, 8, 16.0, 40.0, 3.0, 3, 8.0)
    _run_pair(dev, spec, 8, bias=fwrs.BIAS_NONE, res_from=res_from)


def _plane(res, arena):
    """The resolve plane as a host array [H, W, 3] (read from the caller arena at the offset the
    state view reports), or None while the context reports it stale."""
    v = res.state_view()
    if not v.res:
        return None
    off = v.res - arena.data_ptr()
    assert off == 4 * v.pitch * (1 + 5 * res.k)          # after w_sum, the records and the indices
    n = res.height * res.width * 3
    return arena[off:off + 4 * n].view(torch.float32).view(res.height, res.width, 3).cpu().numpy()


@pytest.mark.parametrize("k", [4, 3])
def test_resolve_plane_across_entry_points(dev, k):
    """Every entry point that changes a context keeps its resolve plane current or marks it stale,
    so a fused pass after any sequence of calls equals the oracle: fused frames from the plane,
    an update without resolve (plane stale), an incremental frame (stale), a resolve-only call,
    a reset, and the plane rebuilt by the frame before the next cached one."""
    spec = synth.StreamSpec(160, 96, k, 16, 16.0, 40.0, 3.0, 4, 8.0)
    p, q = _params(spec)
    src = synth.FrameSource(spec, device=dev, n_frames=16)
    arena = torch.empty(fwrs.state_bytes(spec.width, spec.height, spec.k, p), dtype=torch.uint8, device=dev)
    res = fwrs.Reservoir(spec.width, spec.height, spec.k, p, stream=torch.cuda.current_stream(), arena=arena)
    res.set_resolve_plane_from(1)
    orc = oracle.Oracle(spec.width, spec.height, spec.k, q)
    out = torch.full((spec.height, spec.width, 3), -1.0, device=dev)
    script = ["fused", "fused", "fused", "push", "fused", "fused", "incremental", "fused", "fused", "resolve",
              "fused", "reset", "fused", "fused", "push", "resolve", "fused"]
    t = 0
    for op in script:
        if op == "reset":
            res.reset()
            orc.close()
            orc = oracle.Oracle(spec.width, spec.height, spec.k, q)
            t = 0
            continue
        if op == "resolve":
            res.resolve(out)
        else:
            c, lev, gx, gy = src.frame(t)
            if op == "fused":
                res.step(c, lev, gx, gy, out)
            elif op == "incremental":
                res.step_incremental(c, lev, gx, gy, out)
            else:
                res.push(c, lev, gx, gy)
            orc.push(c.cpu().numpy(), lev.cpu().numpy(), gx, gy)
            t += 1
        res.sync()
        _compare_state(res.download(), orc.state(), f"after {op} at frame {t}")
        if op != "push":
            o = out.cpu().numpy()
            _compare_out(o, orc.resolve(), f"after {op} at frame {t}")
            plane = _plane(res, arena)
            if op == "fused" and t >= 2:
                assert plane is not None, f"plane stale after a fused frame at {t}"
            if plane is not None:
                assert np.array_equal(plane.view(np.uint32), o.view(np.uint32)), f"plane != resolve after {op}"
        else:
            assert _plane(res, arena) is None


def test_no_resolve_plane_flag_gives_identical_results(dev):
    spec = synth.StreamSpec(200, 120, 4, 12, 20.0, 50.0, 3.0, 4, 9.0)
    outs = []
    for flags in (0, fwrs.FLAG_NO_RESOLVE_PLANE):
        p, _ = _params(spec)
        p.flags = flags
        src = synth.FrameSource(spec, device=dev, n_frames=12)
        res = fwrs.Reservoir(spec.width, spec.height, spec.k, p, stream=torch.cuda.current_stream())
        if flags:
            with pytest.raises(fwrs.FwrsError):
                res.set_resolve_plane_from(0)
        else:
            res.set_resolve_plane_from(0)
        out = torch.empty((spec.height, spec.width, 3), device=dev)
        seq = []
        for t in range(12):
            res.step(*src.frame(t), out)
            seq.append(out.clone())
        res.sync()
        outs.append((seq, res.download()))
    for a, b in zip(outs[0][0], outs[1][0]):
        assert torch.equal(a, b)
    np.testing.assert_array_equal(outs[0][1].idx, outs[1][1].idx)


def test_unaligned_buffers_take_the_scalar_path(dev):
    """Colour and output views starting 4 bytes into their allocations: same results."""
    spec = synth.StreamSpec(64, 32, 4, 5, 8.0, 20.0, 2.0, 2, 5.0)
    src = synth.FrameSource(spec, device=dev)
    p, q = _params(spec)
    res = fwrs.Reservoir(spec.width, spec.height, spec.k, p, stream=torch.cuda.current_stream())
    orc = oracle.Oracle(spec.width, spec.height, spec.k, q)
    n = spec.pixels * 3
    cbuf = torch.empty(n + 1, dtype=torch.float32, device=dev)
    obuf = torch.empty(n + 1, dtype=torch.float32, device=dev)
    out = obuf[1:].view(spec.height, spec.width, 3)
    for t in range(5):
        c, lev, gx, gy = src.frame(t)
        cbuf[1:].copy_(c.reshape(-1))
        res.step(cbuf[1:].view(spec.height, spec.width, 3), lev, gx, gy, out)
        orc.push(c.cpu().numpy(), lev.cpu().numpy(), gx, gy)
    res.sync()
    _compare_state(res.download(), orc.state())
    _compare_out(out.cpu().numpy(), orc.resolve())


def test_resolve_before_any_frame_is_zero(dev):
    res = fwrs.Reservoir(40, 20, 4, stream=torch.cuda.current_stream())
    out = torch.full((20, 40, 3), 7.0, device=dev)
    res.resolve(out)
    res.sync()
    assert torch.count_nonzero(out).item() == 0
    st = res.download()
    assert np.all(st.idx == 0xFFFFFFFF) and np.all(st.cnt == 0)


def test_reset_and_caller_arena(dev):
    spec = synth.StreamSpec(128, 64, 4, 4, 12.0, 30.0, 2.0, 2, 6.0)
    p, q = _params(spec)
    arena = torch.empty(fwrs.state_bytes(spec.width, spec.height, spec.k), dtype=torch.uint8, device=dev)
    res = fwrs.Reservoir(spec.width, spec.height, spec.k, p, stream=torch.cuda.current_stream(), arena=arena)
    src = synth.FrameSource(spec, device=dev)
    out = torch.empty((spec.height, spec.width, 3), device=dev)
    for t in range(3):
        res.step(*src.frame(t), out)
    res.reset()
    assert res.frame_index == 0
    orc = oracle.Oracle(spec.width, spec.height, spec.k, q)
    for t in range(4):
        c, lev, gx, gy = src.frame(t)
        res.step(c, lev, gx, gy, out)
        orc.push(c.cpu().numpy(), lev.cpu().numpy(), gx, gy)
    res.sync()
    _compare_state(res.download(), orc.state())
    _compare_out(out.cpu().numpy(), orc.resolve())
    assert res.stats()[2] == 4 * spec.pixels


def test_stats_count_every_slot_replacement(dev):
    spec = synth.StreamSpec(96, 64, 4, 10, 10.0, 25.0, 2.0, 3, 6.0)
    p, q = _params(spec)
    src = synth.FrameSource(spec, device=dev)
    res = fwrs.Reservoir(spec.width, spec.height, spec.k, p, stream=torch.cuda.current_stream())
    orc = oracle.Oracle(spec.width, spec.height, spec.k, q)
    out = torch.empty((spec.height, spec.width, 3), device=dev)
    expected = changed_px = 0
    for t in range(spec.frames):
        c, lev, gx, gy = src.frame(t)
        res.step(c, lev, gx, gy, out)
        orc.push(c.cpu().numpy(), lev.cpu().numpy(), gx, gy)
        now = orc.state().idx == t
        expected += int(np.count_nonzero(now))
        changed_px += int(np.count_nonzero(now.any(axis=0)))
    takes, changed, updates = res.stats()
    assert takes == expected
    assert changed == changed_px
    assert updates == spec.frames * spec.pixels


@pytest.mark.parametrize("bias", [fwrs.BIAS_BERNOULLI, fwrs.BIAS_FULL, fwrs.AES, fwrs.BIAS_MEMORYLESS,
                                  fwrs.BIAS_NONE])
def test_4k_bands_and_whole_frame_properties(dev, bias):
    """3840x2160, k = 4, in the launch configuration the benchmark times: bands of rows
    (through the gaze, the periphery and the image edges) against the oracle every few frames,
    and properties that hold at any size over the whole frame."""
    spec = synth.spec_4k()
    n_frames = 24
    src = synth.FrameSource(spec, device=dev, n_frames=n_frames)
    p, q = _params(spec, bias)
    res = fwrs.Reservoir(spec.width, spec.height, spec.k, p, stream=torch.cuda.current_stream())
    orc = oracle.Oracle(spec.width, spec.height, spec.k, q)
    gy0 = int(src.gaze[0, 1])
    bands = [(0, 4), (max(0, gy0 - 6), min(spec.height, gy0 + 6)), (1000, 1008), (spec.height - 4, spec.height)]
    out = torch.empty((spec.height, spec.width, 3), device=dev)
    for t in range(n_frames):
        c, lev, gx, gy = src.frame(t)
        res.step(c, lev, gx, gy, out)
        cn, ln = c.cpu().numpy(), lev.cpu().numpy()
        for (y0, y1) in bands:
            orc.push_rows(cn, ln, gx, gy, y0, y1)
        orc.advance()
        if t in (0, 5, n_frames - 1):
            res.sync()
            st, so = res.download(), orc.state()
            ref = orc.resolve()
            o = out.cpu().numpy()
            for (y0, y1) in bands:
                sl = slice(y0, y1)
                np.testing.assert_array_equal(st.idx[:, sl], so.idx[:, sl])
                np.testing.assert_array_equal(st.cnt[sl], so.cnt[sl])
                np.testing.assert_array_equal(st.wsum[sl].view(np.uint32), so.wsum[sl].view(np.uint32))
                np.testing.assert_array_equal(st.wt[:, sl].view(np.uint32), so.wt[:, sl].view(np.uint32))
                np.testing.assert_array_equal(st.wslot[:, sl].view(np.uint32), so.wslot[:, sl].view(np.uint32))
                _compare_out(o[sl], ref[sl], f"4K rows {y0}-{y1} frame {t}")
            assert np.all(st.cnt == t + 1)
            assert np.all(st.idx <= t)
            assert np.all(st.wt > 0) and np.all(st.wt <= 1)
            assert np.isfinite(o).all() and o.min() >= 0.0 and o.max() <= 1.0
    takes, changed, updates = res.stats()
    assert updates == n_frames * spec.pixels and takes > 0


@pytest.mark.parametrize("res_from", [None, 1])
def test_4k_whole_frames(dev, res_from):
    """Whole 3840x2160, k = 4 frames 0, 1 and 2 of the benchmark's trace (forward, reversed and forward
    traversals) through the fused call: every state plane and every output pixel against the oracle.
    res_from = 1: frame 0 writes the resolve plane and frames 1 and 2 copy unchanged pixels from it."""
    spec = synth.spec_4k()
    src = synth.FrameSource(spec, device=dev, n_frames=3)
    p, q = _params(spec)
    res = fwrs.Reservoir(spec.width, spec.height, spec.k, p, stream=torch.cuda.current_stream())
    if res_from is not None:
        res.set_resolve_plane_from(res_from)
    orc = oracle.Oracle(spec.width, spec.height, spec.k, q)
    out = torch.full((spec.height, spec.width, 3), -1.0, device=dev)
    for t in range(3):
        c, lev, gx, gy = src.frame(t)
        res.step(c, lev, gx, gy, out)
        orc.push(c.cpu().numpy(), lev.cpu().numpy(), gx, gy)
        res.sync()
        _compare_state(res.download(), orc.state(), f"4K frame {t}")
        _compare_out(out.cpu().numpy(), orc.resolve(), f"4K frame {t}")
    res.close()
    orc.close()


def test_4k_600_frames_bands(dev):
    """The whole 600-frame 3840x2160, k = 4 trace through the fused call with the default launch policy
    (full resolve while the store fills, the resolve plane from frame 32): the oracle follows eight bands of
    rows (the edges, the first fixation, rows spread over the image) every frame, and the bands' state
    planes and outputs are compared at checkpoints through the trace; whole-frame invariants everywhere."""
    spec = synth.spec_4k()
    n_frames = 600
    src = synth.FrameSource(spec, device=dev, n_frames=n_frames)
    p, q = _params(spec)
    res = fwrs.Reservoir(spec.width, spec.height, spec.k, p, stream=torch.cuda.current_stream())
    orc = oracle.Oracle(spec.width, spec.height, spec.k, q)
    gy0 = int(src.gaze[0, 1])
    bands = [(0, 3), (max(0, gy0 - 4), min(spec.height, gy0 + 4)), (300, 304), (700, 704), (1080, 1084),
             (1500, 1504), (1900, 1904), (spec.height - 3, spec.height)]
    cn = np.zeros((spec.height, spec.width, 3), np.float32)     # only the bands' rows are filled
    ln = np.zeros((spec.height, spec.width), np.uint8)
    out = torch.empty((spec.height, spec.width, 3), device=dev)
    checkpoints = {30, 31, 32, 99, 199, 299, 399, 499, n_frames - 1}
    for t in range(n_frames):
        c, lev, gx, gy = src.frame(t)
        res.step(c, lev, gx, gy, out)
        for (y0, y1) in bands:
            cn[y0:y1] = c[y0:y1].cpu().numpy()
            ln[y0:y1] = lev[y0:y1].cpu().numpy()
            orc.push_rows(cn, ln, gx, gy, y0, y1)
        orc.advance()
        if t in checkpoints:
            res.sync()
            st, so = res.download(), orc.state()
            ref = orc.resolve()
            o = out.cpu().numpy()
            for (y0, y1) in bands:
                sl = slice(y0, y1)
                where = f"4K rows {y0}-{y1} frame {t}"
                np.testing.assert_array_equal(st.idx[:, sl], so.idx[:, sl], err_msg=where)
                np.testing.assert_array_equal(st.cnt[sl], so.cnt[sl], err_msg=where)
                for name in ("wsum", "wt", "col", "wslot"):
                    a, b = getattr(st, name), getattr(so, name)
                    a = a[sl] if a.ndim == 2 else (a[:, sl] if a.ndim == 3 else a[:, :, sl])
                    b = b[sl] if b.ndim == 2 else (b[:, sl] if b.ndim == 3 else b[:, :, sl])
                    np.testing.assert_array_equal(a.view(np.uint32), b.view(np.uint32), err_msg=f"{name} {where}")
                _compare_out(o[sl], ref[sl], where)
            assert np.all(st.cnt == t + 1) and np.all(st.idx <= t)
            assert np.all(st.wt > 0) and np.all(st.wt <= 1)
            assert np.isfinite(o).all() and o.min() >= 0.0 and o.max() <= 1.0
            del st, so, ref, o
    takes, changed, updates = res.stats()
    assert updates == n_frames * spec.pixels and 0 < changed <= takes
    res.close()
    orc.close()


# ---------------------------------------------------------------------------
# Batched engine
# ---------------------------------------------------------------------------
def _mix_specs():
    return [synth.StreamSpec(256, 144, 2, 5, 12.8, 32.0, 2.0, 2, 6.0, stream_id=0),
            synth.StreamSpec(200, 100, 4, 5, 10.0, 25.0, 2.0, 2, 6.0, stream_id=1),
            synth.StreamSpec(96, 64, 8, 5, 5.0, 12.5, 1.0, 2, 3.0, stream_id=2),
            synth.StreamSpec(37, 23, 3, 5, 2.0, 5.0, 1.0, 2, 2.0, stream_id=3),
            synth.StreamSpec(320, 180, 4, 5, 16.0, 40.0, 3.0, 2, 9.0, stream_id=4)]


@pytest.mark.parametrize("use_graph", [False, True])
def test_engine_tick_matches_oracle_and_plain_launches(dev, use_graph):
    specs = _mix_specs()
    stream = torch.cuda.current_stream()
    srcs = [synth.FrameSource(s, device=dev) for s in specs]
    eng = fwrs.Engine(len(specs), stream=stream, use_graph=use_graph)
    eng.set_tile(0, 16, 16)
    eng.set_tile(30000, 64, 4)
    batched, plain, orcs, outs_b, outs_p = [], [], [], [], []
    for i, s in enumerate(specs):
        p, q = _params(s)
        batched.append(fwrs.Reservoir(s.width, s.height, s.k, p, stream=stream))
        batched[-1].set_resolve_plane_from(i % 3)      # the frame's op differs between the tick's frames
        plain.append(fwrs.Reservoir(s.width, s.height, s.k, p, stream=stream))
        orcs.append(oracle.Oracle(s.width, s.height, s.k, q))
        outs_b.append(torch.empty((s.height, s.width, 3), device=dev))
        outs_p.append(torch.empty((s.height, s.width, 3), device=dev))
    for t in range(5):
        frames = [src.frame(t) for src in srcs]
        eng.tick([(batched[i], *frames[i], outs_b[i]) for i in range(len(specs))])
        for i in range(len(specs)):
            plain[i].step(*frames[i], outs_p[i])
            c, lev, gx, gy = frames[i]
            orcs[i].push(c.cpu().numpy(), lev.cpu().numpy(), gx, gy)
    torch.cuda.synchronize()
    for i in range(len(specs)):
        assert batched[i].frame_index == 5
        sb = batched[i].download()
        _compare_state(sb, orcs[i].state(), f"stream {i}")
        _compare_out(outs_b[i].cpu().numpy(), orcs[i].resolve(), f"stream {i}")
        assert torch.equal(outs_b[i], outs_p[i])
        assert batched[i].stats() == plain[i].stats()
        # the batched tick leaves `out` as this context's resolve: incremental may follow
        c, lev, gx, gy = srcs[i].frame(4)
        batched[i].step_incremental(c, lev, gx, gy, outs_b[i])
        plain[i].step(c, lev, gx, gy, outs_p[i])
        assert torch.equal(outs_b[i], outs_p[i])
    eng.close()


@pytest.mark.parametrize("use_graph", [False, True])
def test_engine_ticks_of_forty_contexts(dev, use_graph):
    """40 contexts per tick (one launch over all their items), and every other tick walks
    its frames and their items in reverse.  Every context's output and state equal plain launches."""
    ks = (1, 2, 3, 4, 8)
    specs = [synth.StreamSpec(48 + 8 * (i % 3), 32, ks[i % len(ks)], 4, 4.0, 10.0, 1.0, 2, 2.0, stream_id=100 + i)
             for i in range(40)]
    stream = torch.cuda.current_stream()
    srcs = [synth.FrameSource(s, device=dev) for s in specs]
    eng = fwrs.Engine(len(specs), stream=stream, use_graph=use_graph)
    batched, plain, outs_b, outs_p = [], [], [], []
    for i, s in enumerate(specs):
        p, _ = _params(s)
        batched.append(fwrs.Reservoir(s.width, s.height, s.k, p, stream=stream))
        batched[-1].set_resolve_plane_from(i % 4)
        plain.append(fwrs.Reservoir(s.width, s.height, s.k, p, stream=stream))
        outs_b.append(torch.empty((s.height, s.width, 3), device=dev))
        outs_p.append(torch.empty((s.height, s.width, 3), device=dev))
    for t in range(4):
        frames = [src.frame(t) for src in srcs]
        eng.tick([(batched[i], *frames[i], outs_b[i]) for i in range(len(specs))])
        for i in range(len(specs)):
            plain[i].step(*frames[i], outs_p[i])
    torch.cuda.synchronize()
    for i in range(len(specs)):
        assert batched[i].frame_index == 4
        assert torch.equal(outs_b[i], outs_p[i]), f"context {i}"
        _compare_state(batched[i].download(), plain[i].download(), f"context {i}")
        assert batched[i].stats() == plain[i].stats()
        batched[i].close()
        plain[i].close()
    eng.close()


def test_fwrs_tick_equals_plain_calls(dev):
    """fwrs_tick (the batched call of the boundary) on a mix of sizes, slot counts, bias modes and
    resolve-plane policies equals one fwrs_push_frame_resolve per entry, bit for bit, every tick;
    the oracle agrees on every stream at the end."""
    cases = [(256, 144, 2, fwrs.BIAS_BERNOULLI, 0), (200, 100, 4, fwrs.BIAS_BERNOULLI, None),
             (96, 64, 8, fwrs.BIAS_BERNOULLI, 1), (37, 23, 3, fwrs.BIAS_NONE, 0), (160, 90, 4, fwrs.BIAS_FULL, None),
             (64, 48, 4, fwrs.AES, None), (120, 60, 4, fwrs.BIAS_MEMORYLESS, 2), (33, 17, 16, fwrs.BIAS_BERNOULLI, 0)]
    stream = torch.cuda.current_stream()
    specs, srcs, tick_ctx, plain_ctx, orcs, outs_t, outs_p = [], [], [], [], [], [], []
    for i, (w, h, k, bias, res_from) in enumerate(cases):
        s = synth.StreamSpec(w, h, k, 7, 0.1 * w, 0.25 * w, 2.0, 3, 4.0, stream_id=20 + i)
        p, q = _params(s, bias)
        specs.append(s)
        srcs.append(synth.FrameSource(s, device=dev))
        tick_ctx.append(fwrs.Reservoir(w, h, k, p, stream=stream))
        plain_ctx.append(fwrs.Reservoir(w, h, k, p, stream=stream))
        if res_from is not None:
            tick_ctx[-1].set_resolve_plane_from(res_from)
        tick_ctx[-1].set_tile(*[(64, 1), (16, 16), (32, 8)][i % 3])
        orcs.append(oracle.Oracle(w, h, k, q))
        outs_t.append(torch.empty((h, w, 3), device=dev))
        outs_p.append(torch.empty((h, w, 3), device=dev))
    for t in range(7):
        frames = [src.frame(t) for src in srcs]
        fwrs.tick([(tick_ctx[i], *frames[i], outs_t[i]) for i in range(len(cases))], stream=stream)
        for i in range(len(cases)):
            plain_ctx[i].step(*frames[i], outs_p[i])
            c, lev, gx, gy = frames[i]
            orcs[i].push(c.cpu().numpy(), lev.cpu().numpy(), gx, gy)
        torch.cuda.synchronize()
        for i in range(len(cases)):
            assert torch.equal(outs_t[i], outs_p[i]), f"tick {t} case {cases[i]}"
    for i in range(len(cases)):
        assert tick_ctx[i].frame_index == 7
        _compare_state(tick_ctx[i].download(), plain_ctx[i].download(), f"case {cases[i]}")
        _compare_state(tick_ctx[i].download(), orcs[i].state(), f"oracle case {cases[i]}")
        _compare_out(outs_t[i].cpu().numpy(), orcs[i].resolve(), f"case {cases[i]}")
        assert tick_ctx[i].stats() == plain_ctx[i].stats()


def _group_schedule(n_ctx, n_frames, seed):
    """Ticks of a group-tick run: each a list of (context, frame index) in which every context's
    entries are its next consecutive frames (1 to 6 of them, drawn per tick), interleaved across
    contexts at random but in order within each context."""
    rng = np.random.Generator(np.random.PCG64(seed))
    done = [0] * n_ctx
    ticks = []
    while min(done) < n_frames:
        queues = []
        for i in range(n_ctx):
            m = min(int(rng.choice([1, 1, 2, 3, 4, 6])), n_frames - done[i])
            queues.append([(i, done[i] + j) for j in range(m)])
            done[i] += m
        entries = []
        while any(queues):
            live = [q for q in queues if q]
            entries.append(live[int(rng.integers(len(live)))].pop(0))
        ticks.append(entries)
    return ticks


@pytest.mark.parametrize("api", ["tick", "engine_graph", "engine_direct", "noalloc"])
def test_tick_groups_equal_plain_calls(dev, api):
    """Ticks in which a context appears several times -- its consecutive frames, run as one group
    (the pixel state held in registers across the group's frames for k in {1, 2, 4, 8} with one
    w_sum per pixel; each frame through the store in turn otherwise) -- equal one
    fwrs_push_frame_resolve per frame, bit for bit: every frame's output, the state and the
    counters, from the empty store on and through the resolve plane's switch-over (inside groups
    too); the oracle agrees on every stream at the end."""
    nf = 40
    cases = [(256, 144, 2, fwrs.BIAS_BERNOULLI, 0), (200, 100, 4, fwrs.BIAS_BERNOULLI, None),
             (96, 64, 8, fwrs.BIAS_BERNOULLI, 3), (130, 70, 8, fwrs.BIAS_BERNOULLI, None),
             (37, 23, 3, fwrs.BIAS_NONE, 0), (160, 90, 4, fwrs.BIAS_FULL, None), (64, 48, 4, fwrs.AES, None),
             (120, 60, 4, fwrs.BIAS_MEMORYLESS, 2), (33, 17, 16, fwrs.BIAS_BERNOULLI, 0),
             (50, 40, 1, fwrs.BIAS_NONE, 5), (72, 40, 4, fwrs.BIAS_BERNOULLI, "no plane")]
    stream = torch.cuda.current_stream()
    tick_ctx, plain_ctx, orcs, frames, outs_t, outs_p = [], [], [], [], [], []
    for i, (w, h, k, bias, res_from) in enumerate(cases):
        s = synth.StreamSpec(w, h, k, nf, 0.1 * w, 0.25 * w, 2.0, 3, 4.0, stream_id=40 + i)
        p, q = _params(s, bias)
        if res_from == "no plane":
            p.flags = fwrs.FLAG_NO_RESOLVE_PLANE
        tick_ctx.append(fwrs.Reservoir(w, h, k, p, stream=stream))
        plain_ctx.append(fwrs.Reservoir(w, h, k, p, stream=stream))
        if isinstance(res_from, int):
            tick_ctx[-1].set_resolve_plane_from(res_from)
            plain_ctx[-1].set_resolve_plane_from(res_from)
        tick_ctx[-1].set_tile(*[(64, 1), (16, 16), (32, 8)][i % 3])
        orcs.append(oracle.Oracle(w, h, k, q))
        src = synth.FrameSource(s, device=dev, n_frames=nf)
        frames.append([src.frame(t) for t in range(nf)])
        outs_t.append(torch.full((nf, h, w, 3), -1.0, device=dev))
        outs_p.append(torch.full((nf, h, w, 3), -2.0, device=dev))
    eng = fwrs.Engine(128, stream=stream, use_graph=api == "engine_graph") if api.startswith("engine") else None
    ticks = _group_schedule(len(cases), nf, seed=7)
    assert max(len(e) for e in ticks) <= fwrs.TICK_NOALLOC_MAX
    assert any(len(e) > len({i for i, _ in e}) for e in ticks)
    for entries in ticks:
        batch = [(tick_ctx[i], *frames[i][t], outs_t[i][t]) for (i, t) in entries]
        if api == "tick":
            fwrs.tick(batch, stream=stream)
        elif api == "noalloc":
            fwrs.tick_noalloc(batch, stream=stream)
        else:
            eng.tick(batch)
    for i in range(len(cases)):
        for t in range(nf):
            plain_ctx[i].step(*frames[i][t], outs_p[i][t])
            c, lev, gx, gy = frames[i][t]
            orcs[i].push(c.cpu().numpy(), lev.cpu().numpy(), gx, gy)
    torch.cuda.synchronize()
    if eng is not None:
        eng.close()
    for i, case in enumerate(cases):
        for t in range(nf):
            assert torch.equal(outs_t[i][t], outs_p[i][t]), f"frame {t} case {case} ({api})"
        assert tick_ctx[i].frame_index == nf
        _compare_state(tick_ctx[i].download(), plain_ctx[i].download(), f"case {case} ({api})")
        _compare_state(tick_ctx[i].download(), orcs[i].state(), f"oracle case {case} ({api})")
        _compare_out(outs_t[i][nf - 1].cpu().numpy(), orcs[i].resolve(), f"case {case} ({api})")
        assert tick_ctx[i].stats() == plain_ctx[i].stats(), f"case {case} ({api})"
        tick_ctx[i].close()
        plain_ctx[i].close()
        orcs[i].close()


@pytest.mark.parametrize("api", ["tick", "noalloc"])
def test_long_groups_equal_plain_calls(dev, api):
    """Two contexts with 50 frames each in one tick (a group per context far longer than the serving
    loop forms): k = 4 (the register path) and k = 3 (each frame through the store), from the empty
    store through the resolve plane's switch; every frame's output, the state and the counters equal
    one fwrs_push_frame_resolve per frame, bit for bit."""
    nf = 50
    stream = torch.cuda.current_stream()
    cases = [(80, 48, 4, fwrs.BIAS_BERNOULLI, 20), (45, 30, 3, fwrs.BIAS_BERNOULLI, 0)]
    tick_ctx, plain_ctx, frames, outs_t, outs_p = [], [], [], [], []
    for i, (w, h, k, bias, res_from) in enumerate(cases):
        s = synth.StreamSpec(w, h, k, nf, 0.1 * w, 0.25 * w, 2.0, 3, 4.0, stream_id=70 + i)
        p, _ = _params(s, bias)
        tick_ctx.append(fwrs.Reservoir(w, h, k, p, stream=stream))
        plain_ctx.append(fwrs.Reservoir(w, h, k, p, stream=stream))
        tick_ctx[-1].set_resolve_plane_from(res_from)
        plain_ctx[-1].set_resolve_plane_from(res_from)
        src = synth.FrameSource(s, device=dev, n_frames=nf)
        frames.append([src.frame(t) for t in range(nf)])
        outs_t.append(torch.full((nf, h, w, 3), -1.0, device=dev))
        outs_p.append(torch.full((nf, h, w, 3), -2.0, device=dev))
    # the two contexts' frames interleaved, each context's in order
    batch = [(tick_ctx[i], *frames[i][t], outs_t[i][t]) for t in range(nf) for i in range(len(cases))]
    if api == "tick":
        fwrs.tick(batch, stream=stream)
    else:
        fwrs.tick_noalloc(batch, stream=stream)
    for i in range(len(cases)):
        for t in range(nf):
            plain_ctx[i].step(*frames[i][t], outs_p[i][t])
    torch.cuda.synchronize()
    for i, case in enumerate(cases):
        for t in range(nf):
            assert torch.equal(outs_t[i][t], outs_p[i][t]), f"frame {t} case {case} ({api})"
        assert tick_ctx[i].frame_index == nf
        _compare_state(tick_ctx[i].download(), plain_ctx[i].download(), f"case {case} ({api})")
        assert tick_ctx[i].stats() == plain_ctx[i].stats()
        tick_ctx[i].close()
        plain_ctx[i].close()


@pytest.mark.parametrize("k", [4, 8])
def test_4k_group_equals_plain_calls(dev, k):
    """A 4K context's frames 30-37 as one group of 8 (the launch the benchmark's groups section times),
    after 30 plain frames and across the resolve plane's switch at frame 32, equal eight
    fwrs_push_frame_resolve calls on a twin context, bit for bit: every frame's whole output and the
    whole state."""
    spec = synth.spec_4k(frames=600)
    src = synth.FrameSource(spec, device=dev, n_frames=600)
    stream = torch.cuda.current_stream()
    p, _ = _params(spec)
    a = fwrs.Reservoir(spec.width, spec.height, k, p, stream=stream)
    b = fwrs.Reservoir(spec.width, spec.height, k, p, stream=stream)
    tmp = torch.empty((spec.height, spec.width, 3), device=dev)
    for t in range(30):
        fr = src.frame(t)
        a.step(*fr, tmp)
        b.step(*fr, tmp)
    frames = [src.frame(t) for t in range(30, 38)]
    oa = torch.full((8, spec.height, spec.width, 3), -1.0, device=dev)
    ob = torch.full((8, spec.height, spec.width, 3), -2.0, device=dev)
    fwrs.tick([(a, *frames[i], oa[i]) for i in range(8)], stream=stream)
    for i in range(8):
        b.step(*frames[i], ob[i])
    torch.cuda.synchronize()
    for i in range(8):
        assert torch.equal(oa[i], ob[i]), f"frame {30 + i} differs (k={k})"
    assert a.frame_index == b.frame_index == 38
    _compare_state(a.download(), b.download(), f"4K k={k} after the group")
    assert a.stats() == b.stats()
    a.close()
    b.close()


@pytest.mark.parametrize("n,w,h", [(300, 24, 8), (48, 256, 256)])
def test_tick_of_many_frames(dev, n, w, h):
    """Ticks of many frames: 300 one-item frames and 48 frames of 256 items each (12288 blocks in one
    launch), through fwrs_tick and an engine in graph mode, against plain launches, forward and reversed
    ticks."""
    stream = torch.cuda.current_stream()
    specs = [synth.StreamSpec(w, h, (1, 2, 4, 8, 5)[i % 5], 4, 0.2 * w, 0.5 * w, 1.0, 2, 2.0, stream_id=300 + i)
             for i in range(n)]
    srcs = [synth.FrameSource(s, device=dev) for s in specs]
    eng = fwrs.Engine(n, stream=stream, use_graph=True)
    a, b, c_ = [], [], []
    for s in specs:
        p, _ = _params(s)
        a.append(fwrs.Reservoir(s.width, s.height, s.k, p, stream=stream))
        b.append(fwrs.Reservoir(s.width, s.height, s.k, p, stream=stream))
        c_.append(fwrs.Reservoir(s.width, s.height, s.k, p, stream=stream))
    oa = [torch.empty((h, w, 3), device=dev) for _ in specs]
    ob = [torch.empty((h, w, 3), device=dev) for _ in specs]
    oc = [torch.empty((h, w, 3), device=dev) for _ in specs]
    for t in range(4):
        frames = [src.frame(t) for src in srcs]
        fwrs.tick([(a[i], *frames[i], oa[i]) for i in range(n)], stream=stream)
        eng.tick([(b[i], *frames[i], ob[i]) for i in range(n)])
        for i in range(n):
            c_[i].step(*frames[i], oc[i])
    torch.cuda.synchronize()
    for i in range(n):
        assert torch.equal(oa[i], oc[i]) and torch.equal(ob[i], oc[i]), f"frame {i}"
        assert a[i].stats() == c_[i].stats() and b[i].stats() == c_[i].stats()
    _compare_state(a[n // 2].download(), c_[n // 2].download(), "middle context")
    eng.close()


def test_engine_stream_alone_equals_stream_in_mix(dev):
    specs = _mix_specs()
    stream = torch.cuda.current_stream()
    srcs = [synth.FrameSource(s, device=dev) for s in specs]
    eng = fwrs.Engine(len(specs), stream=stream, use_graph=True)
    mix = [fwrs.Reservoir(s.width, s.height, s.k, _params(s)[0], stream=stream) for s in specs]
    alone = fwrs.Reservoir(specs[1].width, specs[1].height, specs[1].k, _params(specs[1])[0], stream=stream)
    outs = [torch.empty((s.height, s.width, 3), device=dev) for s in specs]
    out_alone = torch.empty_like(outs[1])
    for t in range(4):
        frames = [src.frame(t) for src in srcs]
        # the mix changes membership from tick to tick
        members = [i for i in range(len(specs)) if (i + t) % 3 != 0 or i == 1]
        eng.tick([(mix[i], *frames[i], outs[i]) for i in members])
        eng.tick([(alone, *frames[1], out_alone)])
        for i in range(len(specs)):
            if i not in members:
                mix[i].step(*frames[i], outs[i])
    torch.cuda.synchronize()
    assert torch.equal(outs[1], out_alone)
    a, b = mix[1].download(), alone.download()
    np.testing.assert_array_equal(a.idx, b.idx)
    np.testing.assert_array_equal(a.col, b.col)
    eng.close()


def test_engine_rejects_bad_ticks(dev):
    stream = torch.cuda.current_stream()
    eng = fwrs.Engine(2, stream=stream)
    r = fwrs.Reservoir(32, 16, 4, stream=stream)
    c = torch.zeros((16, 32, 3), device=dev)
    lev = torch.zeros((16, 32), dtype=torch.uint8, device=dev)
    out = torch.empty_like(c)
    with pytest.raises(ValueError):
        eng.tick([(r, c, lev, 1.0, 1.0, out)] * 3)                            # over capacity
    with pytest.raises(fwrs.FwrsError):
        eng.tick([(r, c, lev, float("nan"), 1.0, out)])
    with pytest.raises(fwrs.FwrsError):                                       # one bad entry of a group
        eng.tick([(r, c, lev, 1.0, 1.0, out), (r, c, lev, 1.0, float("inf"), out)])
    assert r.frame_index == 0
    eng.tick([(r, c, lev, 1.0, 1.0, out), (r, c, lev, 1.0, 1.0, out)])       # a context's two frames
    assert r.frame_index == 2
    with pytest.raises(fwrs.FwrsError):
        r.set_tile(3, 8)
    eng.close()


# ---------------------------------------------------------------------------
# Full temporal bias (Eq. 7): per-slot w_sum and the CIE94 colour difference
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("bias", [fwrs.BIAS_FULL, fwrs.AES, fwrs.BIAS_MEMORYLESS])
def test_modes_small_workload_every_frame(dev, bias):
    """Eq. 7 and the two ablations (A-ES, memory-less bias) on the 256x256 trace, every frame."""
    spec = synth.spec_small()
    res, _, _ = _run_pair(dev, spec, spec.frames, bias=bias)
    per_slot = bias in (fwrs.BIAS_FULL, fwrs.AES)
    assert res.state_view().wsum_slots == (spec.k if per_slot else 1)
    st = res.download()
    if per_slot:
        assert np.all(st.wsum == 0.0)


@pytest.mark.parametrize("w,h,k,frames", [
    (1, 1, 1, 4), (3, 2, 16, 4), (13, 7, 3, 5), (100, 37, 5, 4), (64, 64, 8, 5), (96, 40, 4, 4), (255, 3, 2, 4),
    (1367, 769, 4, 3),
])
@pytest.mark.parametrize("bias", [fwrs.BIAS_FULL, fwrs.AES, fwrs.BIAS_MEMORYLESS])
def test_modes_sizes_and_slot_counts(dev, w, h, k, frames, bias):
    spec = synth.StreamSpec(w, h, k, frames, max(1.0, 0.1 * w), max(2.5, 0.25 * w), 0.2 * w + 0.5, 2, 0.3 * w + 1,
                            stream_id=k)
    _run_pair(dev, spec, frames, bias=bias)


@pytest.mark.parametrize("k", [4, 3, 8])
@pytest.mark.parametrize("bias", [fwrs.BIAS_FULL, fwrs.AES, fwrs.BIAS_MEMORYLESS])
def test_modes_split_and_incremental_equal_fused(dev, k, bias):
    spec = synth.StreamSpec(160, 96, k, 12, 16.0, 40.0, 3.0, 4, 8.0)
    _, _, out_f = _run_pair(dev, spec, 12, bias=bias, every=4)
    _, _, out_s = _run_pair(dev, spec, 12, mode="split", bias=bias, every=12)
    _, _, out_i = _run_pair(dev, spec, 12, mode="incremental", bias=bias, every=3)
    assert torch.equal(out_f, out_s)
    assert torch.equal(out_f, out_i)


@pytest.mark.parametrize("tile", [(8, 8), (16, 16), (256, 1)])
def test_eq7_tile_shape_never_changes_results(dev, tile):
    spec = synth.StreamSpec(200, 120, 4, 5, 20.0, 50.0, 3.0, 2, 9.0)
    _run_pair(dev, spec, 5, tile=tile, bias=fwrs.BIAS_FULL)


def test_eq7_static_scene_equals_eq6(dev):
    """A stationary gaze over a static scene offers every pixel the same colour each frame:
    |dL| = 0, so the per-slot sums equal Eq. 6's shared sum and the samples agree bit for bit."""
    spec = synth.StreamSpec(128, 72, 4, 10, 8.0, 20.0, 1.0, 4, 3.0)
    gaze = np.tile(np.array([[40.3, 30.6]], np.float32), (10, 1))
    outs, states = [], []
    for bias in (fwrs.BIAS_BERNOULLI, fwrs.BIAS_FULL):
        src = synth.FrameSource(spec, device=dev, gaze=gaze)
        res, _, out = _run_pair(dev, spec, 10, bias=bias, every=10, src=src)
        outs.append(out)
        states.append(res.download())
    assert torch.equal(outs[0], outs[1])
    np.testing.assert_array_equal(states[0].idx, states[1].idx)
    np.testing.assert_array_equal(states[0].wslot, states[1].wslot)


@pytest.mark.parametrize("k", [4, 8, 3])
def test_eq7_repeated_and_edge_colours(dev, k):
    """Eq. 7 on colours that repeat across frames, drawn from edge values (signed zeros, a denormal,
    2^24 and its neighbour below, +-3e7, +-1e30 whose Lab is not finite): samples equal to the new
    pixel and unequal ones share waves, and whole waves hold only equal ones (the left half).
    Every state plane bit-exact with the oracle each frame, through plain calls and ticks; the
    resolve within 1e-5 of the oracle's, relative to the pixel's largest slot colour."""
    w, h, n = 96, 40, 8
    frames = edge_colours.palette_frames(w, h, n, dev, seed=10 + k)
    spec = synth.StreamSpec(w, h, k, n, 8.0, 20.0, 1.0, 2, 3.0, stream_id=k)
    p, q = _params(spec, fwrs.BIAS_FULL)
    stream = torch.cuda.current_stream()
    plain = fwrs.Reservoir(w, h, k, p, stream=stream)
    ticked = fwrs.Reservoir(w, h, k, p, stream=stream)
    orc = oracle.Oracle(w, h, k, q)
    out = torch.empty((h, w, 3), device=dev)
    out_t = torch.empty((h, w, 3), device=dev)
    for t, (c, lev, gx, gy) in enumerate(frames):
        plain.step(c, lev, gx, gy, out)
        fwrs.tick([(ticked, c, lev, gx, gy, out_t)], stream=stream)
        orc.push(c.cpu().numpy(), lev.cpu().numpy(), gx, gy)
        torch.cuda.synchronize()
        so = orc.state()
        _compare_state(plain.download(), so, f"frame {t} k={k}")
        _compare_state(ticked.download(), so, f"tick, frame {t} k={k}")
        err = np.abs(out.cpu().numpy().astype(np.float64) - orc.resolve()).max(axis=2)
        assert np.all(err <= COLOR_TOL * edge_colours.resolve_scale(so.col)), f"frame {t}"
        assert torch.equal(out, out_t)


def test_eq7_caller_arena_is_sized_by_mode(dev):
    spec = synth.StreamSpec(128, 64, 4, 4, 12.0, 30.0, 2.0, 2, 6.0)
    p, q = _params(spec, fwrs.BIAS_FULL)
    shared = fwrs.default_params(spec.width, flags=fwrs.FLAG_NO_RESOLVE_PLANE)
    small = torch.empty(fwrs.state_bytes(spec.width, spec.height, spec.k, shared), dtype=torch.uint8, device=dev)
    with pytest.raises(fwrs.FwrsError):
        fwrs.Reservoir(spec.width, spec.height, spec.k, p, stream=torch.cuda.current_stream(), arena=small)
    arena = torch.full((fwrs.state_bytes(spec.width, spec.height, spec.k, p),), 0xAB,
                       dtype=torch.uint8, device=dev)
    res = fwrs.Reservoir(spec.width, spec.height, spec.k, p, stream=torch.cuda.current_stream(), arena=arena)
    orc = oracle.Oracle(spec.width, spec.height, spec.k, q)
    src = synth.FrameSource(spec, device=dev)
    out = torch.empty((spec.height, spec.width, 3), device=dev)
    for t in range(4):
        c, lev, gx, gy = src.frame(t)
        res.step(c, lev, gx, gy, out)
        orc.push(c.cpu().numpy(), lev.cpu().numpy(), gx, gy)
    res.sync()
    _compare_state(res.download(), orc.state())
    _compare_out(out.cpu().numpy(), orc.resolve())


@pytest.mark.parametrize("use_graph", [False, True])
def test_eq7_engine_mixes_bias_modes(dev, use_graph):
    """One batched tick over contexts of every mode matches the oracle per context."""
    specs = _mix_specs()
    modes = [fwrs.BIAS_FULL, fwrs.BIAS_BERNOULLI, fwrs.AES, fwrs.BIAS_NONE, fwrs.BIAS_MEMORYLESS]
    stream = torch.cuda.current_stream()
    srcs = [synth.FrameSource(s, device=dev) for s in specs]
    eng = fwrs.Engine(len(specs), stream=stream, use_graph=use_graph)
    ctxs, orcs, outs = [], [], []
    for s, m in zip(specs, modes):
        p, q = _params(s, m)
        ctxs.append(fwrs.Reservoir(s.width, s.height, s.k, p, stream=stream))
        orcs.append(oracle.Oracle(s.width, s.height, s.k, q))
        outs.append(torch.empty((s.height, s.width, 3), device=dev))
    for t in range(5):
        frames = [src.frame(t) for src in srcs]
        eng.tick([(ctxs[i], *frames[i], outs[i]) for i in range(len(specs))])
        for i in range(len(specs)):
            c, lev, gx, gy = frames[i]
            orcs[i].push(c.cpu().numpy(), lev.cpu().numpy(), gx, gy)
    torch.cuda.synchronize()
    for i in range(len(specs)):
        _compare_state(ctxs[i].download(), orcs[i].state(), f"stream {i} bias {modes[i]}")
        _compare_out(outs[i].cpu().numpy(), orcs[i].resolve(), f"stream {i}")
    eng.close()


@pytest.mark.parametrize("bias", [fwrs.BIAS_NONE, fwrs.BIAS_BERNOULLI, fwrs.BIAS_FULL, fwrs.BIAS_MEMORYLESS, fwrs.AES])
def test_long_run_every_mode(dev, bias):
    """600 frames of a 128x96 stream with frequent saccades: the weight sums and keys after long
    histories stay bit-identical (no drift between the binary32 sequences)."""
    spec = synth.StreamSpec(128, 96, 4, 600, 10.0, 25.0, 2.0, 15, 6.0, stream_id=9)
    res, orc, _ = _run_pair(dev, spec, 600, bias=bias, every=150)
    takes, changed, updates = res.stats()
    assert updates == 600 * spec.pixels and takes > 0
