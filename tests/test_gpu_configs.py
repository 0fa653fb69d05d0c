"""Parity at the full sizes of the batched workloads, in the launch configuration the benchmark
times (one batched launch per tick over all its frames, replayed as a HIP graph): the stereo pair
(2 x 2064x2208, k = 8, vergence-shifted gaze, 36 ticks) and the 16 uneven streams (720p to 4K, k in
{2, 4, 8}).  The oracle follows
bands of rows (through the gaze, the top and bottom edges) of every stream, bit-exact in every state
plane and within 1e-5 in colour; whole-frame properties are checked everywhere."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import oracle
from paper_2510_03964_amd import fwrs, synth

pytestmark = pytest.mark.gpu
COLOR_TOL = 1e-5


@pytest.fixture(scope="module")
def dev():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    fwrs.load()
    return torch.device("cuda:0")


def _bands(spec, gy):
    H = spec.height
    g = int(min(max(gy, 3), H - 4))
    return [(0, 3), (g - 3, g + 3), (H - 3, H)]


def _compare_bands(ctx, orc, bands, out, where):
    st, so = ctx.download(), orc.state()
    ref = orc.resolve()
    o = out.cpu().numpy()
    for (y0, y1) in bands:
        sl = slice(y0, y1)
        np.testing.assert_array_equal(st.idx[:, sl], so.idx[:, sl], err_msg=where)
        for name in ("wsum", "wt", "col", "wslot"):
            a, b = getattr(st, name), getattr(so, name)
            a = a[sl] if a.ndim == 2 else (a[:, sl] if a.ndim == 3 else a[:, :, sl])
            b = b[sl] if b.ndim == 2 else (b[:, sl] if b.ndim == 3 else b[:, :, sl])
            np.testing.assert_array_equal(a.view(np.uint32), b.view(np.uint32), err_msg=f"{name} {where}")
        err = np.abs(o[sl].astype(np.float64) - ref[sl]).max()
        assert err <= COLOR_TOL, f"resolve differs by {err} {where}"
    return st, o


def _run_batched(dev, specs, gazes, ticks, check_every=None):
    stream = torch.cuda.current_stream()
    eng = fwrs.Engine(len(specs), stream=stream, use_graph=True)
    srcs = [synth.FrameSource(s, device=dev, gaze=g[:ticks]) for s, g in zip(specs, gazes)]
    ctxs, orcs, outs, bands = [], [], [], []
    for s, g in zip(specs, gazes):
        p = fwrs.default_params(s.width, fovea_radius_px=s.fovea_radius_px, seed=synth.PHILOX_SEED,
                                stream_id=s.stream_id)
        q = oracle.default_params(s.width, fovea_radius_px=s.fovea_radius_px, seed=synth.PHILOX_SEED,
                                  stream_id=s.stream_id)
        ctxs.append(fwrs.Reservoir(s.width, s.height, s.k, p, stream=stream))
        orcs.append(oracle.Oracle(s.width, s.height, s.k, q))
        outs.append(torch.empty((s.height, s.width, 3), device=dev))
        bands.append(_bands(s, float(g[0, 1])))
    for t in range(ticks):
        frames = [src.frame(t) for src in srcs]
        eng.tick([(ctxs[i], *frames[i], outs[i]) for i in range(len(specs))])
        for i, (c, lev, gx, gy) in enumerate(frames):
            cn, ln = c.cpu().numpy(), lev.cpu().numpy()
            for (y0, y1) in bands[i]:
                orcs[i].push_rows(cn, ln, gx, gy, y0, y1)
            orcs[i].advance()
        if check_every and (t + 1) % check_every == 0 and t + 1 < ticks:
            torch.cuda.synchronize()
            for i, s in enumerate(specs):
                _compare_bands(ctxs[i], orcs[i], bands[i], outs[i], f"tick {t} stream {i}")
    torch.cuda.synchronize()
    eng.close()
    for i, s in enumerate(specs):
        where = f"stream {i} {s.width}x{s.height} k={s.k}"
        st, o = _compare_bands(ctxs[i], orcs[i], bands[i], outs[i], where)
        assert np.all(st.cnt == ticks) and np.all(st.idx < ticks)
        assert np.all(st.wt > 0) and np.all(st.wt <= 1)
        assert np.isfinite(o).all() and o.min() >= 0.0 and o.max() <= 1.0
        assert ctxs[i].frame_index == ticks
        ctxs[i].close()
        orcs[i].close()
        del st, o


def test_stereo_pair_k8_batched(dev):
    left, right = synth.spec_stereo()
    g_left = synth.gaze_trace(left)
    g_right = g_left + np.array([synth.vergence_shift(), 0.0], dtype=np.float32)
    g_right[:, 0] = np.clip(g_right[:, 0], 0.0, float(right.width))
    # 36 ticks: the fill, the switch to the resolve plane (frame 32) and cached ticks after it,
    # checked every 6 ticks
    _run_batched(dev, [left, right], [g_left, g_right], ticks=36, check_every=6)


def test_uneven_16_streams_batched(dev):
    specs = synth.spec_uneven()
    _run_batched(dev, specs, [synth.gaze_trace(s) for s in specs], ticks=3)
