"""fwrs_tick_noalloc (the batched call that allocates nothing) against fwrs_tick, through the C ABI.

Two calls in a row on the same contexts' twins -- the second with fewer and smaller frames -- and a
third small enough to travel in the kernel's arguments must leave every output and every state
plane bit-identical to fwrs_tick's (the batched results are
decided and copied values; the resolve is the same binary32 computation), and sizes beyond the
fixed table are refused before any device work.
"""
from __future__ import annotations

import ctypes as C

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


def _frames(entries):
    buf = (fwrs.Frame * len(entries))()
    for i, (res, color, level, gx, gy, out) in enumerate(entries):
        buf[i].ctx = res.handle
        buf[i].color = color.data_ptr()
        buf[i].level_map = level.data_ptr()
        buf[i].gaze_x = float(gx)
        buf[i].gaze_y = float(gy)
        buf[i].out = out.data_ptr()
    return buf


def _pair(dev, cases, stream):
    specs, srcs, a, b, oa, ob = [], [], [], [], [], []
    for i, (w, h, k, bias) in enumerate(cases):
        s = synth.StreamSpec(w, h, k, 8, 0.1 * w, 0.25 * w, 2.0, 3, 4.0, stream_id=50 + i)
        p = fwrs.default_params(w, fovea_radius_px=s.fovea_radius_px, seed=synth.PHILOX_SEED, stream_id=s.stream_id,
                                bias_mode=bias)
        specs.append(s)
        srcs.append(synth.FrameSource(s, device=dev))
        a.append(fwrs.Reservoir(w, h, k, p, stream=stream))
        b.append(fwrs.Reservoir(w, h, k, p, stream=stream))
        if bias in (fwrs.BIAS_NONE, fwrs.BIAS_BERNOULLI):
            a[-1].set_resolve_plane_from(1)
            b[-1].set_resolve_plane_from(1)
        oa.append(torch.full((h, w, 3), -1.0, device=dev))
        ob.append(torch.full((h, w, 3), -2.0, device=dev))
    return specs, srcs, a, b, oa, ob


def _check_equal(a, b, oa, ob, where):
    for i in range(len(a)):
        assert torch.equal(oa[i], ob[i]), f"{where}: output of context {i}"
        sa, sb = a[i].download(), b[i].download()
        for name in ("wsum", "cnt", "wt", "idx", "col", "wslot"):
            np.testing.assert_array_equal(getattr(sa, name).view(np.uint32), getattr(sb, name).view(np.uint32),
                                          err_msg=f"{where}: {name} of context {i}")
        assert a[i].frame_index == b[i].frame_index
        assert a[i].stats() == b[i].stats()


def test_noalloc_tick_equals_fwrs_tick(dev):
    L = fwrs.load()
    stream = torch.cuda.current_stream()
    h = stream.cuda_stream
    # call 1: 30 frames (two fill launches) of mixed sizes, slot counts and modes
    cases = [(64 + 16 * (i % 5), 32 + 8 * (i % 3), (1, 2, 4, 8, 3)[i % 5],
              (fwrs.BIAS_BERNOULLI, fwrs.BIAS_NONE, fwrs.BIAS_FULL, fwrs.AES, fwrs.BIAS_MEMORYLESS)[i % 5])
             for i in range(30)]
    specs, srcs, a, b, oa, ob = _pair(dev, cases, stream)
    for t in range(3):
        fr = [src.frame(t) for src in srcs]
        ea = [(a[i], *fr[i], oa[i]) for i in range(len(cases))]
        eb = [(b[i], *fr[i], ob[i]) for i in range(len(cases))]
        assert L.fwrs_tick_noalloc(_frames(ea), len(ea), C.c_void_p(h)) == fwrs.OK
        assert L.fwrs_tick(_frames(eb), len(eb), C.c_void_p(h)) == fwrs.OK
    torch.cuda.synchronize()
    _check_equal(a, b, oa, ob, "first call")
    # call 2: a smaller input -- 24 of the contexts, the smallest frames (still more entries than a
    # kernel's arguments hold, so the fixed table is used again, over the first call's contents)
    keep = sorted(range(len(cases)), key=lambda i: (specs[i].pixels, i))[:24]
    for t in range(3, 5):
        fr = {i: srcs[i].frame(t) for i in keep}
        ea = [(a[i], *fr[i], oa[i]) for i in keep]
        eb = [(b[i], *fr[i], ob[i]) for i in keep]
        assert L.fwrs_tick_noalloc(_frames(ea), len(ea), C.c_void_p(h)) == fwrs.OK
        assert L.fwrs_tick(_frames(eb), len(eb), C.c_void_p(h)) == fwrs.OK
    torch.cuda.synchronize()
    _check_equal([a[i] for i in keep], [b[i] for i in keep], [oa[i] for i in keep], [ob[i] for i in keep],
                 "second call")
    # call 3: 5 contexts, two frames of one of them (a table small enough for the kernel's arguments)
    few = keep[:5]
    ea = [(a[i], *srcs[i].frame(5), oa[i]) for i in few] + [(a[few[0]], *srcs[few[0]].frame(6), oa[few[0]])]
    eb = [(b[i], *srcs[i].frame(5), ob[i]) for i in few] + [(b[few[0]], *srcs[few[0]].frame(6), ob[few[0]])]
    assert L.fwrs_tick_noalloc(_frames(ea), len(ea), C.c_void_p(h)) == fwrs.OK
    assert L.fwrs_tick(_frames(eb), len(eb), C.c_void_p(h)) == fwrs.OK
    torch.cuda.synchronize()
    _check_equal([a[i] for i in few], [b[i] for i in few], [oa[i] for i in few], [ob[i] for i in few], "third call")
    for r in a + b:
        r.close()


def test_noalloc_tick_refuses_sizes_beyond_its_table(dev):
    L = fwrs.load()
    stream = torch.cuda.current_stream()
    r = fwrs.Reservoir(16, 8, 4, stream=stream)
    c = torch.zeros((8, 16, 3), device=dev)
    lev = torch.zeros((8, 16), dtype=torch.uint8, device=dev)
    out = torch.empty_like(c)
    buf = _frames([(r, c, lev, 1.0, 1.0, out)] * 257)
    assert L.fwrs_tick_noalloc(buf, 257, None) == fwrs.E_ARG
    assert L.fwrs_tick_noalloc(None, 1, None) == fwrs.E_ARG
    assert L.fwrs_tick_noalloc(None, 0, None) == fwrs.OK
    assert r.frame_index == 0
    with pytest.raises(ValueError):
        fwrs.tick_noalloc([(r, c, lev, 1.0, 1.0, out)] * 257, stream=stream)
    r.close()
