"""Pins of the oracle's reprojection and depth flush (Sec. 4.3; the fall-back of Sec. 6), CPU only.

What fixes the expected values: with no motion the reprojected pass must be the plain pass; an
integer motion moves every reservoir by exactly that many pixels (checked against numpy slicing of
the previous state); a sub-pixel motion rounds by the pixel that contains the moved centre; a
flushed pixel holds exactly what the first frame of an empty reservoir holds (every slot takes,
w_sum = w, m = 1); the depth test keeps a history within the relative tolerance and drops it
beyond."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2510_03964_amd import synth

W, H, K = 48, 32, 4
TOL = 0.1


def _params(oracle_mod, bias, seed=synth.PHILOX_SEED):
    return oracle_mod.default_params(W, fovea_radius_px=6.0, seed=seed, bias_mode=bias)


def _frames(n, seed=7):
    spec = synth.StreamSpec(W, H, K, n, 6.0, 15.0, 1.5, 3, 4.0)
    src = synth.MovingSource(spec)
    return [src.frame(t) for t in range(n)]


def _np(frame):
    c, lev, mv, d, gx, gy = frame
    return c.numpy(), lev.numpy(), mv.numpy(), d.numpy(), gx, gy


def _still(frame):
    """The frame with no motion and a constant depth."""
    c, lev, mv, d, gx, gy = _np(frame)
    return c, lev, np.zeros_like(mv), np.full_like(d, 5.0), gx, gy


@pytest.mark.parametrize("bias", [0, 1, 2])
def test_no_motion_equals_the_plain_pass(oracle_mod, bias):
    frames = [_still(f) for f in _frames(8)]
    a = oracle_mod.Oracle(W, H, K, _params(oracle_mod, bias))
    b = oracle_mod.Oracle(W, H, K, _params(oracle_mod, bias))
    for (c, lev, mv, d, gx, gy) in frames:
        a.push(c, lev, gx, gy)
        b.push_reproject(c, lev, mv, d, gx, gy, TOL)
    sa, sb = a.state(), b.state()
    for name in ("wsum", "cnt", "wt", "idx", "col", "wslot"):
        np.testing.assert_array_equal(getattr(sa, name), getattr(sb, name), err_msg=name)
    np.testing.assert_array_equal(a.resolve(), b.resolve())
    assert b.flushes == W * H                      # only the first frame (no previous depth)
    np.testing.assert_array_equal(b.depth(), frames[-1][3])


def _prepared(oracle_mod, bias, n=5):
    frames = [_still(f) for f in _frames(n + 1)]
    o = oracle_mod.Oracle(W, H, K, _params(oracle_mod, bias))
    for (c, lev, mv, d, gx, gy) in frames[:n]:
        o.push_reproject(c, lev, mv, d, gx, gy, TOL)
    return o, frames[n]


@pytest.mark.parametrize("bias", [1, 2])
@pytest.mark.parametrize("dx,dy", [(3, -2), (-5, 0), (0, 4)])
def test_integer_motion_moves_every_reservoir(oracle_mod, bias, dx, dy):
    o, (c, lev, mv, d, gx, gy) = _prepared(oracle_mod, bias)
    before = o.state()
    t = o.t
    mv = np.zeros_like(mv)
    mv[..., 0], mv[..., 1] = dx, dy
    f0 = o.flushes
    o.push_reproject(c, lev, mv, d, gx, gy, TOL)
    after = o.state()
    # source of pixel (x, y) is (x - dx, y - dy); inside <=> it exists
    ys, xs = np.mgrid[0:H, 0:W]
    sx, sy = xs - dx, ys - dy
    inside = (sx >= 0) & (sx < W) & (sy >= 0) & (sy < H)
    qy, qx = np.clip(sy, 0, H - 1), np.clip(sx, 0, W - 1)
    assert o.flushes - f0 == int((~inside).sum())
    np.testing.assert_array_equal(after.cnt[inside], before.cnt[qy, qx][inside] + 1)
    assert np.all(after.cnt[~inside] == 1)
    for j in range(K):
        kept = after.idx[j] != t
        # a slot that did not take holds the source pixel's sample, weight and frame index
        m = inside & kept
        np.testing.assert_array_equal(after.idx[j][m], before.idx[j][qy, qx][m])
        np.testing.assert_array_equal(after.wt[j][m], before.wt[j][qy, qx][m])
        for ch in range(3):
            np.testing.assert_array_equal(after.col[j, ch][m], before.col[j, ch][qy, qx][m])
        # a flushed pixel takes the candidate in every slot
        assert np.all(after.idx[j][~inside] == t)
        # a slot that took holds this frame's candidate at its own pixel
        took = after.idx[j] == t
        for ch in range(3):
            np.testing.assert_array_equal(after.col[j, ch][took], c[..., ch][took])


def test_flushed_pixel_is_the_first_frame_of_an_empty_reservoir(oracle_mod):
    """A flushed pixel ends up exactly as an empty reservoir that sees this frame: every slot
    holds the candidate with its weight, w_sum is that weight, m is 1."""
    o, (c, lev, mv, d, gx, gy) = _prepared(oracle_mod, 1)
    d2 = d.copy()
    d2[10:20, 5:30] = 50.0                       # a near surface moved away: disocclusion
    o.push_reproject(c, lev, np.zeros_like(mv), d2, gx, gy, TOL)
    st = o.state()
    fresh = oracle_mod.Oracle(W, H, K, _params(oracle_mod, 1))
    fresh.push(c, lev, gx, gy)
    sf = fresh.state()
    region = np.zeros((H, W), bool)
    region[10:20, 5:30] = True
    np.testing.assert_array_equal(st.wsum[region], sf.wsum[region])
    np.testing.assert_array_equal(st.wt[:, region], sf.wt[:, region])
    np.testing.assert_array_equal(st.col[:, :, region], sf.col[:, :, region])
    assert np.all(st.cnt[region] == 1) and np.all(st.idx[:, region] == o.t - 1)
    assert np.all(st.cnt[~region] == o.t)        # the rest kept its history
    np.testing.assert_array_equal(o.resolve()[region], c[region].astype(np.float64))


def test_depth_tolerance_is_relative_and_inclusive(oracle_mod):
    o, (c, lev, mv, d, gx, gy) = _prepared(oracle_mod, 1)     # previous depth 5 everywhere
    cnt0 = o.state().cnt.copy()
    d2 = np.full_like(d, 5.0)
    d2[:, :8] = 5.5            # |5.5 - 5| = 0.5 <= 0.1 * 5.5: kept
    d2[:, 8:16] = 4.5          # |4.5 - 5| = 0.5 > 0.1 * 4.5 = 0.45: flushed
    d2[:, 16:24] = 5.0 / 0.9 + 0.01    # just beyond the tolerance measured at the current depth
    d2[:, 24:32] = np.nan      # no usable depth: flushed
    f0 = o.flushes
    o.push_reproject(c, lev, np.zeros_like(mv), d2, gx, gy, TOL)
    cnt = o.state().cnt
    np.testing.assert_array_equal(cnt[:, :8], cnt0[:, :8] + 1)
    assert np.all(cnt[:, 8:32] == 1)
    np.testing.assert_array_equal(cnt[:, 32:], cnt0[:, 32:] + 1)
    assert o.flushes - f0 == 24 * H


@pytest.mark.parametrize("m,shift", [(0.49, 0), (0.5, 0), (0.5 + 2 ** -10, 1), (1.49, 1), (-0.5 + 2 ** -10, 0),
                                     (-0.5, -1)])
def test_subpixel_motion_takes_the_pixel_containing_the_moved_centre(oracle_mod, m, shift):
    """The moved centre x + 0.5 - m lies in pixel floor(x + 0.5 - m); a centre on a pixel
    boundary belongs to the pixel on its right."""
    o, (c, lev, mv, d, gx, gy) = _prepared(oracle_mod, 1)
    before = o.state()
    mv = np.zeros_like(mv)
    mv[..., 0] = m
    o.push_reproject(c, lev, mv, d, gx, gy, TOL)
    cnt = o.state().cnt
    src = np.arange(W) - shift
    inside = (src >= 0) & (src < W)
    np.testing.assert_array_equal(cnt[:, inside], before.cnt[:, src[inside]] + 1)
    assert np.all(cnt[:, ~inside] == 1)


def test_motion_out_of_the_image_flushes(oracle_mod):
    o, (c, lev, mv, d, gx, gy) = _prepared(oracle_mod, 1)
    mv = np.full_like(mv, 1e30)
    f0 = o.flushes
    o.push_reproject(c, lev, mv, d, gx, gy, TOL)
    assert o.flushes - f0 == W * H and np.all(o.state().cnt == 1)
    mv = np.full_like(mv, np.nan)
    o.push_reproject(c, lev, mv, d, gx, gy, TOL)
    assert o.flushes - f0 == 2 * W * H


def test_moving_workload_invariants(oracle_mod):
    """The moving-camera workload: every kept sample is a colour some frame rendered, the pixel
    counts never exceed the frame count, the disc's edges flush, and the history survives the
    pan elsewhere."""
    frames = [_np(f) for f in _frames(12)]
    o = oracle_mod.Oracle(W, H, K, _params(oracle_mod, 1))
    for (c, lev, mv, d, gx, gy) in frames:
        o.push_reproject(c, lev, mv, d, gx, gy, TOL)
    st = o.state()
    assert np.all(st.cnt >= 1) and np.all(st.cnt <= 12)
    assert np.all(st.idx <= 11)
    assert o.flushes > W * H                      # more than the first frame's
    assert np.median(st.cnt) > 3                  # most pixels keep a history under the pan
    seen = {tuple(v) for (c, *_rest) in frames for v in c.reshape(-1, 3).tolist()}
    for j in range(K):
        cols = st.col[j].reshape(3, -1).T.tolist()
        assert all(tuple(v) in seen for v in cols)


def test_depth_tolerance_boundary_is_kept(oracle_mod):
    """|4 - 5| = 1 = 0.25 * 4 exactly in binary32: kept at tolerance 0.25, flushed just below it."""
    for tol, kept in [(0.25, True), (0.2499, False)]:
        o, (c, lev, mv, d, gx, gy) = _prepared(oracle_mod, 1)
        cnt0 = o.state().cnt.copy()
        o.push_reproject(c, lev, np.zeros_like(mv), np.full_like(d, 4.0), gx, gy, tol)
        cnt = o.state().cnt
        if kept:
            np.testing.assert_array_equal(cnt, cnt0 + 1)
        else:
            assert np.all(cnt == 1)


@pytest.mark.parametrize("bias", [0, 1])
def test_weight_sum_travels_with_its_history(oracle_mod, bias):
    """Every pixel at full resolution (w = 1): the weight sum is a function of the history length
    alone -- under NONE it is the count itself -- so after a partial flush and an integer motion the
    moved sums must still match the moved counts pixel by pixel."""
    o, (c, lev, mv, d, gx, gy) = _prepared(oracle_mod, bias)
    lev0 = np.zeros_like(lev)
    o2 = oracle_mod.Oracle(W, H, K, _params(oracle_mod, bias))
    for _ in range(4):
        o2.push_reproject(c, lev0, np.zeros_like(mv), d, gx, gy, TOL)
    off = np.zeros_like(mv)
    off[5:20, 10:25] = 1e30                       # these pixels' sources leave the image: flushed
    o2.push_reproject(c, lev0, off, d, gx, gy, TOL)
    o2.push_reproject(c, lev0, np.zeros_like(mv), d, gx, gy, TOL)
    mv2 = np.zeros_like(mv)
    mv2[..., 0], mv2[..., 1] = 7, 3
    o2.push_reproject(c, lev0, mv2, d, gx, gy, TOL)
    st = o2.state()
    assert len(np.unique(st.cnt)) >= 3
    if bias == 0:
        np.testing.assert_array_equal(st.wsum, st.cnt.astype(np.float32))
    else:
        for n in np.unique(st.cnt):
            assert len(np.unique(st.wsum[st.cnt == n])) == 1, n
