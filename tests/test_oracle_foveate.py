"""Pins of the oracle's foveation generator (Sec. 4.3: mipmapping with bilinear filtering, or a
Gaussian blur growing away from the gaze), CPU only.

What fixes the expected values: box means and Gaussian weights evaluated in binary64; bilinear
interpolation and a symmetric normalised blur both reproduce a linear ramp exactly (up to
rounding), and a blur of an impulse is the outer product of its weights; the level rings against
a binary64 evaluation of the distance; the full-resolution ring passes the frame through untouched."""
from __future__ import annotations

import math

import numpy as np
import pytest

from paper_2510_03964_amd import synth


def _ramp(W, H, a=(0.011, -0.004, 0.002), b=(0.003, 0.009, -0.006), c=(0.1, 0.7, 0.5)):
    xs = np.arange(W, dtype=np.float64) + 0.5
    ys = np.arange(H, dtype=np.float64) + 0.5
    img = np.stack([a[i] * xs[None, :] + b[i] * ys[:, None] + c[i] for i in range(3)], -1)
    return img.astype(np.float32)


@pytest.mark.parametrize("W,H", [(64, 48), (37, 23), (1, 1), (5, 2)])
def test_mip_is_the_box_mean(oracle_mod, W, H):
    rng = np.random.Generator(np.random.PCG64(3))
    img = rng.uniform(0, 1, (H, W, 3)).astype(np.float32)
    got = oracle_mod.mip_down(img).astype(np.float64)
    pad = np.full(((H + 1) // 2 * 2, (W + 1) // 2 * 2, 3), np.nan)
    pad[:H, :W] = img
    blocks = pad.reshape(pad.shape[0] // 2, 2, pad.shape[1] // 2, 2, 3)
    want = np.nanmean(blocks, axis=(1, 3))
    assert np.abs(got - want).max() <= 2.0 ** -22
    const = np.full((H, W, 3), 0.3, np.float32)
    assert np.all(oracle_mod.mip_down(const) == np.float32(0.3))


def test_mip_bilinear_reproduces_a_linear_ramp(oracle_mod):
    """Box means of a linear function are its values at the block centres, and bilinear
    interpolation of a linear function is exact: away from the clamped border every level returns
    the ramp at the pixel centre."""
    W, H = 96, 64
    img = _ramp(W, H)
    for gx, gy in [(10.0, 10.0), (48.3, 31.7)]:
        col, lev = oracle_mod.foveate(img, gx, gy, 8.0, 20.0, oracle_mod.FOV_MIP)
        inner = np.zeros((H, W), bool)
        inner[4:-4, 4:-4] = True
        assert np.abs(col[inner].astype(np.float64) - img[inner]).max() < 2e-6
        np.testing.assert_array_equal(col[lev == 0], img[lev == 0])
        assert {0, 1, 2} == set(np.unique(lev).tolist())


def test_levels_are_rings_around_the_gaze(oracle_mod):
    W, H = 120, 80
    img = np.zeros((H, W, 3), np.float32)
    spec = synth.StreamSpec(W, H, 4, 1, 12.0, 30.0, 1.0, 2, 3.0)
    for gx, gy in [(33.3, 40.7), (0.0, 0.0), (119.9, 5.2)]:
        _, lev = oracle_mod.foveate(img, gx, gy, 12.0, 30.0)
        want = synth.level_map(spec, gx, gy).numpy()
        xs = np.arange(W) + 0.5 - gx
        ys = np.arange(H) + 0.5 - gy
        d2 = ys[:, None] ** 2 + xs[None, :] ** 2
        safe = (np.abs(d2 - 144.0) > 1e-3) & (np.abs(d2 - 900.0) > 1e-3)
        np.testing.assert_array_equal(lev[safe], want[safe])


@pytest.mark.parametrize("sigma", [1.0, 2.0, 0.7, 5.0])
def test_gaussian_weights(oracle_mod, sigma):
    w = oracle_mod.gauss_weights(sigma).astype(np.float64)
    R = math.ceil(3 * sigma)
    assert len(w) == 2 * R + 1
    d = np.arange(-R, R + 1, dtype=np.float64)
    g = np.exp(-d * d / (2 * sigma * sigma))
    np.testing.assert_allclose(w, g / g.sum(), rtol=2e-6, atol=1e-9)
    assert abs(w.sum() - 1.0) < 1e-6
    np.testing.assert_array_equal(w, w[::-1])


def test_blur_constant_ramp_and_impulse(oracle_mod):
    W, H = 64, 48
    const = np.full((H, W, 3), 0.45, np.float32)
    assert np.abs(oracle_mod.blur(const, 2.0).astype(np.float64) - 0.45).max() < 4e-7
    img = _ramp(W, H)
    out = oracle_mod.blur(img, 2.0)
    assert np.abs(out[8:-8, 8:-8].astype(np.float64) - img[8:-8, 8:-8]).max() < 2e-6
    imp = np.zeros((H, W, 3), np.float32)
    imp[20, 30, 1] = 1.0
    out = oracle_mod.blur(imp, 1.0).astype(np.float64)
    w = oracle_mod.gauss_weights(1.0).astype(np.float64)
    want = np.zeros((H, W))
    want[17:24, 27:34] = np.outer(w, w)
    assert np.abs(out[..., 1] - want).max() < 1e-7
    assert np.all(out[..., 0] == 0) and np.all(out[..., 2] == 0)


def test_gaussian_foveation_selects_the_blurs(oracle_mod):
    W, H = 80, 60
    rng = np.random.Generator(np.random.PCG64(9))
    img = rng.uniform(0, 1, (H, W, 3)).astype(np.float32)
    col, lev = oracle_mod.foveate(img, 40.5, 30.5, 10.0, 25.0, oracle_mod.FOV_GAUSS)
    b1, b2 = oracle_mod.blur(img, 1.0), oracle_mod.blur(img, 2.0)
    np.testing.assert_array_equal(col[lev == 0], img[lev == 0])
    np.testing.assert_array_equal(col[lev == 1], b1[lev == 1])
    np.testing.assert_array_equal(col[lev == 2], b2[lev == 2])
    # blurring removes detail: the periphery has far less variance than the input
    assert col[lev == 2].var() < 0.2 * img[lev == 2].var()


def test_mip_foveation_matches_block_replication_on_the_grid(oracle_mod):
    """Where the bilinear weights vanish in one direction the sample is a plain mip texel: the mip
    texel covering a pixel is the grid-aligned block mean the static workload replicates."""
    W, H = 64, 64
    rng = np.random.Generator(np.random.PCG64(10))
    img = rng.uniform(0, 1, (H, W, 3)).astype(np.float32)
    m1 = oracle_mod.mip_down(img)
    m2 = oracle_mod.mip_down(m1)
    blk2 = img.astype(np.float64).reshape(32, 2, 32, 2, 3).mean(axis=(1, 3))
    blk4 = img.astype(np.float64).reshape(16, 4, 16, 4, 3).mean(axis=(1, 3))
    assert np.abs(m1 - blk2).max() < 2 ** -22
    assert np.abs(m2 - blk4).max() < 2 ** -21
