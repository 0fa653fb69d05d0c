"""Seeded frame sequences whose colours repeat from frame to frame, drawn from a
palette of edge values: signed zeros, a denormal, the values on both sides of
2^24, and magnitudes whose Lab (linear RGB -> XYZ -> Lab) is not finite.

Used by the Eq. 7 parity tests: a reservoir sample whose colour equals the new
pixel's is a case the kernels treat on their own, and these frames put such
samples beside unequal ones in the same waves.  No method arithmetic here."""
from __future__ import annotations

import numpy as np
import torch

PALETTE = np.array([0.0, -0.0, 0.25, 1.0, 7.5e-3, 1e-40, -0.5, 16777215.0, 16777216.0, 3.0e7, -3.0e7,
                    1e30, -1e30], np.float32)


def palette_frames(width: int, height: int, n: int, device, seed: int = 5, p_change: float = 0.3):
    """n frames of (colour [H, W, 3] f32, level [H, W] u8, gaze x, gaze y) on `device`.

    The left half of the image keeps its colours for the whole sequence (up to the
    sign of zeros, redrawn every frame); on the right half each pixel redraws its
    colour with probability p_change per frame.  Levels are fixed, random in 0..2."""
    rng = np.random.default_rng(seed)
    idx = rng.integers(0, len(PALETTE), size=(height, width, 3))
    level = torch.from_numpy(rng.integers(0, 3, size=(height, width)).astype(np.uint8)).to(device)
    gx, gy = 0.37 * width, 0.55 * height
    frames = []
    for _ in range(n):
        change = rng.random((height, width, 1)) < p_change
        change[:, : width // 2] = False
        idx = np.where(change, rng.integers(0, len(PALETTE), size=(height, width, 3)), idx)
        c = PALETTE[idx]
        zero = c == 0.0
        c[zero] = np.where(rng.random(int(zero.sum())) < 0.5, np.float32(-0.0), np.float32(0.0))
        frames.append((torch.from_numpy(np.ascontiguousarray(c)).to(device), level, gx, gy))
    return frames


def resolve_scale(col: np.ndarray) -> np.ndarray:
    """Per pixel, max(1, largest |colour| among its slots) from an oracle state's col [k, 3, H, W]:
    the scale of the binary32 rounding of a resolve over those slots."""
    return np.maximum(1.0, np.abs(col.astype(np.float64)).max(axis=(0, 1)))
