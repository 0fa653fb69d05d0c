"""Seeded synthetic inputs shaped like the paper's workload.

The paper evaluates on Unity scenes rendered with a foveation post-process and
on eye-tracker scanpaths (Sec. 4.3, 5.3); none of those assets exist here.
This module stands in for them with:

* a static procedural scene per stream: 8 random plane waves per RGB channel
  plus an 8-pixel checkerboard, values in [0, 1];
* a foveation simulation with three concentric levels around the gaze: full
  resolution inside the foveal radius (level 0), grid-aligned 2x2 block means
  out to 2.5 foveal radii (level 1), grid-aligned 4x4 block means beyond
  (level 2); the same "render at reduced resolution and replicate" model the
  paper's mipmap foveation is equivalent to (Sec. 4.3);
* a gaze trace: fixation with per-frame Gaussian microsaccade jitter and a
  saccade to a uniform random target with Gaussian landing scatter every P
  frames (Sec. 2.1.2 describes both eye movements);
* for a moving camera (the lateral back-and-forth motion of Sec. 5.3), a
  panning view of the same procedural scene with a textured foreground disc
  moving at its own speed in front of it, with per-pixel motion vectors and
  depth (MovingSource).

It holds none of the reservoir method's arithmetic and is used by both the
GPU path's callers and the oracle's tests: random numbers come only from
numpy's PCG64 with fixed seeds, scene values are computed in float64 and
stored as float32.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch

#: Philox key word 0 used by every workload.
PHILOX_SEED = 0x25103964
#: Horizontal field of view covered by the image width (degrees).
FOV_DEG = 70.0


@dataclass(frozen=True)
class StreamSpec:
    """One pixel-stream workload: image size, slots, trace length and the
    foveation / gaze model parameters (pixels)."""

    width: int
    height: int
    k: int
    frames: int
    fovea_radius_px: float
    ring_radius_px: float
    sigma_micro: float
    saccade_period: int
    sigma_landing: float
    stream_id: int = 0

    @property
    def pixels(self) -> int:
        return self.width * self.height


def _scaled(width: int, height: int, k: int, frames: int, rf: float, stream_id: int) -> StreamSpec:
    """4K gaze-model values (sigma 8, period 90, scatter 24) scaled by width / 3840."""
    s = width / 3840.0
    return StreamSpec(width, height, k, frames, rf, 2.5 * rf, 8.0 * s, 90, 24.0 * s, stream_id)


def spec_small(stream_id: int = 0) -> StreamSpec:
    """256x256, k=4, 60 frames; fovea 32 px, ring 80 px; jitter 2 px, saccade
    every 20 frames, landing scatter 6 px (the CPU-fast single-stream case)."""
    return StreamSpec(256, 256, 4, 60, 32.0, 80.0, 2.0, 20, 6.0, stream_id)


def spec_4k(stream_id: int = 0, frames: int = 600) -> StreamSpec:
    """3840x2160, k=4, 600 frames; fovea 216 px, ring 540 px; jitter 8 px,
    saccade every 90 frames, landing scatter 24 px (the 4K headline case)."""
    return StreamSpec(3840, 2160, 4, frames, 216.0, 540.0, 8.0, 90, 24.0, stream_id)


def spec_stereo(frames: int = 900) -> tuple[StreamSpec, StreamSpec]:
    """Two eyes of 2064x2208, k=8, 900 frames, fovea 5% of width (103 px)."""
    left = _scaled(2064, 2208, 8, frames, 103.0, 0)
    right = _scaled(2064, 2208, 8, frames, 103.0, 1)
    return left, right


def spec_uneven(frames: int = 300, seed: int = 77) -> list[StreamSpec]:
    """16 streams, 4 each of 1280x720, 1920x1080, 2560x1440, 3840x2160, with k
    drawn from {2, 4, 8} and a fovea of 5% of width."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = [(1280, 720), (1920, 1080), (2560, 1440), (3840, 2160)]
    out = []
    sid = 0
    for (w, h) in sizes:
        for _ in range(4):
            k = int(rng.choice([2, 4, 8]))
            out.append(_scaled(w, h, k, frames, 0.05 * w, sid))
            sid += 1
    return out


# --------------------------------------------------------------------------
# Scene
# --------------------------------------------------------------------------
def scene(width: int, height: int, stream_id: int = 0, device="cpu") -> torch.Tensor:
    """Static procedural scene [H, W, 3] float32 in [0, 1].

    Per channel, S is the mean of 8 plane waves sin(2 pi f (u cos th + v sin th)
    / 256 + phi) over pixel centres (u, v), with th ~ U[0, pi), f ~ U[0.5, 16]
    cycles per 256 px, phi ~ U[0, 2 pi); C is a +-1 checkerboard of 8-px squares
    whose seeded offset is not aligned to the 4-px block grid.  Value =
    0.5 + 0.35 S + 0.15 C, computed in float64 (seed 1000 + stream_id)."""
    rng = np.random.Generator(np.random.PCG64(1000 + stream_id))
    theta = rng.uniform(0.0, math.pi, size=(3, 8))
    freq = rng.uniform(0.5, 16.0, size=(3, 8))
    phase = rng.uniform(0.0, 2.0 * math.pi, size=(3, 8))
    off = rng.choice([1, 2, 3, 5, 6, 7], size=2)
    dev = torch.device(device)
    u = torch.arange(width, dtype=torch.float64, device=dev) + 0.5
    v = torch.arange(height, dtype=torch.float64, device=dev) + 0.5
    out = torch.empty((height, width, 3), dtype=torch.float32, device=dev)
    xi = torch.arange(width, device=dev, dtype=torch.int64)
    yi = torch.arange(height, device=dev, dtype=torch.int64)
    cx = torch.div(xi + int(off[0]), 8, rounding_mode="floor")
    cy = torch.div(yi + int(off[1]), 8, rounding_mode="floor")
    checker = torch.where(((cy[:, None] + cx[None, :]) % 2) == 0, 1.0, -1.0).to(torch.float64)
    for c in range(3):
        acc = torch.zeros((height, width), dtype=torch.float64, device=dev)
        for i in range(8):
            kx = 2.0 * math.pi * freq[c, i] * math.cos(theta[c, i]) / 256.0
            ky = 2.0 * math.pi * freq[c, i] * math.sin(theta[c, i]) / 256.0
            acc += torch.sin((v * ky)[:, None] + (u * kx)[None, :] + phase[c, i])
        s = acc / 8.0
        out[:, :, c] = (0.5 + 0.35 * s + 0.15 * checker).to(torch.float32)
    return out


def block_mean(img: torch.Tensor, b: int) -> torch.Tensor:
    """Grid-aligned b x b block means of an [H, W, 3] float32 image, replicated
    back to full size (a reduced-resolution render, upsampled by replication).
    Partial blocks at the right and bottom edges average their in-image pixels.
    Means are taken in float64 and rounded to float32."""
    H, W, _ = img.shape
    x = img.to(torch.float64).permute(2, 0, 1).unsqueeze(0)
    m = torch.nn.functional.avg_pool2d(x, kernel_size=b, stride=b, ceil_mode=True)
    m = m.repeat_interleave(b, dim=2).repeat_interleave(b, dim=3)[:, :, :H, :W]
    return m[0].permute(1, 2, 0).to(torch.float32).contiguous()


@dataclass
class FoveatedScene:
    """The three precomputed renderings of a static scene: full resolution,
    1/2 resolution (2x2 means) and 1/4 resolution (4x4 means)."""

    full: torch.Tensor
    half: torch.Tensor
    quarter: torch.Tensor
    stack: torch.Tensor = field(init=False)

    def __post_init__(self):
        self.stack = torch.stack([self.full, self.half, self.quarter])  # [3, H, W, 3]


def foveated_scene(spec: StreamSpec, device="cpu") -> FoveatedScene:
    full = scene(spec.width, spec.height, spec.stream_id, device="cpu")
    fs = FoveatedScene(full, block_mean(full, 2), block_mean(full, 4))
    if str(device) != "cpu":
        fs = FoveatedScene(fs.full.to(device), fs.half.to(device), fs.quarter.to(device))
    return fs


# --------------------------------------------------------------------------
# Gaze
# --------------------------------------------------------------------------
def gaze_trace(spec: StreamSpec, n_frames: int | None = None) -> np.ndarray:
    """Gaze points [n, 2] float32 in continuous pixel coordinates.

    Fixation f0 ~ U over the central 60% of the image; g_t = f + N(0, s_m^2)
    per frame; every `saccade_period` frames the fixation jumps to a uniform
    random target plus N(0, s_l^2) landing scatter.  Clamped to the image.
    Seed 2000 + stream_id."""
    n = spec.frames if n_frames is None else n_frames
    rng = np.random.Generator(np.random.PCG64(2000 + spec.stream_id))
    W, H = float(spec.width), float(spec.height)
    fix = np.array([rng.uniform(0.2 * W, 0.8 * W), rng.uniform(0.2 * H, 0.8 * H)])
    out = np.empty((n, 2), dtype=np.float64)
    for t in range(n):
        if t > 0 and t % spec.saccade_period == 0:
            target = np.array([rng.uniform(0.0, W), rng.uniform(0.0, H)])
            fix = target + rng.normal(0.0, spec.sigma_landing, size=2)
            fix = np.clip(fix, [0.0, 0.0], [W, H])
        g = fix + rng.normal(0.0, spec.sigma_micro, size=2)
        out[t] = np.clip(g, [0.0, 0.0], [W, H])
    return out.astype(np.float32)


def vergence_shift(seed: int = 3000) -> float:
    """Horizontal offset (px) of the right eye's gaze, drawn once from U[0, 12]."""
    return float(np.random.Generator(np.random.PCG64(seed)).uniform(0.0, 12.0))


# --------------------------------------------------------------------------
# Frames
# --------------------------------------------------------------------------
def level_map(spec: StreamSpec, gx: float, gy: float, device="cpu") -> torch.Tensor:
    """Foveation level per pixel [H, W] uint8 from the squared distance of the
    pixel centre to the gaze: <= r_f^2 -> 0, <= ring^2 -> 1, else 2 (float64)."""
    dev = torch.device(device)
    u = torch.arange(spec.width, dtype=torch.float64, device=dev) + 0.5 - float(gx)
    v = torch.arange(spec.height, dtype=torch.float64, device=dev) + 0.5 - float(gy)
    d2 = (v * v)[:, None] + (u * u)[None, :]
    lev = torch.full((spec.height, spec.width), 2, dtype=torch.uint8, device=dev)
    lev[d2 <= spec.ring_radius_px * spec.ring_radius_px] = 1
    lev[d2 <= spec.fovea_radius_px * spec.fovea_radius_px] = 0
    return lev


def foveated_frame(fs: FoveatedScene, level: torch.Tensor) -> torch.Tensor:
    """Select the rendering each pixel was drawn at: [H, W, 3] float32."""
    idx = level.to(torch.int64)[None, :, :, None].expand(1, -1, -1, 3)
    return torch.gather(fs.stack, 0, idx)[0].contiguous()


class FrameSource:
    """Frames of one stream: (colour [H, W, 3] f32, level [H, W] u8, gx, gy)."""

    def __init__(self, spec: StreamSpec, device="cpu", gaze: np.ndarray | None = None,
                 n_frames: int | None = None):
        self.spec = spec
        self.device = device
        self.fs = foveated_scene(spec, device)
        self.gaze = gaze if gaze is not None else gaze_trace(spec, n_frames)

    def __len__(self) -> int:
        return len(self.gaze)

    def frame(self, t: int):
        gx, gy = float(self.gaze[t, 0]), float(self.gaze[t, 1])
        lev = level_map(self.spec, gx, gy, self.device)
        return foveated_frame(self.fs, lev), lev, gx, gy

    def __iter__(self):
        for t in range(len(self)):
            yield self.frame(t)


# --------------------------------------------------------------------------
# Moving camera
# --------------------------------------------------------------------------
@dataclass(frozen=True)
class MotionSpec:
    """Lateral back-and-forth camera motion and one moving occluder (pixels, frames).

    The camera offset is c(t) = pan_amp sin(2 pi t / pan_period): pixel u of
    frame t shows scene point u + c(t).  A disc of radius disc_radius (depth
    disc_depth) centred at (W/2 + disc_amp sin(2 pi t / disc_period + 1), 0.55 H)
    carries its own texture; the background's depth is bg_depth (1 + 0.05
    sin(2 pi v / H)).  Both periods divide `period`, so frame t and frame
    t + period are identical and a ring of `period` frames loops seamlessly."""

    pan_amp: float
    pan_period: int
    disc_radius: float
    disc_amp: float
    disc_period: int
    disc_depth: float = 3.0
    bg_depth: float = 10.0

    @property
    def period(self) -> int:
        return math.lcm(self.pan_period, self.disc_period)


def motion_for(spec: StreamSpec) -> MotionSpec:
    """Motion scaled by the image width: the pan swings 4% of the width (at 4K up to
    about 4 px per frame over a 240-frame back-and-forth), the disc (6% of the width
    in radius) swings 25% of the width over 120 frames."""
    W = float(spec.width)
    return MotionSpec(0.04 * W, 240, 0.06 * W, 0.25 * W, 120)


def _waves(rng):
    theta = rng.uniform(0.0, math.pi, size=(3, 8))
    freq = rng.uniform(0.5, 16.0, size=(3, 8))
    phase = rng.uniform(0.0, 2.0 * math.pi, size=(3, 8))
    off = rng.choice([1, 2, 3, 5, 6, 7], size=2)
    return theta, freq, phase, off


def _texture(waves, X: torch.Tensor, Y: torch.Tensor) -> torch.Tensor:
    """The procedural texture of scene() at continuous coordinates (float64 [H, W] each),
    [H, W, 3] float64."""
    theta, freq, phase, off = waves
    cx = torch.floor((X + float(off[0])) / 8.0)
    cy = torch.floor((Y + float(off[1])) / 8.0)
    checker = torch.where(torch.remainder(cx + cy, 2.0) == 0.0, 1.0, -1.0).to(torch.float64)
    out = torch.empty(X.shape + (3,), dtype=torch.float64, device=X.device)
    for c in range(3):
        acc = torch.zeros_like(X)
        for i in range(8):
            kx = 2.0 * math.pi * freq[c, i] * math.cos(theta[c, i]) / 256.0
            ky = 2.0 * math.pi * freq[c, i] * math.sin(theta[c, i]) / 256.0
            acc += torch.sin(Y * ky + X * kx + phase[c, i])
        out[..., c] = 0.5 + 0.35 * (acc / 8.0) + 0.15 * checker
    return out


class MovingSource:
    """Frames of one stream under camera and object motion:
    (colour [H, W, 3] f32, level [H, W] u8, motion [H, W, 2] f32, depth [H, W] f32, gx, gy).

    Frame t renders the panned background and the disc at full resolution (float64), takes
    grid-aligned 2x2 and 4x4 block means of that frame for the reduced levels, and selects by
    the level map of gaze t (as FrameSource).  Motion vectors are the displacement of each
    pixel's surface point since frame t - 1 (current minus previous position): c(t-1) - c(t)
    horizontally on the background, the disc's own displacement inside it.  Background texture
    seed 1000 + stream_id, disc texture seed 1500 + stream_id; gaze as FrameSource."""

    def __init__(self, spec: StreamSpec, motion: MotionSpec | None = None, device="cpu",
                 gaze: np.ndarray | None = None, n_frames: int | None = None):
        self.spec = spec
        self.motion = motion or motion_for(spec)
        self.device = torch.device(device)
        self.gaze = gaze if gaze is not None else gaze_trace(spec, n_frames)
        self._bg = _waves(np.random.Generator(np.random.PCG64(1000 + spec.stream_id)))
        self._disc = _waves(np.random.Generator(np.random.PCG64(1500 + spec.stream_id)))
        dev = self.device
        self._u = (torch.arange(spec.width, dtype=torch.float64, device=dev) + 0.5)[None, :].expand(spec.height, -1)
        self._v = (torch.arange(spec.height, dtype=torch.float64, device=dev) + 0.5)[:, None].expand(-1, spec.width)

    def __len__(self) -> int:
        return len(self.gaze)

    def pan(self, t: int) -> float:
        m = self.motion
        return m.pan_amp * math.sin(2.0 * math.pi * t / m.pan_period)

    def disc_x(self, t: int) -> float:
        m = self.motion
        return 0.5 * self.spec.width + m.disc_amp * math.sin(2.0 * math.pi * t / m.disc_period + 1.0)

    def render(self, t: int):
        """Full-resolution colour [H, W, 3] f32, motion [H, W, 2] f32 and depth [H, W] f32."""
        m, spec = self.motion, self.spec
        u, v = self._u, self._v
        c, c_prev = self.pan(t), self.pan(t - 1)
        ox, ox_prev = self.disc_x(t), self.disc_x(t - 1)
        oy = 0.55 * spec.height
        inside = (u - ox) ** 2 + (v - oy) ** 2 <= m.disc_radius ** 2
        bg = _texture(self._bg, u + c, v)
        disc = _texture(self._disc, u - ox, v - oy)
        colour = torch.where(inside[..., None], disc, bg).to(torch.float32)
        mv = torch.zeros((spec.height, spec.width, 2), dtype=torch.float64, device=self.device)
        mv[..., 0] = torch.where(inside, ox - ox_prev, c_prev - c)
        depth = torch.where(inside, torch.full_like(u, m.disc_depth),
                            m.bg_depth * (1.0 + 0.05 * torch.sin(2.0 * math.pi * v / spec.height)))
        return colour.contiguous(), mv.to(torch.float32).contiguous(), depth.to(torch.float32).contiguous()

    def frame(self, t: int):
        gx, gy = float(self.gaze[t, 0]), float(self.gaze[t, 1])
        full, mv, depth = self.render(t)
        fs = FoveatedScene(full, block_mean(full, 2), block_mean(full, 4))
        lev = level_map(self.spec, gx, gy, self.device)
        return foveated_frame(fs, lev), lev, mv, depth, gx, gy

    def __iter__(self):
        for t in range(len(self)):
            yield self.frame(t)
