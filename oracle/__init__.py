"""CPU oracle for per-pixel weighted reservoir sampling (arXiv 2510.03964).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` import this package.  The product package
never imports it, and this package never imports the product package.

The arithmetic lives in ``fwrs_oracle.c`` (plain C, one IEEE binary32 operation
at a time for everything that decides a slot, binary64 for the resolve); this
module only marshals numpy arrays through ctypes.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

from . import build as _build

BIAS_NONE = 0
BIAS_BERNOULLI = 1
BIAS_FULL = 2
BIAS_MEMORYLESS = 3
AES = 4

_lib = None


class Params(C.Structure):
    """Mirror of ``fwrs_oracle_params`` (fwrs_oracle.h)."""

    _fields_ = [
        ("seed", C.c_uint32),
        ("stream_id", C.c_uint32),
        ("fov_deg", C.c_float),
        ("fovea_radius_px", C.c_float),
        ("bias_mode", C.c_uint32),
        ("r_m", C.c_float),
        ("a_k", C.c_float),
        ("r2k", C.c_float),
        ("rek", C.c_float),
        ("lambda_decay", C.c_float),
    ]


def _ptr(a: np.ndarray, ctype):
    return a.ctypes.data_as(C.POINTER(ctype))


def lib(path: str | None = None):
    """Load (building if needed) the oracle shared library."""
    global _lib
    if path is not None:
        return _bind(C.CDLL(path))
    if _lib is None:
        override = os.environ.get("FWRS_ORACLE_LIB")   # a variant built by the mutation tests
        if override:
            _lib = _bind(C.CDLL(override))
            return _lib
        p = _build.LIB
        if not os.path.exists(p) or os.path.getmtime(p) < os.path.getmtime(_build.SRC):
            _build.build(force=True)
        _lib = _bind(C.CDLL(p))
    return _lib


def _bind(L):
    vp = C.c_void_p
    L.fwrs_oracle_default_params.argtypes = [C.c_int, C.POINTER(Params)]
    L.fwrs_oracle_create.argtypes = [C.c_int, C.c_int, C.c_int, C.POINTER(Params)]
    L.fwrs_oracle_create.restype = vp
    L.fwrs_oracle_destroy.argtypes = [vp]
    L.fwrs_oracle_push.argtypes = [vp, C.POINTER(C.c_float), C.POINTER(C.c_uint8), C.c_float, C.c_float]
    L.fwrs_oracle_push_rows.argtypes = [vp, C.POINTER(C.c_float), C.POINTER(C.c_uint8), C.c_float, C.c_float,
                                        C.c_int, C.c_int]
    L.fwrs_oracle_advance.argtypes = [vp]
    L.fwrs_oracle_resolve.argtypes = [vp, C.POINTER(C.c_double)]
    L.fwrs_oracle_resolve_rows.argtypes = [vp, C.POINTER(C.c_double), C.c_int, C.c_int]
    L.fwrs_oracle_frame_index.argtypes = [vp]
    L.fwrs_oracle_frame_index.restype = C.c_uint32
    L.fwrs_oracle_constants.argtypes = [vp, C.POINTER(C.c_float)]
    L.fwrs_oracle_state.argtypes = [vp, C.POINTER(C.c_float), C.POINTER(C.c_uint32), C.POINTER(C.c_float),
                                    C.POINTER(C.c_uint32), C.POINTER(C.c_float)]
    L.fwrs_oracle_philox_many.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_uint32),
                                          C.POINTER(C.c_uint32), C.c_size_t]
    L.fwrs_oracle_exp2p_many.argtypes = [C.POINTER(C.c_float), C.POINTER(C.c_float), C.c_size_t]
    L.fwrs_oracle_cbrt_many.argtypes = [C.POINTER(C.c_float), C.POINTER(C.c_float), C.c_size_t]
    L.fwrs_oracle_lab_many.argtypes = [C.POINTER(C.c_float), C.POINTER(C.c_float), C.c_size_t]
    L.fwrs_oracle_de94_many.argtypes = [C.POINTER(C.c_float), C.POINTER(C.c_float), C.POINTER(C.c_float),
                                        C.c_size_t]
    L.fwrs_oracle_slot_sums.argtypes = [vp, C.POINTER(C.c_float)]
    L.fwrs_oracle_density_many.argtypes = [vp, C.POINTER(C.c_float), C.POINTER(C.c_float), C.c_size_t]
    L.fwrs_oracle_eccentricity.argtypes = [vp, C.c_int, C.c_int, C.c_float, C.c_float]
    L.fwrs_oracle_eccentricity.restype = C.c_float
    L.fwrs_oracle_weight.argtypes = [vp, C.c_int, C.c_int, C.c_uint8, C.c_float, C.c_float]
    L.fwrs_oracle_weight.restype = C.c_float
    L.fwrs_oracle_weight_image.argtypes = [vp, C.POINTER(C.c_uint8), C.c_float, C.c_float,
                                           C.POINTER(C.c_float)]
    L.fwrs_oracle_trials.argtypes = [C.c_int, C.c_int, C.c_int, C.POINTER(Params), C.c_int, C.c_int,
                                     C.c_uint32, C.c_int, C.c_int, C.POINTER(C.c_float),
                                     C.POINTER(C.c_uint8), C.POINTER(C.c_float), C.POINTER(C.c_uint32),
                                     C.POINTER(C.c_float)]
    L.fwrs_oracle_trials.restype = C.c_int
    L.fwrs_oracle_push_reproject.argtypes = [vp, C.POINTER(C.c_float), C.POINTER(C.c_uint8), C.POINTER(C.c_float),
                                             C.POINTER(C.c_float), C.c_float, C.c_float, C.c_float]
    L.fwrs_oracle_push_reproject.restype = C.c_int
    L.fwrs_oracle_depth.argtypes = [vp, C.POINTER(C.c_float)]
    fp = C.POINTER(C.c_float)
    L.fwrs_oracle_foveate.argtypes = [fp, C.c_int, C.c_int, C.c_float, C.c_float, C.c_float, C.c_float, C.c_uint32,
                                      fp, C.POINTER(C.c_uint8)]
    L.fwrs_oracle_foveate.restype = C.c_int
    L.fwrs_oracle_mip_down.argtypes = [fp, C.c_int, C.c_int, fp]
    L.fwrs_oracle_gauss_weights.argtypes = [C.c_float, fp]
    L.fwrs_oracle_gauss_weights.restype = C.c_int
    L.fwrs_oracle_blur.argtypes = [fp, C.c_int, C.c_int, C.c_float, fp, fp]
    L.fwrs_oracle_log2u_many.argtypes = [C.POINTER(C.c_uint32), C.POINTER(C.c_float), C.c_size_t]
    L.fwrs_oracle_decay.argtypes = [vp]
    L.fwrs_oracle_decay.restype = C.c_float
    L.fwrs_oracle_flushes.argtypes = [vp]
    L.fwrs_oracle_flushes.restype = C.c_uint64
    return L


def default_params(width: int, **overrides) -> Params:
    p = Params()
    lib().fwrs_oracle_default_params(int(width), C.byref(p))
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


@dataclass
class State:
    wsum: np.ndarray   # [H, W] float32
    cnt: np.ndarray    # [H, W] uint32
    wt: np.ndarray     # [k, H, W] float32
    idx: np.ndarray    # [k, H, W] uint32
    col: np.ndarray    # [k, 3, H, W] float32
    wslot: np.ndarray  # [k, H, W] float32 per-slot w_sum (the shared w_sum k times unless BIAS_FULL)


class Oracle:
    """One pixel-stream context of the oracle (a width x height image, k slots)."""

    def __init__(self, width: int, height: int, k: int, params: Params | None = None, library=None):
        self._L = library or lib()
        self.width, self.height, self.k = int(width), int(height), int(k)
        self.params = params if params is not None else default_params(width)
        h = self._L.fwrs_oracle_create(self.width, self.height, self.k, C.byref(self.params))
        if not h:
            raise ValueError(f"oracle create failed for {width}x{height} k={k}")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            self._L.fwrs_oracle_destroy(self._h)
            self._h = None

    __del__ = close

    @property
    def t(self) -> int:
        return int(self._L.fwrs_oracle_frame_index(self._h))

    def push(self, color: np.ndarray, level: np.ndarray, gx: float, gy: float) -> None:
        color = np.ascontiguousarray(color, dtype=np.float32)
        level = np.ascontiguousarray(level, dtype=np.uint8)
        assert color.shape == (self.height, self.width, 3) and level.shape == (self.height, self.width)
        self._L.fwrs_oracle_push(self._h, _ptr(color, C.c_float), _ptr(level, C.c_uint8),
                                 C.c_float(gx), C.c_float(gy))

    def push_rows(self, color: np.ndarray, level: np.ndarray, gx: float, gy: float, y0: int, y1: int) -> None:
        """Update only rows [y0, y1) of the frame (the frame index does not advance; call advance())."""
        color = np.ascontiguousarray(color, dtype=np.float32)
        level = np.ascontiguousarray(level, dtype=np.uint8)
        assert color.shape == (self.height, self.width, 3) and level.shape == (self.height, self.width)
        self._L.fwrs_oracle_push_rows(self._h, _ptr(color, C.c_float), _ptr(level, C.c_uint8),
                                      C.c_float(gx), C.c_float(gy), int(y0), int(y1))

    def advance(self) -> None:
        self._L.fwrs_oracle_advance(self._h)

    def push_reproject(self, color: np.ndarray, level: np.ndarray, motion: np.ndarray, depth: np.ndarray,
                       gx: float, gy: float, depth_tol: float) -> None:
        """One frame with reverse reprojection by `motion` ([H, W, 2], pixels, current minus previous
        position) and the depth-based flush (`depth` [H, W], relative tolerance `depth_tol`)."""
        color = np.ascontiguousarray(color, dtype=np.float32)
        level = np.ascontiguousarray(level, dtype=np.uint8)
        motion = np.ascontiguousarray(motion, dtype=np.float32)
        depth = np.ascontiguousarray(depth, dtype=np.float32)
        H, W = self.height, self.width
        assert color.shape == (H, W, 3) and level.shape == (H, W) and motion.shape == (H, W, 2)
        assert depth.shape == (H, W)
        rc = self._L.fwrs_oracle_push_reproject(self._h, _ptr(color, C.c_float), _ptr(level, C.c_uint8),
                                                _ptr(motion, C.c_float), _ptr(depth, C.c_float), C.c_float(gx),
                                                C.c_float(gy), C.c_float(depth_tol))
        if rc != 0:
            raise MemoryError("oracle reprojection: out of memory")

    def depth(self) -> np.ndarray:
        out = np.empty((self.height, self.width), np.float32)
        self._L.fwrs_oracle_depth(self._h, _ptr(out, C.c_float))
        return out

    @property
    def flushes(self) -> int:
        return int(self._L.fwrs_oracle_flushes(self._h))

    def resolve(self) -> np.ndarray:
        out = np.empty((self.height, self.width, 3), dtype=np.float64)
        self._L.fwrs_oracle_resolve(self._h, _ptr(out, C.c_double))
        return out

    def resolve_rows(self, out: np.ndarray, y0: int, y1: int) -> None:
        """Rows [y0, y1) of the resolve into `out` ([H, W, 3] float64, C-contiguous)."""
        assert out.shape == (self.height, self.width, 3) and out.dtype == np.float64 and out.flags.c_contiguous
        self._L.fwrs_oracle_resolve_rows(self._h, _ptr(out, C.c_double), int(y0), int(y1))

    def state(self) -> State:
        H, W, k = self.height, self.width, self.k
        s = State(np.empty((H, W), np.float32), np.empty((H, W), np.uint32), np.empty((k, H, W), np.float32),
                  np.empty((k, H, W), np.uint32), np.empty((k, 3, H, W), np.float32), np.empty((k, H, W), np.float32))
        self._L.fwrs_oracle_state(self._h, _ptr(s.wsum, C.c_float), _ptr(s.cnt, C.c_uint32),
                                  _ptr(s.wt, C.c_float), _ptr(s.idx, C.c_uint32), _ptr(s.col, C.c_float))
        self._L.fwrs_oracle_slot_sums(self._h, _ptr(s.wslot, C.c_float))
        return s

    @property
    def decay(self) -> np.float32:
        return np.float32(self._L.fwrs_oracle_decay(self._h))

    def constants(self) -> dict:
        out = np.empty(9, np.float32)
        self._L.fwrs_oracle_constants(self._h, _ptr(out, C.c_float))
        names = ["A", "B", "IR2", "IRM", "C", "ppd", "iPPD", "rf", "Drf"]
        return {n: np.float32(v) for n, v in zip(names, out)}

    def density(self, e: np.ndarray) -> np.ndarray:
        e = np.ascontiguousarray(e, dtype=np.float32)
        out = np.empty_like(e)
        self._L.fwrs_oracle_density_many(self._h, _ptr(e, C.c_float), _ptr(out, C.c_float), e.size)
        return out

    def eccentricity(self, x: int, y: int, gx: float, gy: float) -> np.float32:
        return np.float32(self._L.fwrs_oracle_eccentricity(self._h, int(x), int(y), C.c_float(gx), C.c_float(gy)))

    def weight(self, x: int, y: int, level: int, gx: float, gy: float) -> np.float32:
        return np.float32(self._L.fwrs_oracle_weight(self._h, int(x), int(y), int(level),
                                                     C.c_float(gx), C.c_float(gy)))

    def weight_image(self, level: np.ndarray, gx: float, gy: float) -> np.ndarray:
        level = np.ascontiguousarray(level, dtype=np.uint8)
        out = np.empty((self.height, self.width), np.float32)
        self._L.fwrs_oracle_weight_image(self._h, _ptr(level, C.c_uint8), C.c_float(gx), C.c_float(gy),
                                         _ptr(out, C.c_float))
        return out


def philox(keys: np.ndarray, ctrs: np.ndarray) -> np.ndarray:
    """Philox4x32-10 blocks: keys [n, 2] uint32, counters [n, 4] uint32 -> [n, 4] uint32."""
    keys = np.ascontiguousarray(keys, dtype=np.uint32)
    ctrs = np.ascontiguousarray(ctrs, dtype=np.uint32)
    n = ctrs.shape[0]
    out = np.empty((n, 4), np.uint32)
    lib().fwrs_oracle_philox_many(_ptr(keys, C.c_uint32), _ptr(ctrs, C.c_uint32), _ptr(out, C.c_uint32), n)
    return out


FOV_MIP = 0
FOV_GAUSS = 1


def foveate(full: np.ndarray, gx: float, gy: float, r0: float, r1: float, mode: int = FOV_MIP):
    """Foveated frame [H, W, 3] float32 and level map [H, W] uint8 from a full frame [H, W, 3]."""
    full = np.ascontiguousarray(full, dtype=np.float32)
    H, W, _ = full.shape
    color = np.empty_like(full)
    level = np.empty((H, W), np.uint8)
    rc = lib().fwrs_oracle_foveate(_ptr(full, C.c_float), W, H, C.c_float(gx), C.c_float(gy), C.c_float(r0),
                                   C.c_float(r1), int(mode), _ptr(color, C.c_float), _ptr(level, C.c_uint8))
    if rc != 0:
        raise ValueError(f"oracle foveate failed ({rc})")
    return color, level


def mip_down(img: np.ndarray) -> np.ndarray:
    img = np.ascontiguousarray(img, dtype=np.float32)
    H, W, _ = img.shape
    out = np.empty(((H + 1) // 2, (W + 1) // 2, 3), np.float32)
    lib().fwrs_oracle_mip_down(_ptr(img, C.c_float), W, H, _ptr(out, C.c_float))
    return out


def gauss_weights(sigma: float) -> np.ndarray:
    w = np.empty(65, np.float32)
    R = lib().fwrs_oracle_gauss_weights(C.c_float(sigma), _ptr(w, C.c_float))
    if R < 0:
        raise ValueError("radius too large")
    return w[:2 * R + 1].copy()


def blur(img: np.ndarray, sigma: float) -> np.ndarray:
    img = np.ascontiguousarray(img, dtype=np.float32)
    H, W, _ = img.shape
    tmp = np.empty_like(img)
    out = np.empty_like(img)
    lib().fwrs_oracle_blur(_ptr(img, C.c_float), W, H, C.c_float(sigma), _ptr(tmp, C.c_float),
                           _ptr(out, C.c_float))
    return out


def log2u(bits: np.ndarray) -> np.ndarray:
    """log2 of the uniform variate ((bits >> 8) + 1) * 2^-24 (binary32), as A-ES uses it."""
    bits = np.ascontiguousarray(bits, dtype=np.uint32)
    out = np.empty(bits.shape, np.float32)
    lib().fwrs_oracle_log2u_many(_ptr(bits, C.c_uint32), _ptr(out, C.c_float), bits.size)
    return out


def cbrt(t: np.ndarray) -> np.ndarray:
    t = np.ascontiguousarray(t, dtype=np.float32)
    out = np.empty_like(t)
    lib().fwrs_oracle_cbrt_many(_ptr(t, C.c_float), _ptr(out, C.c_float), t.size)
    return out


def lab(rgb: np.ndarray) -> np.ndarray:
    """Linear RGB [..., 3] -> CIE Lab [..., 3] (D65), binary32."""
    rgb = np.ascontiguousarray(rgb, dtype=np.float32)
    out = np.empty_like(rgb)
    lib().fwrs_oracle_lab_many(_ptr(rgb, C.c_float), _ptr(out, C.c_float), rgb.size // 3)
    return out


def de94(ref_lab: np.ndarray, x_lab: np.ndarray) -> np.ndarray:
    ref_lab = np.ascontiguousarray(ref_lab, dtype=np.float32)
    x_lab = np.ascontiguousarray(x_lab, dtype=np.float32)
    out = np.empty(ref_lab.size // 3, np.float32)
    lib().fwrs_oracle_de94_many(_ptr(ref_lab, C.c_float), _ptr(x_lab, C.c_float), _ptr(out, C.c_float), out.size)
    return out


def exp2p(y: np.ndarray) -> np.ndarray:
    y = np.ascontiguousarray(y, dtype=np.float32)
    out = np.empty_like(y)
    lib().fwrs_oracle_exp2p_many(_ptr(y, C.c_float), _ptr(out, C.c_float), y.size)
    return out


def trials(width: int, height: int, k: int, params: Params, px: int, py: int, seed0: int, n_trials: int,
           rgb: np.ndarray, lev: np.ndarray, gaze: np.ndarray, library=None):
    """Final slot frame indices [n_trials, k] (and final w_sum [n_trials]) of the single stream at
    pixel (px, py), repeated with Philox seeds seed0, seed0 + 1, ..."""
    L = library or lib()
    rgb = np.ascontiguousarray(rgb, dtype=np.float32).reshape(-1, 3)
    lev = np.ascontiguousarray(lev, dtype=np.uint8).reshape(-1)
    gaze = np.ascontiguousarray(gaze, dtype=np.float32).reshape(-1, 2)
    n_frames = lev.size
    assert rgb.shape[0] == n_frames and gaze.shape[0] == n_frames
    idx = np.empty((n_trials, k), np.uint32)
    wsum = np.empty(n_trials, np.float32)
    rc = L.fwrs_oracle_trials(width, height, k, C.byref(params), px, py, seed0, n_trials, n_frames,
                              _ptr(rgb, C.c_float), _ptr(lev, C.c_uint8), _ptr(gaze, C.c_float),
                              _ptr(idx, C.c_uint32), _ptr(wsum, C.c_float))
    if rc != 0:
        raise ValueError(f"oracle trials failed ({rc})")
    return idx, wsum
