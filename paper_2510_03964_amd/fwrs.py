"""Python binding of the C ABI in include/fwrs.h (ctypes; argument marshalling only).

Torch tensors supply device memory (``data_ptr()``) and HIP streams
(``torch.cuda.Stream.cuda_stream``); every step of the method runs in the HIP
kernels of ``libfwrs.so``.  There is no fallback: if the library is missing or
the GPU is absent the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfwrs.so")

OK, E_ARG, E_NOMEM, E_HIP, E_STATE = 0, 1, 2, 3, 4
BIAS_NONE, BIAS_BERNOULLI, BIAS_FULL, BIAS_MEMORYLESS, AES = 0, 1, 2, 3, 4
FLAG_REPROJECT = 1
FLAG_NO_RESOLVE_PLANE = 2
FOV_MIP, FOV_GAUSS = 0, 1
MAX_K = 16

#: every symbol include/fwrs.h declares
EXPORTS = (
    "fwrs_default_params", "fwrs_state_bytes", "fwrs_state_bytes_params", "fwrs_state_host_bytes", "fwrs_create", "fwrs_create_ex",
    "fwrs_destroy", "fwrs_set_stream", "fwrs_reset", "fwrs_push_frame", "fwrs_resolve",
    "fwrs_push_frame_resolve", "fwrs_push_frame_resolve_incremental", "fwrs_push_frame_reproject",
    "fwrs_frame_index", "fwrs_get_state", "fwrs_download_state", "fwrs_get_stats",
    "fwrs_set_tile", "fwrs_set_resolve_plane_from", "fwrs_sync", "fwrs_strerror", "fwrs_tick", "fwrs_tick_noalloc", "fwrs_engine_create", "fwrs_engine_tick",
    "fwrs_engine_set_tile", "fwrs_engine_destroy", "fwrs_foveator_create", "fwrs_foveate",
    "fwrs_push_frame_foveated", "fwrs_foveator_destroy", "fwrs_method_constants", "fwrs_gauss_weights",
)


class FwrsError(RuntimeError):
    def __init__(self, status: int, what: str):
        super().__init__(f"{what}: {strerror(status)} ({status})")
        self.status = status


class Params(C.Structure):
    """``fwrs_params``."""

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
        ("flags", C.c_uint32),
        ("lambda_decay", C.c_float),
    ]


class StateView(C.Structure):
    """``fwrs_state_view``."""

    _fields_ = [
        ("width", C.c_int),
        ("height", C.c_int),
        ("k", C.c_int),
        ("frame_index", C.c_uint32),
        ("pitch", C.c_size_t),
        ("wsum", C.c_void_p),
        ("rec", C.c_void_p),
        ("idx", C.c_void_p),
        ("wsum_slots", C.c_int),
        ("cnt", C.c_void_p),
        ("depth", C.c_void_p),
        ("res", C.c_void_p),
    ]


class Frame(C.Structure):
    """``fwrs_frame``."""

    _fields_ = [
        ("ctx", C.c_void_p),
        ("color", C.c_void_p),
        ("level_map", C.c_void_p),
        ("gaze_x", C.c_float),
        ("gaze_y", C.c_float),
        ("out", C.c_void_p),
    ]


_lib = None


def load(path: str | None = None):
    """Load libfwrs.so (built by ``paper_2510_03964_amd.build``).  Raises if absent."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or os.environ.get("FWRS_LIB") or LIB_PATH
    if not os.path.exists(p):
        raise FileNotFoundError(f"{p} is missing: build it with `python -m paper_2510_03964_amd.build`")
    L = C.CDLL(p)
    vp, i, f, u32, sz = C.c_void_p, C.c_int, C.c_float, C.c_uint32, C.c_size_t
    sig = {
        "fwrs_default_params": (i, [i, C.POINTER(Params)]),
        "fwrs_state_bytes": (sz, [i, i, i]),
        "fwrs_state_bytes_params": (sz, [i, i, i, C.POINTER(Params)]),
        "fwrs_state_host_bytes": (sz, [i, i, i]),
        "fwrs_create": (i, [i, i, i, C.POINTER(vp)]),
        "fwrs_create_ex": (i, [i, i, i, C.POINTER(Params), vp, vp, sz, C.POINTER(vp)]),
        "fwrs_destroy": (i, [vp]),
        "fwrs_set_stream": (i, [vp, vp]),
        "fwrs_reset": (i, [vp]),
        "fwrs_push_frame": (i, [vp, vp, vp, f, f]),
        "fwrs_resolve": (i, [vp, vp]),
        "fwrs_push_frame_resolve": (i, [vp, vp, vp, f, f, vp]),
        "fwrs_push_frame_resolve_incremental": (i, [vp, vp, vp, f, f, vp]),
        "fwrs_push_frame_reproject": (i, [vp, vp, vp, vp, vp, f, f, f, vp]),
        "fwrs_frame_index": (i, [vp, C.POINTER(u32)]),
        "fwrs_get_state": (i, [vp, C.POINTER(StateView)]),
        "fwrs_download_state": (i, [vp, vp, sz]),
        "fwrs_get_stats": (i, [vp, C.POINTER(C.c_uint64), C.POINTER(C.c_uint64), C.POINTER(C.c_uint64),
                               C.POINTER(C.c_uint64)]),
        "fwrs_set_tile": (i, [vp, i, i]),
        "fwrs_set_resolve_plane_from": (i, [vp, u32]),
        "fwrs_sync": (i, [vp]),
        "fwrs_strerror": (C.c_char_p, [i]),
        "fwrs_tick": (i, [C.POINTER(Frame), i, vp]),
        "fwrs_tick_noalloc": (i, [C.POINTER(Frame), i, vp]),
        "fwrs_engine_create": (i, [vp, i, i, C.POINTER(vp)]),
        "fwrs_engine_tick": (i, [vp, C.POINTER(Frame), i]),
        "fwrs_engine_set_tile": (i, [vp, C.c_longlong, i, i]),
        "fwrs_engine_destroy": (i, [vp]),
        "fwrs_foveator_create": (i, [i, i, f, f, u32, vp, C.POINTER(vp)]),
        "fwrs_foveate": (i, [vp, vp, f, f, vp, vp]),
        "fwrs_push_frame_foveated": (i, [vp, vp, vp, f, f, vp]),
        "fwrs_foveator_destroy": (i, [vp]),
        "fwrs_method_constants": (i, [i, C.POINTER(Params), C.POINTER(f)]),
        "fwrs_gauss_weights": (i, [f, C.POINTER(f)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    if path is None:
        _lib = L
    return L


def strerror(status: int) -> str:
    try:
        return load().fwrs_strerror(int(status)).decode()
    except FileNotFoundError:
        return f"status {status}"


def _check(status: int, what: str) -> None:
    if status != OK:
        raise FwrsError(status, what)


def default_params(width: int, **overrides) -> Params:
    p = Params()
    _check(load().fwrs_default_params(int(width), C.byref(p)), "fwrs_default_params")
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


def state_bytes(width: int, height: int, k: int, params: Params | None = None) -> int:
    """Device bytes of a context's store (``params`` None: the defaults' layout)."""
    if params is None:
        return int(load().fwrs_state_bytes(int(width), int(height), int(k)))
    return int(load().fwrs_state_bytes_params(int(width), int(height), int(k), C.byref(params)))


def method_constants(width: int, params: Params | None = None) -> np.ndarray:
    """The constants a context passes to the kernels (fwrs_method_constants), float32[9]."""
    p = params if params is not None else default_params(width)
    out = (C.c_float * 9)()
    _check(load().fwrs_method_constants(int(width), C.byref(p), out), "fwrs_method_constants")
    return np.array(out[:], dtype=np.float32)


def gauss_weights(sigma: float) -> np.ndarray:
    """The foveation generator's normalised Gaussian weights (fwrs_gauss_weights), float32[2R + 1]."""
    out = (C.c_float * 65)()
    R = int(load().fwrs_gauss_weights(float(sigma), out))
    if R < 0:
        raise ValueError(f"no Gaussian weights for sigma {sigma}")
    return np.array(out[:2 * R + 1], dtype=np.float32)


def state_host_bytes(width: int, height: int, k: int) -> int:
    return int(load().fwrs_state_host_bytes(int(width), int(height), int(k)))


def _stream_handle(stream) -> int | None:
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream or None
    return int(stream.cuda_stream) or None


def _ptr(t) -> int:
    return int(t.data_ptr())


def _f32(t) -> bool:
    return str(t.dtype) == "torch.float32"


def _u8(t) -> bool:
    return str(t.dtype) == "torch.uint8"


@dataclass
class HostState:
    """A packed host copy of a context's reservoir store (see fwrs_download_state)."""

    wsum: np.ndarray   # [H, W] f32
    cnt: np.ndarray    # [H, W] u32
    wt: np.ndarray     # [k, H, W] f32
    idx: np.ndarray    # [k, H, W] u32
    col: np.ndarray    # [k, 3, H, W] f32
    wslot: np.ndarray  # [k, H, W] f32: slot j's w_sum (its own under BIAS_FULL, else wsum)


class Reservoir:
    """A context: the k-slot reservoirs of every pixel of a width x height stream.

    ``arena`` may be a caller-owned device tensor (uint8, at least
    ``state_bytes(width, height, k, params)`` bytes, 256-byte aligned) that holds the
    store; otherwise the library allocates it."""

    def __init__(self, width: int, height: int, k: int, params: Params | None = None, stream=None, arena=None):
        self._L = load()
        self.width, self.height, self.k = int(width), int(height), int(k)
        self.params = params if params is not None else default_params(width)
        self._arena = arena
        h = C.c_void_p()
        ap = _ptr(arena) if arena is not None else None
        ab = arena.numel() * arena.element_size() if arena is not None else 0
        _check(self._L.fwrs_create_ex(self.width, self.height, self.k, C.byref(self.params), _stream_handle(stream),
                                      ap, ab, C.byref(h)), "fwrs_create_ex")
        self._h = h

    @property
    def handle(self) -> int:
        return self._h.value

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(self._L.fwrs_destroy(self._h), "fwrs_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def set_stream(self, stream) -> None:
        _check(self._L.fwrs_set_stream(self._h, _stream_handle(stream)), "fwrs_set_stream")

    def set_tile(self, tile_x: int, tile_y: int) -> None:
        _check(self._L.fwrs_set_tile(self._h, int(tile_x), int(tile_y)), "fwrs_set_tile")

    def reset(self) -> None:
        _check(self._L.fwrs_reset(self._h), "fwrs_reset")

    def set_resolve_plane_from(self, frame_index: int) -> None:
        """fwrs_set_resolve_plane_from: the frame index from which fused passes copy unchanged
        pixels' resolves from the resolve plane (a launch policy; results never change)."""
        _check(self._L.fwrs_set_resolve_plane_from(self._h, int(frame_index)), "fwrs_set_resolve_plane_from")

    def _check_frame(self, color, level) -> None:
        H, W = self.height, self.width
        if tuple(color.shape) != (H, W, 3) or not _f32(color) or not color.is_contiguous():
            raise ValueError(f"color must be contiguous float32 [{H}, {W}, 3]")
        if tuple(level.shape) != (H, W) or not _u8(level) or not level.is_contiguous():
            raise ValueError(f"level must be contiguous uint8 [{H}, {W}]")
        if not (color.is_cuda and level.is_cuda):
            raise ValueError("color and level must be device tensors")

    def _check_out(self, out) -> None:
        if tuple(out.shape) != (self.height, self.width, 3) or not _f32(out) or not out.is_contiguous():
            raise ValueError("out must be contiguous float32 [H, W, 3]")
        if not out.is_cuda:
            raise ValueError("out must be a device tensor")

    def push(self, color, level, gaze_x: float, gaze_y: float) -> None:
        self._check_frame(color, level)
        _check(self._L.fwrs_push_frame(self._h, _ptr(color), _ptr(level), float(gaze_x), float(gaze_y)),
               "fwrs_push_frame")

    def resolve(self, out) -> None:
        self._check_out(out)
        _check(self._L.fwrs_resolve(self._h, _ptr(out)), "fwrs_resolve")

    def step(self, color, level, gaze_x: float, gaze_y: float, out) -> None:
        """fwrs_push_frame_resolve: one frame of update and resolve in one pass."""
        self._check_frame(color, level)
        self._check_out(out)
        _check(self._L.fwrs_push_frame_resolve(self._h, _ptr(color), _ptr(level), float(gaze_x), float(gaze_y),
                                               _ptr(out)), "fwrs_push_frame_resolve")

    def step_incremental(self, color, level, gaze_x: float, gaze_y: float, out) -> None:
        """fwrs_push_frame_resolve_incremental: like step(), writing only the pixels whose
        reservoir changed; `out` must hold this context's previous resolve."""
        self._check_frame(color, level)
        self._check_out(out)
        _check(self._L.fwrs_push_frame_resolve_incremental(self._h, _ptr(color), _ptr(level), float(gaze_x),
                                                           float(gaze_y), _ptr(out)),
               "fwrs_push_frame_resolve_incremental")

    def step_reproject(self, color, level, motion, depth, gaze_x: float, gaze_y: float, depth_tol: float,
                       out=None) -> None:
        """fwrs_push_frame_reproject: one frame with reverse reprojection by `motion` ([H, W, 2]
        float32 pixels) and the depth flush (`depth` [H, W] float32), resolving into `out` if
        given.  The context must have been created with FLAG_REPROJECT."""
        self._check_frame(color, level)
        H, W = self.height, self.width
        if tuple(motion.shape) != (H, W, 2) or not _f32(motion) or not motion.is_contiguous():
            raise ValueError(f"motion must be contiguous float32 [{H}, {W}, 2]")
        if tuple(depth.shape) != (H, W) or not _f32(depth) or not depth.is_contiguous():
            raise ValueError(f"depth must be contiguous float32 [{H}, {W}]")
        if not (motion.is_cuda and depth.is_cuda):
            raise ValueError("motion and depth must be device tensors")
        if out is not None:
            self._check_out(out)
        _check(self._L.fwrs_push_frame_reproject(self._h, _ptr(color), _ptr(level), _ptr(motion), _ptr(depth),
                                                 float(gaze_x), float(gaze_y), float(depth_tol),
                                                 _ptr(out) if out is not None else None),
               "fwrs_push_frame_reproject")

    def step_foveated(self, foveator: "Foveator", full, gaze_x: float, gaze_y: float, out=None) -> None:
        """fwrs_push_frame_foveated: the foveator degrades the full frame and the reservoir pass
        samples its candidates from the level images directly; resolves into `out` if given."""
        foveator._check_full(full)
        if out is not None:
            self._check_out(out)
        _check(self._L.fwrs_push_frame_foveated(self._h, foveator._h, _ptr(full), float(gaze_x), float(gaze_y),
                                                _ptr(out) if out is not None else None),
               "fwrs_push_frame_foveated")

    @property
    def frame_index(self) -> int:
        t = C.c_uint32()
        _check(self._L.fwrs_frame_index(self._h, C.byref(t)), "fwrs_frame_index")
        return int(t.value)

    def state_view(self) -> StateView:
        v = StateView()
        _check(self._L.fwrs_get_state(self._h, C.byref(v)), "fwrs_get_state")
        return v

    def download(self) -> HostState:
        H, W, k = self.height, self.width, self.k
        N = H * W
        buf = np.empty(state_host_bytes(W, H, k), np.uint8)
        _check(self._L.fwrs_download_state(self._h, buf.ctypes.data, buf.nbytes), "fwrs_download_state")
        o = 0

        def take(dtype, count, shape):
            nonlocal o
            a = buf[o:o + 4 * count].view(dtype).reshape(shape)
            o += 4 * count
            return a

        return HostState(take(np.float32, N, (H, W)), take(np.uint32, N, (H, W)), take(np.float32, k * N, (k, H, W)),
                         take(np.uint32, k * N, (k, H, W)), take(np.float32, 3 * k * N, (k, 3, H, W)),
                         take(np.float32, k * N, (k, H, W)))

    def stats(self) -> tuple[int, int, int]:
        """(slot takes, pixel updates with a take, pixel updates) since creation or reset."""
        a, b, c = C.c_uint64(), C.c_uint64(), C.c_uint64()
        _check(self._L.fwrs_get_stats(self._h, C.byref(a), C.byref(b), C.byref(c), None), "fwrs_get_stats")
        return int(a.value), int(b.value), int(c.value)

    def flushes(self) -> int:
        """Reprojected pixel updates whose history was flushed, since creation or reset."""
        a = C.c_uint64()
        _check(self._L.fwrs_get_stats(self._h, None, None, None, C.byref(a)), "fwrs_get_stats")
        return int(a.value)

    def sync(self) -> None:
        _check(self._L.fwrs_sync(self._h), "fwrs_sync")


TICK_MAX = 4096


def _fill_frames(buf, entries, capacity: int) -> int:
    """Writes (Reservoir, color, level, gaze_x, gaze_y, out) entries into a ctypes Frame array."""
    n = 0
    for (res, color, level, gx, gy, out) in entries:
        if n >= capacity:
            raise ValueError("too many frames for one tick")
        res._check_frame(color, level)
        res._check_out(out)
        fr = buf[n]
        fr.ctx = res.handle
        fr.color = _ptr(color)
        fr.level_map = _ptr(level)
        fr.gaze_x = float(gx)
        fr.gaze_y = float(gy)
        fr.out = _ptr(out)
        n += 1
    return n


def tick(entries, stream=None) -> None:
    """fwrs_tick: one batched launch advances every entry's context by one frame per entry on
    `stream` (a context's several entries are its consecutive frames, in order, run as one group).
    entries: iterable of (Reservoir, color, level, gaze_x, gaze_y, out)."""
    entries = list(entries)
    buf = (Frame * max(1, len(entries)))()
    n = _fill_frames(buf, entries, TICK_MAX)
    _check(load().fwrs_tick(buf, n, _stream_handle(stream)), "fwrs_tick")


TICK_NOALLOC_MAX = 256


def tick_noalloc(entries, stream=None) -> None:
    """fwrs_tick_noalloc: fwrs_tick through the library's fixed device table (at most 256
    entries; allocates nothing).  The caller orders the tick against the contexts' streams."""
    entries = list(entries)
    if len(entries) > TICK_NOALLOC_MAX:
        raise ValueError(f"at most {TICK_NOALLOC_MAX} entries per fwrs_tick_noalloc call")
    buf = (Frame * max(1, len(entries)))()
    n = _fill_frames(buf, entries, TICK_NOALLOC_MAX)
    _check(load().fwrs_tick_noalloc(buf, n, _stream_handle(stream)), "fwrs_tick_noalloc")


class Engine:
    """Batched ticks: one kernel launch advances many contexts, each by one frame per entry."""

    def __init__(self, max_frames: int, stream=None, use_graph: bool = False):
        self._L = load()
        h = C.c_void_p()
        _check(self._L.fwrs_engine_create(_stream_handle(stream), int(max_frames), 1 if use_graph else 0,
                                          C.byref(h)), "fwrs_engine_create")
        self._h = h
        self.max_frames = int(max_frames)
        self._frames = (Frame * self.max_frames)()

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(self._L.fwrs_engine_destroy(self._h), "fwrs_engine_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_tile(self, min_pixels: int, tile_x: int, tile_y: int) -> None:
        _check(self._L.fwrs_engine_set_tile(self._h, int(min_pixels), int(tile_x), int(tile_y)),
               "fwrs_engine_set_tile")

    def tick(self, entries) -> None:
        """entries: iterable of (Reservoir, color, level, gaze_x, gaze_y, out)."""
        n = _fill_frames(self._frames, entries, self.max_frames)
        _check(self._L.fwrs_engine_tick(self._h, self._frames, n), "fwrs_engine_tick")


class Foveator:
    """The foveation generator: full frame -> degraded frame + level map (mip + bilinear or
    Gaussian), standalone or fused into a context's frame (Reservoir.step_foveated)."""

    def __init__(self, width: int, height: int, fovea_radius_px: float, ring_radius_px: float,
                 mode: int = FOV_MIP, stream=None):
        self._L = load()
        self.width, self.height, self.mode = int(width), int(height), int(mode)
        h = C.c_void_p()
        _check(self._L.fwrs_foveator_create(self.width, self.height, float(fovea_radius_px), float(ring_radius_px),
                                            self.mode, _stream_handle(stream), C.byref(h)), "fwrs_foveator_create")
        self._h = h

    def _check_full(self, full) -> None:
        H, W = self.height, self.width
        if tuple(full.shape) != (H, W, 3) or not _f32(full) or not full.is_contiguous() or not full.is_cuda:
            raise ValueError(f"full must be a contiguous float32 device tensor [{H}, {W}, 3]")

    def foveate(self, full, gaze_x: float, gaze_y: float, color, level) -> None:
        self._check_full(full)
        H, W = self.height, self.width
        if tuple(color.shape) != (H, W, 3) or not _f32(color) or not color.is_contiguous() or not color.is_cuda:
            raise ValueError("color must be a contiguous float32 device tensor [H, W, 3]")
        if tuple(level.shape) != (H, W) or not _u8(level) or not level.is_contiguous() or not level.is_cuda:
            raise ValueError("level must be a contiguous uint8 device tensor [H, W]")
        _check(self._L.fwrs_foveate(self._h, _ptr(full), float(gaze_x), float(gaze_y), _ptr(color), _ptr(level)),
               "fwrs_foveate")

    def close(self) -> None:
        if getattr(self, "_h", None) is not None and self._h.value:
            _check(self._L.fwrs_foveator_destroy(self._h), "fwrs_foveator_destroy")
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
