"""Tile-shape autotuner for the weighted-reservoir-sampling kernels.

A tile is tile_x x tile_y pixels processed by one wave group (one thread per
pixel; 64, 128 or 256 threads).  The shape only changes the memory access
pattern, never the results, so the tuner may pick freely: for each candidate it
resets one context, primes it with a few frames (so the reservoir is past its
all-slots-replaced first frames), times a fixed run of frames with HIP events
and keeps the fastest median.  Every candidate sees the identical work (same
frames, same frame indices, same random draws).

Results are cached in a JSON file keyed by (architecture, width, height, k):
$FWRS_AUTOTUNE_CACHE, else ~/.cache/fwrs/autotune.json.
"""
from __future__ import annotations

import json
import os
import statistics

import torch

from . import fwrs, synth

#: the shapes the tuner tries (tile_x pixels, tile_y rows)
CANDIDATES = ((8, 8), (16, 16), (32, 8), (64, 1), (64, 4), (128, 2), (256, 1))


def cache_path() -> str:
    return os.environ.get("FWRS_AUTOTUNE_CACHE") or os.path.join(os.path.expanduser("~"), ".cache", "fwrs",
                                                                   "autotune.json")


def _arch(device) -> str:
    props = torch.cuda.get_device_properties(device)
    return getattr(props, "gcnArchName", props.name).split(":")[0]


def _key(arch: str, width: int, height: int, k: int) -> str:
    return f"{arch}:{width}x{height}:k{k}"


def load_cache() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def save_cache(cache: dict) -> None:
    path = cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune(width: int, height: int, k: int, device="cuda", frames: int = 12, prime: int = 16, reps: int = 3,
         candidates=CANDIDATES, use_cache: bool = True, stream=None) -> dict:
    """Best tile for a width x height, k-slot context on `device`.  Returns
    {"tile": (tile_x, tile_y), "ms": {shape: median ms per frame}, "cached": bool}."""
    device = torch.device(device)
    arch = _arch(device)
    key = _key(arch, width, height, k)
    cache = load_cache() if use_cache else {}
    if use_cache and key in cache:
        e = cache[key]
        return {"tile": tuple(e["tile"]), "ms": e["ms"], "cached": True}
    stream = stream or torch.cuda.current_stream(device)
    spec = synth.StreamSpec(width, height, k, prime + frames, 0.05 * width, 0.125 * width, 8.0 * width / 3840,
                            90, 24.0 * width / 3840, stream_id=0)
    src = synth.FrameSource(spec, device=device)
    seq = [src.frame(t) for t in range(prime + frames)]
    p = fwrs.default_params(width, fovea_radius_px=spec.fovea_radius_px, seed=synth.PHILOX_SEED)
    res = fwrs.Reservoir(width, height, k, p, stream=stream)
    out = torch.empty((height, width, 3), dtype=torch.float32, device=device)
    timings: dict[str, float] = {}
    try:
        for (tx, ty) in candidates:
            res.set_tile(tx, ty)
            runs = []
            for _ in range(reps):
                res.reset()
                for t in range(prime):
                    res.step(*seq[t], out)
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record(stream)
                for t in range(prime, prime + frames):
                    res.step(*seq[t], out)
                b.record(stream)
                b.synchronize()
                runs.append(a.elapsed_time(b) / frames)
            timings[f"{tx}x{ty}"] = statistics.median(runs)
    finally:
        res.close()
    best = min(timings, key=timings.get)
    tile = tuple(int(v) for v in best.split("x"))
    if use_cache:
        cache[key] = {"tile": list(tile), "ms": timings}
        save_cache(cache)
    return {"tile": tile, "ms": timings, "cached": False}


def tune_engine(engine: "fwrs.Engine", classes, device="cuda", **kw) -> dict:
    """Tunes one tile per resolution class and installs it in a batched engine.
    classes: iterable of (width, height, k) -- one representative per class; the
    class of a context is chosen by its pixel count (largest threshold first)."""
    chosen = {}
    for (w, h, k) in sorted(set(classes), key=lambda c: c[0] * c[1]):
        r = tune(w, h, k, device=device, **kw)
        chosen[(w, h, k)] = r
        engine.set_tile(w * h, *r["tile"])
    return chosen
