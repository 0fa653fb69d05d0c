"""Benchmark: 4K, k = 4 weighted-reservoir-sampling update + resolve on one MI355X.

Workload: 3840x2160 RGB float32 foveated frames, k = 4 slots per pixel, the
600-frame synthetic gaze trace (fovea 216 px, 2x2 ring to 540 px, 4x4 beyond;
microsaccades sigma 8 px, a saccade every 90 frames with 24 px landing
scatter), Philox seed 0x25103964, Bernoulli bias.  All frames are generated on
the device before timing; a step is one fused update + resolve
(fwrs_push_frame_resolve) of one frame, starting from an empty reservoir.

Prints one JSON line: Gpixel-updates/s, ms per frame, the roofline of the
fused kernel (algorithmic bytes per pixel-update 33 + 16k + 20 r, with r the
slot replacements per pixel-update counted by the kernel, over its average
launch time from HIP events on its stream), and the CPU oracle timed on a
bounded sample of the same workload.  The same frames are then run through
the incremental entry point (output rewritten only where a slot changed),
reported in its own object with its own byte model.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "4K k=4 update+resolve ms & Gpix/s, %HBM peak; multi-stream p99 vs plain"
HBM_PEAK_GBPS = 8000.0
COUNTERS = os.path.join(ROOT, "profiles", "fused_k4_4k_counters.json")


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def bytes_per_update(k: int, rbar: float) -> float:
    """Algorithmic HBM bytes per pixel-update of the fused pass: colour in (12), level (1),
    w_sum read and written (8), output (12), every slot's colour and weight read for the
    resolve (16 k), and colour + weight + index written per replaced slot (20 per take)."""
    return 33.0 + 16.0 * k + 20.0 * rbar


def bytes_per_update_incremental(k: int, rbar: float, changed: float) -> float:
    """Same for the incremental pass: level (1) and w_sum read + write (8) everywhere; colour in,
    the record read and the output written (12 + 16 k + 12) only at the fraction `changed` of
    pixel-updates where some slot was replaced; 20 bytes per replaced slot."""
    return 9.0 + changed * (24.0 + 16.0 * k) + 20.0 * rbar


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2510_03964_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_counters(n_pixels: int) -> float | None:
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it was taken on the
    current kernel sources and workload; None otherwise."""
    if not os.path.exists(COUNTERS):
        return None
    with open(COUNTERS) as f:
        c = json.load(f)
    if c.get("source_hash") != kernel_source_hash() or c.get("pixels") != n_pixels:
        return None
    return 1024.0 * (c["fetch_kib_per_dispatch"] * c["fetch_scale"] + c["write_kib_per_dispatch"] * c["write_scale"])


def timed_run(res, frames, out, stream, step):
    """Times len(frames) calls of `step` (one per frame) with HIP events on `stream`: per-launch
    start/end events and one pair around the whole region."""
    import numpy as np
    import torch

    K = len(frames)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(K)]
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start.record(stream)
    for t in range(K):
        c, lev, gx, gy = frames[t]
        ev[t][0].record(stream)
        step(c, lev, gx, gy, out)
        ev[t][1].record(stream)
    t_end.record(stream)
    torch.cuda.synchronize()
    return t_start.elapsed_time(t_end), np.array([a.elapsed_time(b) for (a, b) in ev])


def cpu_baseline(frames_host, spec, n_frames: int) -> dict:
    import oracle

    q = oracle.default_params(spec.width, fovea_radius_px=spec.fovea_radius_px, seed=0x25103964)
    o = oracle.Oracle(spec.width, spec.height, spec.k, q)
    t0 = time.perf_counter()
    for (c, lev, gx, gy) in frames_host[:n_frames]:
        o.push(c, lev, gx, gy)
        o.resolve()
    dt = time.perf_counter() - t0
    px = spec.pixels * n_frames
    return {"value": px / dt / 1e9, "unit": "Gpixel-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"first {n_frames} frames of the same 3840x2160 k=4 trace, full frames, update + resolve, "
                      f"single-threaded C oracle ({dt:.1f} s)", "ms_per_frame": 1000.0 * dt / n_frames}


def copy_bandwidth(torch, dev, nbytes: int = 1 << 30, reps: int = 20) -> float:
    """Achievable HBM bandwidth of a plain device-to-device copy (GB/s, read + write)."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    a.fill_(1.0)
    for _ in range(3):
        b.copy_(a)
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        b.copy_(a)
    e.record()
    torch.cuda.synchronize()
    sec = s.elapsed_time(e) / 1000.0 / reps
    del a, b
    return 2.0 * nbytes / sec / 1e9


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=600, help="timed frames (from an empty reservoir)")
    ap.add_argument("--warmup", type=int, default=10, help="untimed frames on a separate context")
    ap.add_argument("--cpu-frames", type=int, default=8, help="frames of the oracle CPU baseline (0: skip)")
    ap.add_argument("--tile", type=str, default="", help="tile_x,tile_y override")
    ap.add_argument("--no-copy", action="store_true", help="skip the copy-bandwidth reference")
    ap.add_argument("--no-incremental", action="store_true", help="skip the incremental-resolve run")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): every pixel stream is independent "
              "and this build measures the single-GPU pass.", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    from paper_2510_03964_amd import fwrs, synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    spec = synth.spec_4k(frames=max(600, args.steps))
    K, W = args.steps, args.warmup
    log(f"generating {K + W} frames of {spec.width}x{spec.height} on {torch.cuda.get_device_name(0)}")
    src = synth.FrameSource(spec, device=dev, n_frames=max(K, W))
    t0 = time.perf_counter()
    frames = []
    for t in range(K):
        frames.append(src.frame(t))
        if (t + 1) % 100 == 0:
            torch.cuda.synchronize()
            log(f"  {t + 1} frames")
    torch.cuda.synchronize()
    log(f"frames resident in HBM ({time.perf_counter() - t0:.1f} s)")

    p = fwrs.default_params(spec.width, fovea_radius_px=spec.fovea_radius_px, seed=synth.PHILOX_SEED)
    tile = tuple(int(v) for v in args.tile.split(",")) if args.tile else None
    out = torch.empty((spec.height, spec.width, 3), dtype=torch.float32, device=dev)

    # warm-up on a throwaway context (code load, clocks)
    warm = fwrs.Reservoir(spec.width, spec.height, spec.k, p, stream=stream)
    if tile:
        warm.set_tile(*tile)
    for t in range(W):
        warm.step(*frames[t % len(frames)], out)
    warm.sync()
    warm.close()

    res = fwrs.Reservoir(spec.width, spec.height, spec.k, p, stream=stream)
    if tile:
        res.set_tile(*tile)
    total_ms, per = timed_run(res, frames, out, stream, res.step)
    log(f"timed {K} frames: {total_ms:.2f} ms on the GPU clock")
    takes, changed, updates = res.stats()
    assert updates == K * spec.pixels
    st_ok = res.frame_index == K
    res.close()
    rbar = takes / updates
    B = bytes_per_update(spec.k, rbar)
    kern_ms = float(per.mean())
    achieved = spec.pixels * B / (kern_ms / 1e3) / 1e9
    traffic = traffic_from_counters(spec.pixels)
    ms_per_step = total_ms / K
    value = spec.pixels * K / (total_ms / 1e3) / 1e9

    incremental = None
    if not args.no_incremental:
        inc = fwrs.Reservoir(spec.width, spec.height, spec.k, p, stream=stream)
        if tile:
            inc.set_tile(*tile)
        inc.step(*frames[0], out)            # frame 0: every pixel takes, full resolve
        inc_ms, inc_per = timed_run(inc, frames[1:], out, stream, inc.step_incremental)
        i_takes, i_changed, i_updates = inc.stats()
        inc.close()
        n_inc = K - 1
        i_rbar = (i_takes - spec.k * spec.pixels) / (n_inc * spec.pixels)
        i_changed_frac = (i_changed - spec.pixels) / (n_inc * spec.pixels)
        i_B = bytes_per_update_incremental(spec.k, i_rbar, i_changed_frac)
        i_kern = float(inc_per.mean())
        i_ach = spec.pixels * i_B / (i_kern / 1e3) / 1e9
        incremental = {"entry": "fwrs_push_frame_resolve_incremental", "frames": n_inc,
                       "ms_per_step": inc_ms / n_inc, "value": spec.pixels * n_inc / (inc_ms / 1e3) / 1e9,
                       "unit": "Gpixel-updates/s", "ms_per_frame_p50": float(np.percentile(inc_per, 50)),
                       "ms_per_frame_p99": float(np.percentile(inc_per, 99)),
                       "roofline": {"bound": "hbm", "achieved": i_ach, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                                    "frac": i_ach / HBM_PEAK_GBPS, "kernel_ms_avg": i_kern,
                                    "bytes_per_pixel_update": i_B, "slot_takes_per_pixel_update": i_rbar,
                                    "changed_pixel_fraction": i_changed_frac}}
        log(f"incremental: {inc_ms / n_inc:.4f} ms/frame")

    copy_gbps = None if args.no_copy else copy_bandwidth(torch, dev)

    cpu = None
    if args.cpu_frames > 0:
        log(f"timing the CPU oracle on {args.cpu_frames} frames")
        host = [(c.cpu().numpy(), lev.cpu().numpy(), gx, gy) for (c, lev, gx, gy) in frames[:args.cpu_frames]]
        cpu = cpu_baseline(host, spec, args.cpu_frames)

    line = {
        "metric": METRIC,
        "value": value,
        "unit": "Gpixel-updates/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"3840x2160 RGB f32 foveated frames, k=4, {K}-frame synthetic gaze trace "
                               f"(fovea 216 px, ring 540 px), fused update+resolve from an empty reservoir",
                   "width": spec.width, "height": spec.height, "k": spec.k, "frames": K,
                   "bias": "bernoulli", "tile": list(tile) if tile else "default"},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS,
                     "traffic": traffic,
                     "kernel": "fwrs::frame_kernel<4, 3> (fused update + full resolve)",
                     "kernel_ms_avg": kern_ms, "bytes_per_pixel_update": B, "slot_takes_per_pixel_update": rbar},
        "cpu_baseline": cpu,
        "ms_per_frame_p50": float(np.percentile(per, 50)),
        "ms_per_frame_p99": float(np.percentile(per, 99)),
        "pixels_changed_per_pixel_update": changed / updates,
        "incremental": incremental,
        "copy_gbps": copy_gbps,
        "state_ok": bool(st_ok),
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
