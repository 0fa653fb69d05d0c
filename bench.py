"""Benchmark: 4K, k = 4 weighted-reservoir-sampling update + resolve on one MI355X.

Workload (the paper-scale plain method): 3840x2160 RGB float32 foveated frames, k = 4 slots per
pixel, Bernoulli bias (Eq. 6), the 600-frame synthetic gaze trace (fovea 216 px, 2x2 ring to
540 px, 4x4 beyond; microsaccades sigma 8 px, a saccade every 90 frames with 24 px landing
scatter), Philox seed 0x25103964.  All frames are generated on the device before timing.

Timed region: the whole trace from an empty reservoir -- frames 0 .. 599 through
fwrs_push_frame_resolve, one launch per frame -- as --steps steps of ceil(600 / steps) consecutive
frames (20 steps of 30 frames for --steps 20); --warmup steps of the same size run first on a
throwaway context.  The library runs the full resolve while the store fills (frames 0-30), writes
the resolve plane at frame 31 and copies unchanged pixels from it from frame 32 on, so the trace
launches three kernels; the dominant one (frames 32-599) is the roofline's.

Prints one JSON line: Gpixel-updates/s over the trace, ms per frame, the roofline of the dominant
kernel (algorithmic bytes per pixel-update of update + resolve, 41 + 16k + 20 r, r = slot replacements per
pixel-update counted by the kernel, over its average launch time from HIP events on its stream;
beside it the 33-byte variant, the kernel's measured HBM traffic from the committed counter
summary of the same window, and the whole-trace and first-20-frame figures), and the CPU oracle
timed on a bounded sample of the same workload.  Further sections run the same frames through
the incremental entry point and through Eq. 7, the update-rule ablations, the foveation
generator, the moving-camera reprojection, the batched ticks and the serving loop.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "4K k=4 update+resolve ms & Gpix/s, %HBM peak; multi-stream p99 vs plain"
HBM_PEAK_GBPS = 8000.0
TRACE_FRAMES = 600
#: the frame index from which the library's fused passes use the resolve plane (its default, set explicitly)
PLANE_FROM = 32
COUNTERS = os.path.join(ROOT, "profiles", "fused_k4_4k_counters.json")
INC_COUNTERS = os.path.join(ROOT, "profiles", "incremental_k4_4k_counters.json")
EQ7_COUNTERS = os.path.join(ROOT, "profiles", "eq7_k4_4k_counters.json")
VALU_COUNTERS = os.path.join(ROOT, "profiles", "fused_valu_4k_counters.json")
KERNEL_PLAIN = "void fwrs::frame_kernel<4, 3, false>(fwrs::FrameDesc)"
KERNEL_FILL = "void fwrs::frame_kernel<4, 9, false>(fwrs::FrameDesc)"
KERNEL_CACHED = "void fwrs::frame_kernel<4, 7, false>(fwrs::FrameDesc)"
#: VALU issue peak of the MI355X for non-packed instructions, in lane-operations per second: one wave64
#: instruction per compute unit and clock, 256 CUs x 64 lanes x 2.4 GHz (profiles/valu_issue_rate.md measures
#: non-packed fp32 fma / mul / add at 0.92-0.98 of it; the published 157.3 TFLOP/s fp32 vector rate counts packed
#: instructions, which the library does not issue, and a fused multiply-add as two flops)
VALU_PEAK_TOPS = 39.3


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def bytes_per_update(k: int, rbar: float) -> float:
    """Algorithmic HBM bytes per pixel-update of update + resolve: colour in (12), level (1),
    w_sum read and written (8), the per-pixel count read and written (8; kept here as the context's frame
    index), output (12), every slot's colour and weight read for the resolve (16 k), and colour + weight +
    index written per replaced slot (20 per take)."""
    return 41.0 + 16.0 * k + 20.0 * rbar


def bytes_per_update_33(k: int, rbar: float) -> float:
    """The same without the per-pixel count (8 bytes), which the library keeps once per context."""
    return 33.0 + 16.0 * k + 20.0 * rbar


def bytes_per_update_incremental(k: int, rbar: float, changed: float) -> float:
    """Same for the incremental pass: level (1) and w_sum read + write (8) everywhere; colour in,
    the record read and the output written (12 + 16 k + 12) only at the fraction `changed` of
    pixel-updates where some slot was replaced; 20 bytes per replaced slot."""
    return 9.0 + changed * (24.0 + 16.0 * k) + 20.0 * rbar


def bytes_per_update_eq7(k: int, rbar: float) -> float:
    """Same for the fused pass under Eq. 7: colour in (12, every pixel compares it with its
    slots), level (1), each slot's own w_sum read and written (8 k), every slot's record read
    (16 k), output (12) and 20 bytes per replaced slot."""
    return 25.0 + 24.0 * k + 20.0 * rbar


def bytes_per_update_reproject(k: int, wsum_slots: int = 1) -> float:
    """Algorithmic HBM bytes per pixel-update of the reprojecting pass (a gather from the previous
    bank, a dense write of the next): motion (8), depth (4), the source's previous depth (4), level
    (1), colour (12), the source's w_sum(s) (4 s), count (4), records (16 k) and frame indices (4 k)
    read; records, indices, w_sum(s), count, depth (4) and output (12) written."""
    return 8 + 4 + 4 + 1 + 12 + 4 * wsum_slots + 4 + 20 * k + 20 * k + 4 * wsum_slots + 4 + 4 + 12


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2510_03964_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_from_counters(kernel: str, n_pixels: int, window: dict, path: str = COUNTERS) -> float | None:
    """HBM bytes per launch of `kernel` from a committed rocprofv3 counter summary, if it was taken on the
    current kernel sources, this frame size and this timed window (steps, frames per step, frames); None
    otherwise, so traffic measured on another window is never attached to this one."""
    if not os.path.exists(path):
        return None
    with open(path) as f:
        c = json.load(f)
    if c.get("source_hash") != kernel_source_hash() or c.get("pixels") != n_pixels or c.get("window") != window:
        return None
    k = c.get("kernels", {}).get(kernel)
    if not k:
        return None
    return 1024.0 * (k["fetch_kib_per_dispatch"] * c["fetch_scale"] + k["write_kib_per_dispatch"] * c["write_scale"])


def valu_per_pixel(kernel: str) -> float | None:
    """VALU instructions per pixel of `kernel` (one thread per pixel) from the committed counter summary, if it was
    taken on the current kernel sources; None otherwise."""
    if not os.path.exists(VALU_COUNTERS):
        return None
    with open(VALU_COUNTERS) as f:
        c = json.load(f)
    if c.get("source_hash") != kernel_source_hash() or kernel not in c.get("kernels", {}):
        return None
    return float(c["kernels"][kernel]["valu_insts_per_wave"])


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
        args = frames[t]
        ev[t][0].record(stream)
        step(*args, out)
        ev[t][1].record(stream)
    t_end.record(stream)
    torch.cuda.synchronize()
    return t_start.elapsed_time(t_end), np.array([a.elapsed_time(b) for (a, b) in ev])


def multistream(dev, stream, specs, gazes, ticks: int, ring: int, use_graph: bool, label: str) -> dict:
    """Batched ticks (one launch per tick over all its frames, tiles from the autotuner per resolution
    class) against plain per-frame launches of the same kernels on the same stream, on the same
    frames.  Frame t of a stream is frame t mod `ring` of its trace (a ring of distinct frames
    kept resident in HBM).  The first 3 ticks of each mode are untimed."""
    import numpy as np
    import torch

    from paper_2510_03964_amd import autotune, fwrs, synth

    srcs = [synth.FrameSource(s, device=dev, gaze=g) for s, g in zip(specs, gazes)]
    frames = [[src.frame(t % len(src)) for t in range(ring)] for src in srcs]
    torch.cuda.synchronize()
    eng = fwrs.Engine(len(specs), stream=stream, use_graph=use_graph)
    eng_direct = fwrs.Engine(len(specs), stream=stream, use_graph=False)
    classes = {}
    for s in specs:   # one representative k per resolution class: the most frequent
        classes.setdefault((s.width, s.height), []).append(s.k)
    reps = [(w, h, max(set(ks), key=ks.count)) for (w, h), ks in classes.items()]
    tuned = autotune.tune_engine(eng, reps, device=dev)
    tiles = {(w, h): r["tile"] for (w, h, _), r in tuned.items()}
    for (w, h), t in tiles.items():
        eng_direct.set_tile(w * h, *t)
    log(f"{label}: tiles {tiles}")

    def make():
        out = []
        for s in specs:
            p = fwrs.default_params(s.width, fovea_radius_px=s.fovea_radius_px, seed=synth.PHILOX_SEED,
                                    stream_id=s.stream_id)
            r = fwrs.Reservoir(s.width, s.height, s.k, p, stream=stream)
            r.set_tile(*tiles[(s.width, s.height)])
            out.append((r, torch.empty((s.height, s.width, 3), dtype=torch.float32, device=dev)))
        return out

    px_tick = sum(s.pixels for s in specs)
    result = {"streams": len(specs), "ticks": ticks, "ring": ring, "pixels_per_tick": px_tick,
              "tiles": {f"{w}x{h}": list(t) for (w, h), t in tiles.items()}}
    outs = {}
    for mode in ("batched", "batched_direct", "plain"):
        ctx = make()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(ticks)]
        torch.cuda.synchronize()
        for t in range(ticks):
            fr = [frames[i][t % ring] for i in range(len(specs))]
            ev[t][0].record(stream)
            if mode != "plain":
                (eng if mode == "batched" else eng_direct).tick([(ctx[i][0], *fr[i], ctx[i][1])
                                                                 for i in range(len(specs))])
            else:
                for i in range(len(specs)):
                    ctx[i][0].step(*fr[i], ctx[i][1])
            ev[t][1].record(stream)
        torch.cuda.synchronize()
        lat = np.array([a.elapsed_time(b) for (a, b) in ev[3:]])
        total = float(lat.sum())
        result[mode] = {"ms_per_tick_mean": float(lat.mean()), "ms_per_tick_p50": float(np.percentile(lat, 50)),
                        "ms_per_tick_p99": float(np.percentile(lat, 99)),
                        "gpix_per_s": px_tick * len(lat) / (total / 1e3) / 1e9}
        outs[mode] = [c[1] for c in ctx]
        for r, _ in ctx:
            r.close()
    result["identical_outputs"] = all(torch.equal(a, b) and torch.equal(a, c) for a, b, c in
                                      zip(outs["batched"], outs["plain"], outs["batched_direct"]))
    result["batched_over_plain_throughput"] = result["batched"]["gpix_per_s"] / result["plain"]["gpix_per_s"]
    result["batched"]["launch"] = "HIP graph replay" if use_graph else "direct launch"
    result["batched_direct"]["launch"] = "direct launch"
    eng.close()
    eng_direct.close()
    log(f"{label}: batched {result['batched']['ms_per_tick_p50']:.3f} ms p50 / {result['batched']['ms_per_tick_p99']:.3f} "
        f"p99, plain {result['plain']['ms_per_tick_p50']:.3f} / {result['plain']['ms_per_tick_p99']:.3f}")
    return result


def group_ticks(dev, stream, spec, frames, tile, ks=(4, 8), sizes=(1, 2, 4, 8), n: int = 96, warm: int = 40) -> dict:
    """A session's consecutive frames as one group: one 4K stream, past its resolve-plane switch
    (`warm` untimed frames first), runs the next n resident frames through fwrs_tick as groups of
    F consecutive frames (one launch per group) and, on a second context, as one plain launch per
    frame; milliseconds per frame on the GPU clock for each slot count k and group size F."""
    import torch

    from paper_2510_03964_amd import fwrs, synth

    result = {"width": spec.width, "height": spec.height, "frames": n, "warm_frames": warm}
    for k in ks:
        p = fwrs.default_params(spec.width, fovea_radius_px=spec.fovea_radius_px, seed=synth.PHILOX_SEED)
        row = {}
        for F in (0, *sizes):                      # F = 0: plain launches
            r = fwrs.Reservoir(spec.width, spec.height, k, p, stream=stream)
            if tile:
                r.set_tile(*tile)
            out = torch.empty((spec.height, spec.width, 3), dtype=torch.float32, device=dev)
            for t in range(warm):
                r.step(*frames[t], out)
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            a.record(stream)
            if F == 0:
                for t in range(warm, warm + n):
                    r.step(*frames[t], out)
            else:
                for g in range(warm, warm + n, F):
                    fwrs.tick([(r, *frames[t], out) for t in range(g, min(g + F, warm + n))], stream=stream)
            b.record(stream)
            torch.cuda.synchronize()
            ms = a.elapsed_time(b) / n
            row["plain" if F == 0 else f"group_{F}"] = {"ms_per_frame": ms,
                                                        "gpix_per_s": spec.pixels / (ms / 1e3) / 1e9}
            r.close()
        for F in sizes:
            row[f"group_{F}"]["speedup_over_plain"] = row["plain"]["ms_per_frame"] / row[f"group_{F}"]["ms_per_frame"]
        result[f"k{k}"] = row
        log(f"groups k={k}: plain {row['plain']['ms_per_frame']:.4f} ms/frame, " +
            ", ".join(f"F={F} {row[f'group_{F}']['ms_per_frame']:.4f}" for F in sizes))
    return result


def serving(dev, stream, time_scale: float, fps_scale: float, ring: int, label: str, max_group: int = 8) -> dict:
    """32 sessions arriving as a Poisson process (mean 1/s; lifetime U[10, 60] s; 1920x1080 or
    3840x2160; k in {4, 8}; 72, 90 or 120 Hz), arrivals and lifetimes compressed by `time_scale`
    (same concurrency and offered load, shorter run), frame rates multiplied by `fps_scale`.
    Reservoir budget 64 GB.  The same session mix and scheduler (each tick takes up to `max_group`
    due frames of every session) run through the batched executor (one direct batched launch per
    tick, a session's several frames in it as one group; graph replay adds a few microseconds per
    tick on this GPU) and the plain one (one launch per frame)."""
    import torch

    from paper_2510_03964_amd import autotune, serve, synth

    base = serve.poisson_sessions(n=32, rate_per_s=1.0, seed=4242, time_scale=time_scale)
    sessions = [serve.SessionSpec(s.sid, s.arrival_s, s.lifetime_s, s.width, s.height, s.k, s.fps * fps_scale)
                for s in base]
    rings, tiles = {}, {}
    for (w, h) in sorted({(s.width, s.height) for s in sessions}):
        spec = synth.StreamSpec(w, h, 4, ring, 0.05 * w, 0.125 * w, 8.0 * w / 3840, 90, 24.0 * w / 3840,
                                stream_id=w)
        src = synth.FrameSource(spec, device=dev)
        rings[(w, h)] = [src.frame(t) for t in range(ring)]
        tiles[(w, h)] = autotune.tune(w, h, 4, device=dev)["tile"]
    torch.cuda.synchronize()
    offered = sum(s.pixels * s.fps * s.lifetime_s for s in sessions) / (
        max(s.arrival_s + s.lifetime_s for s in sessions) - min(s.arrival_s for s in sessions)) / 1e9
    out = {"sessions": len(sessions), "time_scale": time_scale, "fps_scale": fps_scale,
           "offered_gpix_per_s_avg": offered, "budget_gb": 64, "max_group": max_group}
    for mode in ("batched", "plain"):
        ex = (serve.BatchedExecutor(rings, max_frames=32 * max_group, stream=stream, tiles=tiles, use_graph=False)
              if mode == "batched"
              else serve.PlainExecutor(rings, stream=stream, tiles=tiles))
        st = serve.Scheduler(ex, budget_bytes=64 * 10**9, max_active=32, max_group=max_group).run(sessions)
        out[mode] = st.summary()
        log(f"{label} {mode}: {out[mode]['frames']} frames, {out[mode]['gpix_per_s']:.2f} Gpix/s, "
            f"p50 {out[mode]['latency_ms_p50']:.3f} ms, p99 {out[mode]['latency_ms_p99']:.3f} ms, "
            f"{out[mode]['frames_per_tick']:.2f} frames/tick, largest group {st.max_group}")
        del ex
        torch.cuda.synchronize()
    out["batched_over_plain_throughput"] = out["batched"]["gpix_per_s"] / out["plain"]["gpix_per_s"]
    return out


def reprojection(dev, stream, spec, steps: int, warmup: int, ring: int, tile) -> dict:
    """The moving-camera workload at the headline size: a ring of `ring` distinct frames (camera
    pan and occluder both periodic in it) resident in HBM, `steps` reprojected frames timed after
    `warmup` untimed ones on a throwaway context."""
    import numpy as np
    import torch

    from paper_2510_03964_amd import fwrs, synth

    tol = 0.1
    gaze = synth.gaze_trace(spec, ring)
    src = synth.MovingSource(spec, device=dev, gaze=gaze)
    assert ring % src.motion.period == 0, "the ring must hold whole motion periods"
    log(f"reprojection: generating {ring} moving frames of {spec.width}x{spec.height}")
    t0 = time.perf_counter()
    frames = []
    for t in range(ring):
        frames.append(src.frame(t))
        if (t + 1) % 60 == 0:
            torch.cuda.synchronize()
            log(f"  {t + 1} frames")
    torch.cuda.synchronize()
    log(f"  resident ({time.perf_counter() - t0:.1f} s)")
    p = fwrs.default_params(spec.width, fovea_radius_px=spec.fovea_radius_px, seed=synth.PHILOX_SEED,
                            flags=fwrs.FLAG_REPROJECT)
    out = torch.empty((spec.height, spec.width, 3), dtype=torch.float32, device=dev)

    def run(res, n):
        def step(c, lev, mv, d, gx, gy, o):
            res.step_reproject(c, lev, mv, d, gx, gy, tol, o)
        return timed_run(res, [frames[t % ring] for t in range(n)], out, stream, step)

    warm = fwrs.Reservoir(spec.width, spec.height, spec.k, p, stream=stream)
    if tile:
        warm.set_tile(*tile)
    run(warm, max(warmup, 2))
    warm.close()
    res = fwrs.Reservoir(spec.width, spec.height, spec.k, p, stream=stream)
    if tile:
        res.set_tile(*tile)
    total_ms, per = run(res, steps)
    takes, changed, updates = res.stats()
    flushed = res.flushes()
    res.close()
    del frames
    torch.cuda.empty_cache()
    B = bytes_per_update_reproject(spec.k)
    kern = float(per.mean())
    ach = spec.pixels * B / (kern / 1e3) / 1e9
    log(f"reprojection: {total_ms / steps:.4f} ms/frame")
    return {"entry": "fwrs_push_frame_reproject", "frames": steps, "ring": ring,
            "workload": f"{spec.width}x{spec.height} k={spec.k}: lateral camera pan (4% of the width, "
                        f"240-frame back-and-forth) and a moving occluding disc, motion vectors + depth, "
                        f"relative depth tolerance {tol}",
            "ms_per_step": total_ms / steps, "value": spec.pixels * steps / (total_ms / 1e3) / 1e9,
            "unit": "Gpixel-updates/s", "ms_per_frame_p50": float(np.percentile(per, 50)),
            "ms_per_frame_p99": float(np.percentile(per, 99)),
            "flushed_per_pixel_update": flushed / updates, "slot_takes_per_pixel_update": takes / updates,
            "roofline": {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                         "frac": ach / HBM_PEAK_GBPS, "kernel_ms_avg": kern, "bytes_per_pixel_update": B}}


ABLATION_MODES = (("none", 0), ("bernoulli", 1), ("full_eq7", 2), ("memoryless", 3), ("aes", 4))


def ablations(dev, stream, spec, frames, tile, sample_every: int = 10) -> dict:
    """The update rules side by side on the headline frames (4K, k = 4, static camera): A-Chao
    without bias, with the Bernoulli bias (Eq. 6), with Eq. 7, with the memory-less bias, and
    A-ES.  Per mode: the fused pass's time per frame (one pass, per-launch HIP events), and in a
    second pass the retention of full-fidelity samples -- over the pixels that have been inside
    the fovea at some frame but are outside it now, the fraction of slots still holding a
    level-0 sample (weight 1) -- sampled every `sample_every` frames from the store in a
    caller-owned arena."""
    import numpy as np
    import torch

    from paper_2510_03964_amd import fwrs, synth

    out = torch.empty((spec.height, spec.width, 3), dtype=torch.float32, device=dev)
    N, k = spec.pixels, spec.k
    result = {}
    for name, mode in ABLATION_MODES:
        p = fwrs.default_params(spec.width, fovea_radius_px=spec.fovea_radius_px, seed=synth.PHILOX_SEED,
                                bias_mode=mode)
        arena = torch.empty(fwrs.state_bytes(spec.width, spec.height, k, p), dtype=torch.uint8, device=dev)
        res = fwrs.Reservoir(spec.width, spec.height, k, p, stream=stream, arena=arena)
        if tile:
            res.set_tile(*tile)
        total_ms, per = timed_run(res, frames, out, stream, res.step)
        takes, _, updates = res.stats()
        rbar = takes / updates
        per_slot = mode in (fwrs.BIAS_FULL, fwrs.AES)
        B = bytes_per_update_eq7(k, rbar) if per_slot else bytes_per_update(k, rbar)
        gbps = N * B / (float(per.mean()) / 1e3) / 1e9
        res.reset()
        view = res.state_view()
        ws = view.wsum_slots
        wt = arena.view(torch.float32)[ws * view.pitch: ws * view.pitch + 4 * k * N].view(N, k, 4)[:, :, 0]
        ever = torch.zeros(N, dtype=torch.bool, device=dev)
        fracs = []
        for t, (c, lev, gx, gy) in enumerate(frames):
            res.step(c, lev, gx, gy, out)
            l0 = lev.view(-1) == 0
            ever |= l0
            if (t + 1) % sample_every == 0:
                sel = ever & ~l0
                n_sel = int(sel.sum())
                if n_sel:
                    fracs.append(float((wt[sel] == 1.0).float().mean()))
        torch.cuda.synchronize()
        res.close()
        del arena
        result[name] = {"bias_mode": mode, "ms_per_frame": total_ms / len(frames),
                        "kernel_ms_avg": float(per.mean()),
                        "hbm": {"achieved": gbps, "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": gbps / HBM_PEAK_GBPS,
                                "bytes_per_pixel_update": B, "slot_takes_per_pixel_update": rbar,
                                "bytes_model": ("25 + 24k + 20r (per-slot sums, every record read)" if per_slot
                                                else "41 + 16k + 20r (whole trace; counts the record reads that the resolve "
                                                     "plane avoids from frame 32, so frac is an effective bandwidth and "
                                                     "exceeds 1 where few pixels change)")},
                        "level0_retention_mean": float(np.mean(fracs)) if fracs else None,
                        "level0_retention_last": fracs[-1] if fracs else None}
        log(f"ablation {name}: {total_ms / len(frames):.4f} ms/frame, {gbps / HBM_PEAK_GBPS:.3f} of HBM, level-0 retention "
            f"{result[name]['level0_retention_mean']:.4f}")
    result["definition"] = ("fraction of slots holding a weight-1 (level-0) sample over the pixels that were "
                            f"in the fovea earlier but are not now, sampled every {sample_every} frames")
    return result


def foveated(dev, stream, spec, steps: int, tile) -> dict:
    """The foveation generator ahead of the reservoir pass at the headline size: the full-resolution
    scene frame, degraded per gaze sample by mipmap + bilinear filtering (and by the Gaussian
    levels), timed (a) as the generator writing a frame + level map followed by the plain fused
    pass, and (b) as the fused form, where the reservoir pass samples the level images directly."""
    import numpy as np
    import torch

    from paper_2510_03964_amd import fwrs, synth

    full = synth.scene(spec.width, spec.height, spec.stream_id, device=dev)
    gaze = synth.gaze_trace(spec, steps)
    p = fwrs.default_params(spec.width, fovea_radius_px=spec.fovea_radius_px, seed=synth.PHILOX_SEED)
    out = torch.empty((spec.height, spec.width, 3), dtype=torch.float32, device=dev)
    col = torch.empty_like(out)
    lev = torch.empty((spec.height, spec.width), dtype=torch.uint8, device=dev)
    result = {}
    for name, mode in (("mip_bilinear", fwrs.FOV_MIP), ("gaussian", fwrs.FOV_GAUSS)):
        fov = fwrs.Foveator(spec.width, spec.height, spec.fovea_radius_px, spec.ring_radius_px, mode, stream=stream)
        runs = {}
        for form in ("separate", "fused"):
            res = fwrs.Reservoir(spec.width, spec.height, spec.k, p, stream=stream)
            if tile:
                res.set_tile(*tile)

            def step(gx, gy, o, _res=res, _fov=fov, _form=form):
                if _form == "fused":
                    _res.step_foveated(_fov, full, gx, gy, o)
                else:
                    _fov.foveate(full, gx, gy, col, lev)
                    _res.step(col, lev, gx, gy, o)
            for t in range(3):
                step(float(gaze[t, 0]), float(gaze[t, 1]), out)
            res.reset()
            total_ms, per = timed_run(res, [(float(g[0]), float(g[1])) for g in gaze], out, stream, step)
            runs[form] = {"ms_per_frame": total_ms / steps, "ms_per_frame_p50": float(np.percentile(per, 50)),
                          "value": spec.pixels * steps / (total_ms / 1e3) / 1e9}
            res.close()
        fov.close()
        runs["unit"] = "Gpixel-updates/s"
        runs["fused_speedup"] = runs["separate"]["ms_per_frame"] / runs["fused"]["ms_per_frame"]
        result[name] = runs
        log(f"foveated {name}: separate {runs['separate']['ms_per_frame']:.4f} ms, "
            f"fused {runs['fused']['ms_per_frame']:.4f} ms/frame")
    result["workload"] = (f"{spec.width}x{spec.height} k={spec.k} full-resolution scene frame, {steps}-frame gaze "
                          f"trace, rings {spec.fovea_radius_px:g}/{spec.ring_radius_px:g} px, Bernoulli bias")
    return result


def cpu_baseline(frames_host, spec, n_frames: int, threads: int = 16) -> dict:
    """The C oracle on the host: single-threaded over the first n_frames frames (the baseline's value), and
    the same frames again with each frame's update and resolve split into row bands over `threads`
    threads (pixels are independent, so the bands give the same results; at most 16 threads, the GPU's
    share of the host)."""
    from concurrent.futures import ThreadPoolExecutor

    import numpy as np

    import oracle

    q = oracle.default_params(spec.width, fovea_radius_px=spec.fovea_radius_px, seed=0x25103964)
    o = oracle.Oracle(spec.width, spec.height, spec.k, q)
    t0 = time.perf_counter()
    for (c, lev, gx, gy) in frames_host[:n_frames]:
        o.push(c, lev, gx, gy)
        o.resolve()
    dt = time.perf_counter() - t0
    o.close()
    px = spec.pixels * n_frames
    nt = max(1, min(threads, os.cpu_count() or 1))
    cuts = [spec.height * i // nt for i in range(nt + 1)]
    bands = list(zip(cuts[:-1], cuts[1:]))
    o = oracle.Oracle(spec.width, spec.height, spec.k, q)
    out = np.empty((spec.height, spec.width, 3), np.float64)
    with ThreadPoolExecutor(nt) as pool:
        t0 = time.perf_counter()
        for (c, lev, gx, gy) in frames_host[:n_frames]:
            list(pool.map(lambda b: o.push_rows(c, lev, gx, gy, b[0], b[1]), bands))
            o.advance()
            list(pool.map(lambda b: o.resolve_rows(out, b[0], b[1]), bands))
        dtp = time.perf_counter() - t0
    o.close()
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), model)
    except OSError:
        pass
    return {"value": px / dt / 1e9, "unit": "Gpixel-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"first {n_frames} frames of the same 3840x2160 k=4 trace, full frames, update + resolve, "
                      f"single-threaded C oracle ({dt:.1f} s)", "ms_per_frame": 1000.0 * dt / n_frames,
            "parallel": {"value": px / dtp / 1e9, "unit": "Gpixel-updates/s", "cores": nt,
                         "ms_per_frame": 1000.0 * dtp / n_frames,
                         "sample": f"the same {n_frames} frames, each frame's update and resolve as {nt} row bands "
                                   f"on {nt} threads ({dtp:.1f} s)"},
            "cpu_model": model, "host_threads_available": os.cpu_count()}


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


def headline(dev, stream, spec, frames, steps: int, warmup: int, fps: int, tile) -> dict:
    """The timed trace (see the module docstring) and its rooflines; a second, untimed pass over the same
    frames reads the slot counters at frames 20 and PLANE_FROM (results are deterministic, so its counts are
    the timed run's) for the slot replacements per pixel-update of each window."""
    import numpy as np
    import torch

    from paper_2510_03964_amd import fwrs, synth

    p = fwrs.default_params(spec.width, fovea_radius_px=spec.fovea_radius_px, seed=synth.PHILOX_SEED)
    out = torch.empty((spec.height, spec.width, 3), dtype=torch.float32, device=dev)

    def context():
        r = fwrs.Reservoir(spec.width, spec.height, spec.k, p, stream=stream)
        r.set_resolve_plane_from(PLANE_FROM)
        if tile:
            r.set_tile(*tile)
        return r

    n = len(frames)
    warm = context()
    for t in range(warmup * fps):
        warm.step(*frames[t % n], out)
    warm.sync()
    warm.close()
    log(f"dispatch plan: warm-up frames 0..{warmup * fps - 1} on a throwaway context, then the timed frames "
        f"0..{n - 1}, then the same frames untimed for the counters")
    res = context()
    total_ms, per = timed_run(res, frames, out, stream, res.step)
    takes, changed, updates = res.stats()
    assert updates == n * spec.pixels and res.frame_index == n
    res.close()
    # slot replacements per window, from an identical untimed pass
    cnt = context()
    marks = {}
    for t in range(n):
        if t in (20, PLANE_FROM):
            marks[t] = cnt.stats()
        cnt.step(*frames[t], out)
    end = cnt.stats()
    cnt.close()
    assert end[0] == takes, "the untimed pass must replay the timed one"
    N, k = spec.pixels, spec.k

    def rbar(a, b):
        ta = marks[a][0] if a else 0
        tb = marks[b][0] if b < n else end[0]
        return (tb - ta) / ((b - a) * N)

    window = {"steps": steps, "frames_per_step": fps, "frames": n}
    t_cached = float(per[PLANE_FROM:].mean())
    r_cached = rbar(PLANE_FROM, n)
    B = bytes_per_update(k, r_cached)
    B33 = bytes_per_update_33(k, r_cached)
    ach = N * B / (t_cached / 1e3) / 1e9
    traffic = traffic_from_counters(KERNEL_CACHED, N, window)
    vpp = valu_per_pixel(KERNEL_CACHED)
    roof = {"bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": ach / HBM_PEAK_GBPS,
            "traffic": traffic,
            "traffic_frac": None if traffic is None else traffic / (t_cached / 1e3) / 1e9 / HBM_PEAK_GBPS,
            "kernel": f"{KERNEL_CACHED} (fused update + resolve, unchanged pixels from the resolve plane)",
            "frames": [PLANE_FROM, n], "launches": n - PLANE_FROM, "kernel_ms_avg": t_cached,
            "bytes_per_pixel_update": B, "bytes_model": "41 + 16k + 20r (update + resolve, per-pixel count plane included)",
            "slot_takes_per_pixel_update": r_cached,
            "bytes_model_33": {"bytes_per_pixel_update": B33,
                               "frac": N * B33 / (t_cached / 1e3) / 1e9 / HBM_PEAK_GBPS,
                               "model": "33 + 16k + 20r (no per-pixel count plane)"},
            "valu_per_pixel": vpp,
            "valu_tops": None if vpp is None else N * vpp / (t_cached / 1e3) / 1e12}
    if vpp is not None:
        roof["valu_frac"] = roof["valu_tops"] / VALU_PEAK_TOPS
    r_all = takes / updates
    t_all = float(per.mean())
    trace = {"frames": n, "kernel_ms_avg": t_all, "ms_per_frame": total_ms / n,
             "slot_takes_per_pixel_update": r_all, "bytes_per_pixel_update": bytes_per_update(k, r_all),
             "frac": N * bytes_per_update(k, r_all) / (t_all / 1e3) / 1e9 / HBM_PEAK_GBPS,
             "pixels_changed_per_pixel_update": changed / updates,
             "by_kernel": {KERNEL_PLAIN: {"frames": [0, PLANE_FROM - 1], "kernel_ms_avg": float(per[:PLANE_FROM - 1].mean())},
                           KERNEL_FILL: {"frames": [PLANE_FROM - 1, PLANE_FROM],
                                         "kernel_ms_avg": float(per[PLANE_FROM - 1])},
                           KERNEL_CACHED: {"frames": [PLANE_FROM, n], "kernel_ms_avg": t_cached}}}
    r20 = rbar(0, 20)
    t20 = float(per[:20].mean())
    first20 = {"frames": [0, 20], "kernel_ms_avg": t20, "slot_takes_per_pixel_update": r20,
               "bytes_per_pixel_update": bytes_per_update(k, r20),
               "frac": N * bytes_per_update(k, r20) / (t20 / 1e3) / 1e9 / HBM_PEAK_GBPS}
    log(f"trace: {total_ms / n:.4f} ms/frame; dominant kernel {t_cached * 1e3:.1f} us = {roof['frac']:.3f} of HBM "
        f"(41 + 16k + 20r bytes), first 20 frames {t20 * 1e3:.1f} us")
    return {"total_ms": total_ms, "per": per, "roofline": roof, "trace": trace, "first_20_frames": first20,
            "changed": changed / updates}


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20, help="timed steps; a step is ceil(600 / steps) consecutive frames")
    ap.add_argument("--warmup", type=int, default=5, help="untimed steps on a throwaway context")
    ap.add_argument("--cpu-frames", type=int, default=24, help="frames of the oracle CPU baseline (0: skip)")
    ap.add_argument("--tile", type=str, default="", help="tile_x,tile_y override")
    ap.add_argument("--headline-only", action="store_true",
                    help="run only the timed trace and the copy reference (for profiling)")
    ap.add_argument("--no-copy", action="store_true", help="skip the copy-bandwidth reference")
    ap.add_argument("--no-incremental", action="store_true", help="skip the incremental-resolve run")
    ap.add_argument("--no-eq7", action="store_true", help="skip the Eq. 7 (full temporal bias) run")
    ap.add_argument("--no-ablations", action="store_true", help="skip the update-rule comparison")
    ap.add_argument("--no-foveated", action="store_true", help="skip the foveation-generator runs")
    ap.add_argument("--no-reproject", action="store_true", help="skip the moving-camera (reprojection) run")
    ap.add_argument("--reproject-ring", type=int, default=240, help="distinct moving frames kept resident")
    ap.add_argument("--no-multistream", action="store_true", help="skip the batched-vs-plain runs")
    ap.add_argument("--ring", type=int, default=48, help="distinct frames per stream kept resident (multistream)")
    ap.add_argument("--no-groups", action="store_true", help="skip the grouped-frames run")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving runs")
    ap.add_argument("--serving-scale", type=float, default=0.25, help="time compression of the serving run")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}): every pixel stream is independent "
              "and this benchmark measures the single-GPU pass.", file=sys.stderr)
        return 2
    if args.steps < 1 or args.warmup < 0:
        print("--steps must be >= 1 and --warmup >= 0", file=sys.stderr)
        return 2
    if args.headline_only:
        # the copy-bandwidth reference stays: it is the counters' calibration kernel
        for name in ("no_incremental", "no_eq7", "no_ablations", "no_foveated", "no_reproject",
                     "no_multistream", "no_groups", "no_serving"):
            setattr(args, name, True)
        args.cpu_frames = 0

    import numpy as np
    import torch

    from paper_2510_03964_amd import fwrs, synth

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    K, W = args.steps, args.warmup
    fps = max(1, math.ceil(TRACE_FRAMES / K))          # frames per step
    n_frames = K * fps                                  # the timed frames: the whole trace (or more)
    spec = synth.spec_4k(frames=max(TRACE_FRAMES, n_frames))
    log(f"generating {n_frames} frames of {spec.width}x{spec.height} on {torch.cuda.get_device_name(0)}")
    src = synth.FrameSource(spec, device=dev, n_frames=n_frames)
    t0 = time.perf_counter()
    frames = []
    for t in range(n_frames):
        frames.append(src.frame(t))
        if (t + 1) % 100 == 0:
            torch.cuda.synchronize()
            log(f"  {t + 1} frames")
    torch.cuda.synchronize()
    log(f"frames resident in HBM ({time.perf_counter() - t0:.1f} s)")

    p = fwrs.default_params(spec.width, fovea_radius_px=spec.fovea_radius_px, seed=synth.PHILOX_SEED)
    tile = tuple(int(v) for v in args.tile.split(",")) if args.tile else None
    out = torch.empty((spec.height, spec.width, 3), dtype=torch.float32, device=dev)

    h = headline(dev, stream, spec, frames, K, W, fps, tile)
    total_ms, per = h["total_ms"], h["per"]
    log(f"timed {n_frames} frames: {total_ms:.2f} ms on the GPU clock")
    ms_per_step = total_ms / K
    value = spec.pixels * n_frames / (total_ms / 1e3) / 1e9

    incremental = None
    if not args.no_incremental:
        inc = fwrs.Reservoir(spec.width, spec.height, spec.k, p, stream=stream)
        if tile:
            inc.set_tile(*tile)
        inc.step(*frames[0], out)            # frame 0: every pixel takes, full resolve
        inc_ms, inc_per = timed_run(inc, frames[1:], out, stream, inc.step_incremental)
        i_takes, i_changed, i_updates = inc.stats()
        inc.close()
        n_inc = n_frames - 1
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
                                    "frac": i_ach / HBM_PEAK_GBPS,
                                    "traffic": traffic_from_counters(
                                        "void fwrs::frame_kernel<4, 5, false>(fwrs::FrameDesc)", spec.pixels,
                                        {"steps": K, "frames_per_step": fps, "frames": n_frames}, INC_COUNTERS),
                                    "kernel_ms_avg": i_kern,
                                    "bytes_per_pixel_update": i_B, "slot_takes_per_pixel_update": i_rbar,
                                    "changed_pixel_fraction": i_changed_frac}}
        log(f"incremental: {inc_ms / n_inc:.4f} ms/frame")

    eq7 = None
    if not args.no_eq7:
        pf = fwrs.default_params(spec.width, fovea_radius_px=spec.fovea_radius_px, seed=synth.PHILOX_SEED,
                                 bias_mode=fwrs.BIAS_FULL)
        full = fwrs.Reservoir(spec.width, spec.height, spec.k, pf, stream=stream)
        if tile:
            full.set_tile(*tile)
        for t in range(min(W, 8)):
            full.step(*frames[t], out)
        full.reset()
        f_ms, f_per = timed_run(full, frames, out, stream, full.step)
        f_takes, f_changed, f_updates = full.stats()
        full.close()
        f_rbar = f_takes / f_updates
        f_B = bytes_per_update_eq7(spec.k, f_rbar)
        f_kern = float(f_per.mean())
        f_ach = spec.pixels * f_B / (f_kern / 1e3) / 1e9
        e7_kernel = "void fwrs::frame_kernel<4, 3, true>(fwrs::FrameDesc)"
        vpp = valu_per_pixel(e7_kernel)
        alu = None
        if vpp is not None:
            a_t = spec.pixels * vpp / (f_kern / 1e3) / 1e12
            alu = {"bound": "alu", "achieved": a_t, "peak": VALU_PEAK_TOPS, "unit": "T VALU lane-ops/s",
                   "frac": a_t / VALU_PEAK_TOPS, "valu_per_pixel": vpp,
                   "wave_insts_per_cu_clock": a_t * 1e12 / 64.0 / 256.0 / 2.4e9,
                   "note": "all VALU instructions (SQ_INSTS_VALU) against one non-packed wave64 instruction per CU "
                           "and clock",
                   "kernel": "fwrs::frame_kernel<4, 3, true> (Eq. 7)"}
        eq7 = {"entry": "fwrs_push_frame_resolve (FWRS_BIAS_FULL)", "frames": n_frames,
               "ms_per_frame": f_ms / n_frames,
               "value": spec.pixels * n_frames / (f_ms / 1e3) / 1e9, "unit": "Gpixel-updates/s",
               "ms_per_frame_p50": float(np.percentile(f_per, 50)),
               "ms_per_frame_p99": float(np.percentile(f_per, 99)),
               "roofline": {"bound": "hbm", "achieved": f_ach, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                            "frac": f_ach / HBM_PEAK_GBPS,
                            "traffic": traffic_from_counters(
                                e7_kernel, spec.pixels, {"steps": K, "frames_per_step": fps, "frames": n_frames},
                                EQ7_COUNTERS),
                            "kernel_ms_avg": f_kern, "bytes_per_pixel_update": f_B,
                            "slot_takes_per_pixel_update": f_rbar},
               "valu": alu}
        log(f"eq7: {f_ms / n_frames:.4f} ms/frame")

    ablation = None if args.no_ablations else ablations(dev, stream, spec, frames, tile)

    groups = None if args.no_groups else group_ticks(dev, stream, spec, frames, tile)

    copy_gbps = None if args.no_copy else copy_bandwidth(torch, dev)

    host = [(c.cpu().numpy(), lev.cpu().numpy(), gx, gy) for (c, lev, gx, gy) in frames[:args.cpu_frames]]

    del frames
    torch.cuda.empty_cache()

    fov = None if args.no_foveated else foveated(dev, stream, spec, n_frames, tile)

    reproject = None
    if not args.no_reproject:
        reproject = reprojection(dev, stream, spec, n_frames, 10, args.reproject_ring, tile)

    multi = None
    if not args.no_multistream:
        left, right = synth.spec_stereo()
        g_left = synth.gaze_trace(left)
        g_right = g_left + np.array([synth.vergence_shift(), 0.0], dtype=np.float32)
        g_right[:, 0] = np.clip(g_right[:, 0], 0.0, float(right.width))
        multi = {
            "stereo_2x2064x2208_k8": multistream(dev, stream, [left, right], [g_left, g_right], ticks=900,
                                                 ring=args.ring, use_graph=True, label="stereo"),
        }
        uneven = synth.spec_uneven()
        multi["uneven_16_streams"] = multistream(dev, stream, uneven, [synth.gaze_trace(s) for s in uneven],
                                                 ticks=300, ring=args.ring, use_graph=True, label="uneven")

    served = None
    if not args.no_serving:
        torch.cuda.empty_cache()
        served = {"paced": serving(dev, stream, args.serving_scale, 1.0, 24, "serving"),
                  "saturated": serving(dev, stream, 0.4 * args.serving_scale, 8.0, 24, "saturated")}

    cpu = None
    if args.cpu_frames > 0:
        log(f"timing the CPU oracle on {args.cpu_frames} frames")
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
        "config": {"workload": f"3840x2160 RGB f32 foveated frames, k=4, Bernoulli bias: the {n_frames}-frame "
                               f"synthetic gaze trace (fovea 216 px, ring 540 px) from an empty reservoir, timed "
                               f"frames 0-{n_frames - 1} as {K} steps of {fps} frames (one fused update + resolve "
                               f"launch per frame)",
                   "width": spec.width, "height": spec.height, "k": spec.k, "frames": n_frames,
                   "frames_per_step": fps, "timed_frames": [0, n_frames], "bias": "bernoulli",
                   "resolve_plane_from_frame": PLANE_FROM, "tile": list(tile) if tile else "default"},
        "roofline": h["roofline"],
        "trace": h["trace"],
        "first_20_frames": h["first_20_frames"],
        "ms_per_frame": total_ms / n_frames,
        "cpu_baseline": cpu,
        "ms_per_frame_p50": float(np.percentile(per, 50)),
        "ms_per_frame_p99": float(np.percentile(per, 99)),
        "pixels_changed_per_pixel_update": h["changed"],
        "incremental": incremental,
        "eq7": eq7,
        "reproject": reproject,
        "ablations": ablation,
        "foveated": fov,
        "multistream": multi,
        "groups": groups,
        "serving": served,
        "copy_gbps": copy_gbps,
    }
    print(json.dumps(line), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
