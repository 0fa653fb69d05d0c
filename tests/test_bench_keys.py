"""bench.py attaches measured counters (HBM traffic, VALU instructions) to a run only when the counter
summary was taken on the same kernel sources, frame size and timed window (CPU only)."""
from __future__ import annotations

import json
import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

KERNEL = bench.KERNEL_CACHED
N = 3840 * 2160
WINDOW = {"steps": 20, "frames_per_step": 30, "frames": 600}


def _summary(tmp_path, **over):
    c = {"source_hash": bench.kernel_source_hash(), "pixels": N, "window": dict(WINDOW),
         "fetch_scale": 2.0, "write_scale": 1.0,
         "kernels": {KERNEL: {"fetch_kib_per_dispatch": 100.0, "write_kib_per_dispatch": 50.0}}}
    c.update(over)
    path = tmp_path / "counters.json"
    path.write_text(json.dumps(c))
    return str(path)


def test_matching_summary_gives_scaled_bytes(tmp_path):
    got = bench.traffic_from_counters(KERNEL, N, dict(WINDOW), _summary(tmp_path))
    assert got == 1024.0 * (100.0 * 2.0 + 50.0 * 1.0)


@pytest.mark.parametrize("field,value", [
    ("source_hash", "0000000000000000"),
    ("pixels", N // 4),
    ("window", {"steps": 10, "frames_per_step": 60, "frames": 600}),
    ("window", {"steps": 20, "frames_per_step": 1, "frames": 20}),
])
def test_any_mismatch_gives_none(tmp_path, field, value):
    assert bench.traffic_from_counters(KERNEL, N, dict(WINDOW), _summary(tmp_path, **{field: value})) is None


def test_other_kernel_or_missing_file_gives_none(tmp_path):
    path = _summary(tmp_path)
    assert bench.traffic_from_counters(bench.KERNEL_PLAIN, N, dict(WINDOW), path) is None
    assert bench.traffic_from_counters(KERNEL, N, dict(WINDOW), str(tmp_path / "absent.json")) is None


def test_valu_counts_key_on_the_sources(tmp_path, monkeypatch):
    path = tmp_path / "valu.json"
    kern = "void fwrs::frame_kernel<4, 3, true>(fwrs::FrameDesc)"
    monkeypatch.setattr(bench, "VALU_COUNTERS", str(path))
    path.write_text(json.dumps({"source_hash": bench.kernel_source_hash(),
                                "kernels": {kern: {"valu_insts_per_wave": 539.0}}}))
    assert bench.valu_per_pixel(kern) == 539.0
    assert bench.valu_per_pixel(KERNEL) is None
    path.write_text(json.dumps({"source_hash": "stale", "kernels": {kern: {"valu_insts_per_wave": 539.0}}}))
    assert bench.valu_per_pixel(kern) is None


def test_committed_summaries_name_their_window_and_sources():
    """Every committed counter summary records the sources, frame size and window it was taken on."""
    for name in ("fused_k4_4k_counters.json", "incremental_k4_4k_counters.json", "eq7_k4_4k_counters.json"):
        with open(os.path.join(ROOT, "profiles", name)) as f:
            c = json.load(f)
        assert len(c["source_hash"]) == 16 and c["pixels"] == N, name
        assert set(c["window"]) == {"steps", "frames_per_step", "frames"}, name
        assert c["fetch_scale"] > 0 and c["write_scale"] > 0, name
