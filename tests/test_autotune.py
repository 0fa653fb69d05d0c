"""The tile autotuner: cache handling on the CPU; on the GPU a tuned tile is one of the candidates,
is cached, and never changes results."""
from __future__ import annotations

import json

import numpy as np
import pytest
import torch

from paper_2510_03964_amd import autotune


def test_cache_roundtrip(tmp_path, monkeypatch):
    path = tmp_path / "sub" / "tiles.json"
    monkeypatch.setenv("FWRS_AUTOTUNE_CACHE", str(path))
    assert autotune.cache_path() == str(path)
    assert autotune.load_cache() == {}
    autotune.save_cache({"gfx950:64x32:k4": {"tile": [64, 1], "ms": {"64x1": 0.1}}})
    assert json.loads(path.read_text())["gfx950:64x32:k4"]["tile"] == [64, 1]
    assert autotune.load_cache()["gfx950:64x32:k4"]["tile"] == [64, 1]
    path.write_text("not json")
    assert autotune.load_cache() == {}


@pytest.mark.gpu
def test_tuned_tile_is_cached_and_never_changes_results(tmp_path, monkeypatch):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_03964_amd import fwrs, synth

    monkeypatch.setenv("FWRS_AUTOTUNE_CACHE", str(tmp_path / "tiles.json"))
    r = autotune.tune(320, 180, 4, frames=3, prime=2, reps=1)
    assert not r["cached"] and r["tile"] in [tuple(c) for c in autotune.CANDIDATES]
    assert set(r["ms"]) == {f"{x}x{y}" for (x, y) in autotune.CANDIDATES}
    again = autotune.tune(320, 180, 4, frames=3, prime=2, reps=1)
    assert again["cached"] and again["tile"] == r["tile"]
    # the tuned engine's output equals plain launches with the default tile
    dev = torch.device("cuda:0")
    stream = torch.cuda.current_stream()
    spec = synth.StreamSpec(320, 180, 4, 4, 16.0, 40.0, 2.0, 2, 6.0)
    src = synth.FrameSource(spec, device=dev)
    p = fwrs.default_params(spec.width, fovea_radius_px=spec.fovea_radius_px)
    eng = fwrs.Engine(1, stream=stream)
    autotune.tune_engine(eng, [(320, 180, 4)], device=dev, frames=3, prime=2, reps=1)
    a = fwrs.Reservoir(spec.width, spec.height, spec.k, p, stream=stream)
    b = fwrs.Reservoir(spec.width, spec.height, spec.k, p, stream=stream)
    oa = torch.empty((spec.height, spec.width, 3), device=dev)
    ob = torch.empty_like(oa)
    for t in range(4):
        f = src.frame(t)
        eng.tick([(a, *f, oa)])
        b.step(*f, ob)
    torch.cuda.synchronize()
    assert torch.equal(oa, ob)
    np.testing.assert_array_equal(a.download().idx, b.download().idx)
    eng.close()
