"""The C-ABI library loads and exports every symbol include/fwrs.h declares; host-side
argument handling (no GPU work).  CPU only."""
from __future__ import annotations

import ctypes as C
import os
import re
import subprocess

import pytest

from paper_2510_03964_amd import fwrs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fwrs.h")


def _declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(fwrs_[a-z_0-9]+)\s*\(", text, flags=re.M)))


def test_header_declares_the_binding_exports():
    assert _declared_functions() == sorted(fwrs.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = fwrs.load()
    for name in _declared_functions():
        assert hasattr(L, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", fwrs.LIB_PATH], capture_output=True, text=True, check=True)
    exported = set(re.findall(r"\bT (fwrs_[a-z_0-9]+)", out.stdout))
    assert set(_declared_functions()) <= exported
    # the C ABI exposes no C++ or torch types
    assert not re.search(r"\bT _Z\S*fwrs_", out.stdout)


def test_library_is_gfx950_code():
    out = subprocess.run(["strings", fwrs.LIB_PATH], capture_output=True, text=True, check=True).stdout
    assert "gfx950" in out


def test_header_compiles_as_plain_c(tmp_path):
    src = tmp_path / "t.c"
    src.write_text('#include "fwrs.h"\nint main(void){ fwrs_params p; return fwrs_default_params(64, &p); }\n')
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.dirname(HEADER), "-c", str(src), "-o",
                    str(tmp_path / "t.o")], check=True)


def test_struct_layouts_match_header(tmp_path):
    src = tmp_path / "l.c"
    src.write_text(
        '#include <stdio.h>\n#include <stddef.h>\n#include "fwrs.h"\n'
        "int main(void){printf(\"%zu %zu %zu %zu %zu\\n\", sizeof(fwrs_params), sizeof(fwrs_state_view),"
        " sizeof(fwrs_frame), offsetof(fwrs_frame, out), offsetof(fwrs_state_view, idx));"
        " printf(\"%zu %u\\n\", offsetof(fwrs_state_view, wsum_slots), FWRS_BIAS_FULL); return 0;}\n")
    exe = tmp_path / "l"
    subprocess.run(["gcc", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert got == [C.sizeof(fwrs.Params), C.sizeof(fwrs.StateView), C.sizeof(fwrs.Frame),
                   fwrs.Frame.out.offset, fwrs.StateView.idx.offset, fwrs.StateView.wsum_slots.offset,
                   fwrs.BIAS_FULL]


def test_default_params_and_sizes():
    p = fwrs.default_params(3840)
    assert p.fov_deg == 70.0 and p.fovea_radius_px == pytest.approx(192.0)
    assert p.bias_mode == fwrs.BIAS_BERNOULLI
    assert p.flags == 0 and p.lambda_decay == pytest.approx(0.0231)
    assert (p.a_k, p.r2k, p.rek) == (pytest.approx(0.9851), pytest.approx(1.058), pytest.approx(22.14))
    N = 3840 * 2160
    # w_sum, k records and frame indices, the resolve plane (3 floats per pixel)
    assert fwrs.state_bytes(3840, 2160, 4) == 4 * N * (1 + 20 + 3) + 24576      # N is a multiple of 64
    assert fwrs.state_host_bytes(3840, 2160, 4) == N * (8 + 96)
    assert fwrs.state_bytes(13, 7, 3) == 4 * 128 * (1 + 15 + 3) + 24576        # pitch rounded up to 64
    # Eq. 7 keeps one w_sum per slot
    def prm(**kw):
        return fwrs.default_params(13, **kw)
    for mode in (fwrs.BIAS_NONE, fwrs.BIAS_BERNOULLI):
        assert fwrs.state_bytes(13, 7, 3, prm(bias_mode=mode)) == fwrs.state_bytes(13, 7, 3)
    assert fwrs.state_bytes(3840, 2160, 4, prm(bias_mode=fwrs.BIAS_FULL)) == 4 * N * (4 + 20) + 24576
    assert fwrs.state_bytes(13, 7, 3, prm(bias_mode=fwrs.BIAS_FULL)) == 4 * 128 * (3 + 15) + 24576
    assert fwrs.state_bytes(13, 7, 3, prm(bias_mode=fwrs.BIAS_MEMORYLESS)) == fwrs.state_bytes(13, 7, 3)
    assert fwrs.state_bytes(13, 7, 3, prm(bias_mode=fwrs.AES)) == 4 * 128 * (3 + 15) + 24576
    assert fwrs.state_bytes(13, 7, 3, prm(bias_mode=5)) == 0
    # a reprojecting context keeps two banks, each with a count and a depth per pixel
    assert fwrs.state_bytes(13, 7, 3, prm(flags=fwrs.FLAG_REPROJECT)) == 2 * 4 * 128 * (1 + 15 + 2) + 24576
    assert fwrs.state_bytes(13, 7, 3, prm(flags=fwrs.FLAG_REPROJECT, bias_mode=fwrs.BIAS_FULL)) == \
        2 * 4 * 128 * (3 + 15 + 2) + 24576
    # without the resolve plane
    assert fwrs.state_bytes(13, 7, 3, prm(flags=fwrs.FLAG_NO_RESOLVE_PLANE)) == 4 * 128 * (1 + 15) + 24576
    assert fwrs.state_bytes(13, 7, 3, prm(flags=fwrs.FLAG_NO_RESOLVE_PLANE, bias_mode=fwrs.BIAS_FULL)) == \
        fwrs.state_bytes(13, 7, 3, prm(bias_mode=fwrs.BIAS_FULL))
    assert fwrs.state_bytes(13, 7, 3, prm(flags=4)) == 0
    for bad in [(0, 5, 4), (5, 0, 4), (5, 5, 0), (5, 5, 17), (65536, 65536, 1)]:
        assert fwrs.state_bytes(*bad) == 0


def test_invalid_arguments_are_rejected_before_any_gpu_work():
    L = fwrs.load()
    h = C.c_void_p()
    p = fwrs.default_params(64)
    assert L.fwrs_create(0, 10, 4, C.byref(h)) == fwrs.E_ARG
    assert L.fwrs_create(10, 10, 17, C.byref(h)) == fwrs.E_ARG
    assert L.fwrs_create(10, 10, 4, None) == fwrs.E_ARG
    for field, value in [("fov_deg", 0.0), ("fovea_radius_px", float("nan")), ("bias_mode", 7), ("a_k", 1.5),
                         ("r_m", -1.0), ("rek", float("inf")), ("flags", 6), ("bias_mode", 5),
                         ("lambda_decay", -0.5), ("lambda_decay", float("nan"))]:
        q = fwrs.default_params(64)
        setattr(q, field, value)
        assert L.fwrs_create_ex(64, 64, 4, C.byref(q), None, None, 0, C.byref(h)) == fwrs.E_ARG, field
    # a caller arena that is too small or misaligned
    assert L.fwrs_create_ex(64, 64, 4, C.byref(p), None, 256, 16, C.byref(h)) == fwrs.E_ARG
    assert L.fwrs_create_ex(64, 64, 4, C.byref(p), None, 4100, 1 << 30, C.byref(h)) == fwrs.E_ARG
    # an arena sized for the shared-sum layout without the resolve plane is too small under Eq. 7
    q = fwrs.default_params(64)
    q.bias_mode = fwrs.BIAS_FULL
    small = fwrs.state_bytes(64, 64, 4, fwrs.default_params(64, flags=fwrs.FLAG_NO_RESOLVE_PLANE))
    assert L.fwrs_create_ex(64, 64, 4, C.byref(q), None, 256, small, C.byref(h)) == fwrs.E_ARG
    assert L.fwrs_push_frame(None, None, None, 0.0, 0.0) == fwrs.E_ARG
    assert L.fwrs_push_frame_reproject(None, None, None, None, None, 0.0, 0.0, 0.1, None) == fwrs.E_ARG
    assert L.fwrs_resolve(None, None) == fwrs.E_ARG
    assert L.fwrs_destroy(None) == fwrs.OK
    assert L.fwrs_engine_destroy(None) == fwrs.OK
    assert L.fwrs_engine_create(None, 0, 0, C.byref(h)) == fwrs.E_ARG
    assert L.fwrs_engine_create(None, 4097, 0, C.byref(h)) == fwrs.E_ARG
    # fwrs_tick: an empty tick is a no-op; bad sizes and missing frames are rejected
    frames = (fwrs.Frame * 2)()
    assert L.fwrs_tick(None, 0, None) == fwrs.OK
    assert L.fwrs_tick(None, 1, None) == fwrs.E_ARG
    assert L.fwrs_tick(frames, -1, None) == fwrs.E_ARG
    assert L.fwrs_tick(frames, 4097, None) == fwrs.E_ARG
    assert L.fwrs_tick(frames, 2, None) == fwrs.E_ARG          # NULL contexts
    # foveation generator: argument checks come before any device work
    for args in [(0, 32, 5.0, 10.0, 0), (64, 32, 10.0, 5.0, 0), (64, 32, 5.0, 10.0, 7), (64, 32, float("nan"), 10.0, 0),
                 (64, 32, -1.0, 10.0, 0)]:
        assert L.fwrs_foveator_create(*args, None, C.byref(h)) == fwrs.E_ARG, args
    assert L.fwrs_foveator_create(64, 32, 5.0, 10.0, 0, None, None) == fwrs.E_ARG
    assert L.fwrs_foveate(None, None, 0.0, 0.0, None, None) == fwrs.E_ARG
    assert L.fwrs_push_frame_foveated(None, None, None, 0.0, 0.0, None) == fwrs.E_ARG
    assert L.fwrs_foveator_destroy(None) == fwrs.OK
    assert fwrs.strerror(fwrs.E_ARG) == "invalid argument"
    assert fwrs.strerror(99) == "unknown status"


@pytest.mark.parametrize("width,rf,lam", [(256, 32.0, 0.0231), (3840, 216.0, 0.0231), (2064, 103.0, 0.5), (37, 2.0, 0.0)])
def test_kernel_constants_are_the_oracles(width, rf, lam):
    """The constants the library derives on the host for its kernels equal the oracle's, bit for bit."""
    import numpy as np
    import oracle

    p = fwrs.default_params(width, fovea_radius_px=rf, lambda_decay=lam)
    got = fwrs.method_constants(width, p)
    o = oracle.Oracle(width, 4, 1, oracle.default_params(width, fovea_radius_px=rf, lambda_decay=lam))
    c = o.constants()
    want = np.array([c["A"], c["B"], c["IR2"], c["IRM"], c["C"], c["iPPD"], c["rf"], c["Drf"], o.decay], np.float32)
    np.testing.assert_array_equal(got.view(np.uint32), want.view(np.uint32))


@pytest.mark.parametrize("sigma", [1.0, 2.0, 0.7, 5.0])
def test_gaussian_weights_are_the_oracles(sigma):
    import numpy as np
    import oracle

    np.testing.assert_array_equal(fwrs.gauss_weights(sigma).view(np.uint32), oracle.gauss_weights(sigma).view(np.uint32))
    assert fwrs.load().fwrs_gauss_weights(float("nan"), (C.c_float * 65)()) == -1
    assert fwrs.load().fwrs_gauss_weights(20.0, (C.c_float * 65)()) == -1
