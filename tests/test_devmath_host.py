"""The kernels' binary32 math functions against the oracle, bit for bit, over every input of
their ranges (CPU only).

The device header is compiled for the host (tests/pins/devmath_host.cpp), so the functions the
gfx950 kernels inline are evaluated here on the CPU with the same IEEE operations (the cube root's
starting estimate excepted: the host build takes it from libm's log2 and exp2 where the device uses
its own instructions, so this checks the correction and rounding that follow it; the device code
itself is checked on the GPU by tests/test_gpu_devmath.py):
  - the cube root of Eq. 7's Lab conversion (Sec. 4.3) for every binary32 in the Lab curve's
    cube-root range [(6/29)^3, 2^8), and every 61st positive normal binary32 beyond;
  - log2 of the A-ES variate (Sec. 3.1) for all 2^24 variates;
  - Lab and the CIE94 difference on random colours, standard-range and HDR;
  - that a colour compared with an equal one (up to the sign of zeros) gives CIE94 exactly 0
    within the bound under which Eq. 7's kernels skip that evaluation, and not always beyond it.
The oracle's versions are the plain definitions (the nearest binary32 to the real cube root and
to the real log2), pinned in test_oracle_eq7.py and test_oracle_ablations.py.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
THREADS = 8


@pytest.fixture(scope="module")
def devmath(tmp_path_factory):
    src = os.path.join(HERE, "pins", "devmath_host.cpp")
    out = str(tmp_path_factory.mktemp("devmath") / "libdevmath_host.so")
    subprocess.run(["hipcc", "-O2", "-std=c++17", "-fPIC", "-shared", "-x", "hip", "--offload-host-only",
                    "-ffp-contract=off", "-o", out, src], check=True, capture_output=True)
    L = C.CDLL(out)
    L.cube_root_mismatches.restype = C.c_int64
    L.cube_root_mismatches.argtypes = [C.c_uint32, C.c_uint32, C.c_uint32, C.c_void_p, C.c_int,
                                       C.POINTER(C.c_uint32)]
    L.log2_unit_mismatches.restype = C.c_int64
    L.log2_unit_mismatches.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_uint32)]
    L.dev_lab.argtypes = [C.c_float, C.c_float, C.c_float, C.POINTER(C.c_float)]
    L.dev_de94.restype = C.c_float
    L.dev_de94.argtypes = [C.POINTER(C.c_float), C.POINTER(C.c_float)]
    L.dev_lab_bounded.restype = C.c_int
    L.dev_lab_bounded.argtypes = [C.c_float, C.c_float, C.c_float]
    return L


def _bits(x):
    return int(np.array([x], np.float32).view(np.uint32)[0])


def _oracle_fn(oracle_mod, name):
    """Address of one of the oracle library's functions (the C loop calls it directly)."""
    return C.cast(getattr(oracle_mod.lib(), name), C.c_void_p)


def test_cube_root_equals_oracle_on_every_input(devmath, oracle_mod):
    ref = _oracle_fn(oracle_mod, "fwrs_oracle_cbrt")
    first = C.c_uint32()
    lo, hi = _bits(216.0 / 24389.0), _bits(256.0)
    n = devmath.cube_root_mismatches(lo, hi, 1, ref, THREADS, C.byref(first))
    assert n == 0, f"{n} inputs differ in [(6/29)^3, 2^8), first bits {first.value:#x}"
    n = devmath.cube_root_mismatches(0x00800000, 0x7F800000, 61, ref, THREADS, C.byref(first))
    assert n == 0, f"{n} sampled normal inputs differ, first bits {first.value:#x}"


def test_log2_unit_equals_oracle_on_every_variate(devmath, oracle_mod):
    ref = _oracle_fn(oracle_mod, "fwrs_oracle_log2u")
    first = C.c_uint32()
    n = devmath.log2_unit_mismatches(ref, THREADS, C.byref(first))
    assert n == 0, f"{n} variates differ, first bits {first.value:#x}"


def test_lab_and_cie94_equal_oracle(devmath, oracle_mod):
    rng = np.random.Generator(np.random.PCG64(33))
    n = 20000
    rgb = np.concatenate([rng.random((n, 3)), 4.0 * rng.random((n // 4, 3)),
                          np.array([[0, 0, 0], [1, 1, 1], [1, 0, 0], [0, 1, 0], [0, 0, 1]])]).astype(np.float32)
    want = oracle_mod.lab(rgb)
    got = np.empty_like(want)
    buf = (C.c_float * 3)()
    for i, (r, g, b) in enumerate(rgb):
        devmath.dev_lab(float(r), float(g), float(b), buf)
        got[i] = buf[:]
    np.testing.assert_array_equal(got.view(np.uint32), want.view(np.uint32))
    # CIE94 of consecutive pairs, the first as the reference colour
    a, b = want[:-1], want[1:]
    want_de = oracle_mod.de94(a, b)
    ra, rb = (C.c_float * 3)(), (C.c_float * 3)()
    got_de = np.empty_like(want_de)
    for i in range(len(a)):
        ra[:] = a[i].tolist()
        rb[:] = b[i].tolist()
        got_de[i] = devmath.dev_de94(ra, rb)
    np.testing.assert_array_equal(got_de.view(np.uint32), want_de.view(np.uint32))


def test_equal_colours_have_zero_cie94_within_the_bound(devmath):
    """Eq. 7's kernels take |dL| = 0 without evaluating Lab and CIE94 when a sample's colour equals
    the new pixel's component by component and every component is below 2^24 in magnitude.  Here
    the device functions (host build) give the same: equal Lab triples, bit for bit, when zeros
    change sign, and CIE94 exactly +0, on colours spread over every binade up to 2^24, signed zeros
    and the components that maximise a* and b*.  Beyond the bound the chroma's squares can overflow
    and CIE94 of a colour with itself be NaN (so |dL| = 1), which is why the bound exists."""
    rng = np.random.default_rng(31)
    n = 20000
    mag = np.exp2(rng.uniform(-30.0, 24.0, size=(n, 3))).astype(np.float32)
    mag = np.minimum(mag, np.float32(16777215.0))
    col = np.where(rng.random((n, 3)) < 0.5, -mag, mag).astype(np.float32)
    col[rng.random((n, 3)) < 0.15] = 0.0
    B = np.float32(16777215.0)
    extremes = np.array([[B, -B, 0.0], [-B, B, 0.0], [0.0, B, -B], [B, 0.0, -B], [-B, -B, B], [B, B, B],
                         [-B, -B, -B], [0.0, 0.0, 0.0]], np.float32)
    col = np.concatenate([col, extremes])
    a = (C.c_float * 3)()
    b = (C.c_float * 3)()
    for c in col:
        flipped = np.where(c == 0.0, np.where(np.signbit(c), np.float32(0.0), np.float32(-0.0)), c)
        assert devmath.dev_lab_bounded(*map(float, c)) == 1
        devmath.dev_lab(*map(float, c), a)
        devmath.dev_lab(*map(float, flipped), b)
        la = np.frombuffer(a, np.float32).copy()
        lb = np.frombuffer(b, np.float32).copy()
        assert np.all(np.isfinite(la)), c
        np.testing.assert_array_equal(la.view(np.uint32), lb.view(np.uint32), err_msg=str(c))
        d = np.float32(devmath.dev_de94(a, b))
        assert d == 0.0 and not np.signbit(d), (c, d)
    assert devmath.dev_lab_bounded(16777216.0, 0.0, 0.0) == 0
    assert devmath.dev_lab_bounded(0.0, float("nan"), 0.0) == 0
    devmath.dev_lab(1e30, -1e30, 0.5, a)
    assert np.isnan(devmath.dev_de94(a, a))
