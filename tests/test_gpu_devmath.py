"""The kernels' binary32 math functions on the GPU against the oracle, bit for bit, over every input
of their ranges.

The device cube root starts from the GPU's own base-2 logarithm and exponential instructions, which the
host build of the same header (tests/test_devmath_host.py) replaces by libm's, so only a device run
checks the device code: every binary32 in the Lab curve's cube-root range [(6/29)^3, 2^8) and every
61st positive normal binary32 beyond must give the oracle's cube root (the binary32 nearest to the real
one), and every one of the 2^24 variates the oracle's log2.  The helper library is built by
__graft_entry__.build() (tests/pins/devmath_gpu.hip).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import pytest
import torch

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
HELPER = os.path.join(HERE, "pins", "libdevmath_gpu.so")
THREADS = 16


@pytest.fixture(scope="module")
def devmath():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(HELPER):
        raise RuntimeError(f"{HELPER} is missing: run __graft_entry__.build() first")
    L = C.CDLL(HELPER)
    L.gpu_cube_root_mismatches.restype = C.c_int64
    L.gpu_cube_root_mismatches.argtypes = [C.c_uint32, C.c_uint32, C.c_uint32, C.c_void_p, C.c_int,
                                           C.POINTER(C.c_uint32)]
    L.gpu_log2_unit_mismatches.restype = C.c_int64
    L.gpu_log2_unit_mismatches.argtypes = [C.c_void_p, C.c_int, C.POINTER(C.c_uint32)]
    return L


def _bits(x):
    return int(np.array([x], np.float32).view(np.uint32)[0])


def _oracle_fn(oracle_mod, name):
    return C.cast(getattr(oracle_mod.lib(), name), C.c_void_p)


def test_device_cube_root_equals_oracle_on_every_input(devmath, oracle_mod):
    ref = _oracle_fn(oracle_mod, "fwrs_oracle_cbrt")
    first = C.c_uint32()
    n = devmath.gpu_cube_root_mismatches(_bits(216.0 / 24389.0), _bits(256.0), 1, ref, THREADS, C.byref(first))
    assert n == 0, f"{n} inputs differ in [(6/29)^3, 2^8), first bits {first.value:#x}"
    n = devmath.gpu_cube_root_mismatches(0x00800000, 0x7F800000, 61, ref, THREADS, C.byref(first))
    assert n == 0, f"{n} sampled normal inputs differ, first bits {first.value:#x}"


def test_device_log2_unit_equals_oracle_on_every_variate(devmath, oracle_mod):
    ref = _oracle_fn(oracle_mod, "fwrs_oracle_log2u")
    first = C.c_uint32()
    n = devmath.gpu_log2_unit_mismatches(ref, THREADS, C.byref(first))
    assert n == 0, f"{n} variates differ, first bits {first.value:#x}"
