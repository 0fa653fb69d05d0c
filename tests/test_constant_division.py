"""The kernels divide by the constants 0.95047, 1.08883 (Lab white point) and 100 (dE94 scale)
with a product by the rounded reciprocal and one fused multiply-add of the residual, falling back
to the division outside 2^-100 <= |x| <= 2^126.  Within that range this equals the correctly rounded
quotient for every binary32 x (checked exhaustively when the method was adopted); this CPU test
re-checks a stride of 61 over all binary32 patterns, plus the range edges, with the C library's
fmaf.  No GPU."""
from __future__ import annotations

import subprocess

import pytest

SRC = r"""
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <string.h>
static float div_const(float x, float c, float rc) {
    float ax = fabsf(x);
    if (ax >= 0x1p-100f && ax <= 0x1p126f) { float q = x * rc; float r = fmaf(-q, c, x); return fmaf(r, rc, q); }
    return x / c;
}
int main(void) {
    const float cs[3] = {0.95047f, 1.08883f, 100.0f};
    const float rcs[3] = {0x1.0d5728p+0f, 0x1.d63ac2p-1f, 0x1.47ae14p-7f};
    unsigned long long bad = 0, n = 0;
    for (int k = 0; k < 3; ++k) {
        if (rcs[k] != 1.0f / cs[k]) { printf("reciprocal %d differs\n", k); return 2; }
        for (uint64_t b = 0; b < (1ull << 32); b += 61) {
            uint32_t u = (uint32_t)b; float x; memcpy(&x, &u, 4);
            if (!isfinite(x)) continue;
            float a = x / cs[k], g = div_const(x, cs[k], rcs[k]);
            if (memcmp(&a, &g, 4) != 0) { if (bad < 5) printf("c=%g x=%a want %a got %a\n", cs[k], x, a, g); ++bad; }
            ++n;
        }
        const float edges[6] = {0x1p-100f, -0x1p-100f, 0x1p126f, -0x1p126f, 0x1.fffffep-101f, 0x1.000002p126f};
        for (int e = 0; e < 6; ++e) {
            float a = edges[e] / cs[k], g = div_const(edges[e], cs[k], rcs[k]);
            if (memcmp(&a, &g, 4) != 0) { printf("edge %a\n", edges[e]); ++bad; }
        }
    }
    printf("%llu checked, %llu mismatches\n", n, bad);
    return bad != 0;
}
"""


def test_fma_corrected_constant_division_is_correctly_rounded(tmp_path):
    src = tmp_path / "d.c"
    src.write_text(SRC)
    exe = tmp_path / "d"
    subprocess.run(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-o", str(exe), str(src), "-lm"], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout
