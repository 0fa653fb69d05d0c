"""Pins of the oracle's ablation modes (Sec. 3.1): A-ES keys and the memory-less bias, CPU only.

What fixes the expected values: log2 of the 2^24 possible variates against binary64 log2 and a
high-precision decimal log2; the
decay factor against binary64 exp; for a single stream, the Efraimidis-Spirakis theorem (the
largest key u^(1/w) belongs to item i with probability w_i / sum w) and the closed form of the
memory-less bias, P(final = i) = w_i d^(N-i) / sum_j w_j d^(N-j) with d = exp(-lambda), both by
chi-square over 10^5 Philox seeds; lambda = 0 is plain Alg. 2 bit for bit."""
from __future__ import annotations

import math
from decimal import Decimal, localcontext

import numpy as np
import pytest

from paper_2510_03964_amd import synth
from test_oracle_eq7 import _nearest_f32
from test_oracle_pins import P_REJECT, _chi2_pvalue, _pixel_stream, varied_pixel  # noqa: F401


def _log2_decimal(m):
    """log2(m) - 24 to 60 significant digits."""
    with localcontext() as ctx:
        ctx.prec = 60
        return Decimal(int(m)).ln() / Decimal(2).ln() - 24


def test_log2_of_every_variate(oracle_mod):
    """log2 of the variate is the binary32 nearest to log2(m) - 24: against binary64 log2 for all
    2^24 variates (the two agree wherever binary64 is not within 2^-30 ulp of a binary32
    midpoint), and against a 60-digit decimal log2 on random variates and on those nearest a
    midpoint; exact at the powers of two; monotone."""
    m = np.arange(1, 2 ** 24 + 1, dtype=np.uint64)
    bits = ((m - 1) << np.uint64(8)).astype(np.uint32)
    got = oracle_mod.log2u(bits)
    want64 = np.log2(m.astype(np.float64)) - 24.0
    nz = want64 != 0.0
    ulp = np.ldexp(1.0, np.floor(np.log2(np.abs(want64[nz]))).astype(np.int64) - 23)
    dist = np.abs((np.abs(want64[nz]) / ulp) % 1.0 - 0.5)       # distance to a midpoint, in ulps
    clear = dist > 2.0 ** -30
    assert np.array_equal(got[nz][clear], want64[nz][clear].astype(np.float32))
    assert got[~nz].tolist() == [0.0]
    rng = np.random.Generator(np.random.PCG64(32))
    pick = np.concatenate([rng.integers(1, 2 ** 24 + 1, 1000), m[nz][np.argsort(dist)[:300]].astype(np.int64)])
    for mi in pick:
        g = oracle_mod.log2u(np.array([(int(mi) - 1) << 8], np.uint32))[0]
        want = _nearest_f32(_log2_decimal(mi), np.float32(np.log2(float(mi)) - 24.0))
        assert g == want, f"log2 variate m={int(mi)}: {float(g)!r} vs nearest {float(want)!r}"
    # exact at the powers of two; monotone non-decreasing in the variate
    pw = np.array([2 ** e for e in range(25)], np.uint64)
    assert np.array_equal(oracle_mod.log2u(((pw - 1) << np.uint64(8)).astype(np.uint32)),
                          np.arange(25, dtype=np.float32) - 24)
    assert np.all(np.diff(got.astype(np.float64)) >= 0.0)
    # the low 8 bits of the word are not used
    assert np.array_equal(oracle_mod.log2u(bits[:1000] | np.uint32(0xFF)), got[:1000])


@pytest.mark.parametrize("lam", [0.0231, 0.001, 0.5, 2.0])
def test_decay_factor(oracle_mod, lam):
    p = oracle_mod.default_params(64, lambda_decay=lam)
    o = oracle_mod.Oracle(64, 32, 1, p)
    d = float(o.decay)
    want = math.exp(-np.float64(np.float32(lam)))
    assert abs(d - want) <= 4 * np.spacing(np.float32(want))


def test_default_lambda(oracle_mod):
    p = oracle_mod.default_params(64)
    assert p.lambda_decay == pytest.approx(0.0231)
    o = oracle_mod.Oracle(64, 32, 1, p)
    assert float(o.decay) ** 30 == pytest.approx(0.5, rel=0.01)      # a 30-frame half-life


@pytest.mark.parametrize("n_frames", [60, 20])
def test_aes_inclusion_is_proportional_to_weight(oracle_mod, varied_pixel, n_frames):
    """Efraimidis-Spirakis: the largest key rand^(1/w_i) belongs to frame i with probability
    w_i / sum_j w_j, the same law as A-Chao without bias."""
    spec, px, py = varied_pixel
    rgb, lev, gaze, w = _pixel_stream(oracle_mod, spec, px, py, n_frames)
    p = oracle_mod.default_params(spec.width, fovea_radius_px=spec.fovea_radius_px, bias_mode=oracle_mod.AES)
    idx, keys = oracle_mod.trials(spec.width, spec.height, 4, p, px, py, 11, 100_000, rgb, lev, gaze)
    counts = np.bincount(idx.reshape(-1), minlength=n_frames)
    probs = w.astype(np.float64) / w.astype(np.float64).sum()
    assert _chi2_pvalue(counts, probs) > P_REJECT
    assert np.all(keys <= 0.0) and np.all(np.isfinite(keys))


def test_aes_uniform_weights_give_uniform_inclusion(oracle_mod):
    N = 25
    p = oracle_mod.default_params(64, fovea_radius_px=3.0, bias_mode=oracle_mod.AES)
    rgb = np.zeros((N, 3), np.float32)
    lev = np.zeros(N, np.uint8)
    gaze = np.tile(np.array([[50.0, 10.0]], np.float32), (N, 1))
    idx, _ = oracle_mod.trials(64, 32, 8, p, 3, 4, 300, 50_000, rgb, lev, gaze)
    counts = np.bincount(idx.reshape(-1), minlength=N)
    assert _chi2_pvalue(counts, np.full(N, 1.0 / N)) > P_REJECT


def test_aes_keys_are_the_log_of_the_winning_variate(oracle_mod):
    """With w = 1 the stored key of a single slot is log2 of the largest variate seen, which
    the Philox words of the oracle's own layout predict."""
    N = 12
    p = oracle_mod.default_params(64, fovea_radius_px=3.0, bias_mode=oracle_mod.AES, seed=5, stream_id=2)
    rgb = np.zeros((N, 3), np.float32)
    lev = np.zeros(N, np.uint8)
    gaze = np.tile(np.array([[50.0, 10.0]], np.float32), (N, 1))
    px, py = 3, 4
    idx, keys = oracle_mod.trials(64, 32, 1, p, px, py, 5, 1, rgb, lev, gaze)
    pix = py * 64 + px
    ctrs = np.array([[pix, t, 0, 0] for t in range(N)], np.uint32)
    words = oracle_mod.philox(np.tile(np.array([[5, 2]], np.uint32), (N, 1)), ctrs)[:, 0]
    lk = oracle_mod.log2u(words)
    assert idx[0, 0] == int(np.argmax(lk))                 # first of equal maxima: ties keep
    assert keys[0] == lk.max()


def _memoryless_law(w, d):
    N = len(w)
    a = w.astype(np.float64) * d ** (N - 1 - np.arange(N))
    return a / a.sum()


@pytest.mark.parametrize("lam", [0.0231, 0.2])
def test_memoryless_bias_matches_closed_form(oracle_mod, varied_pixel, lam):
    """Multiplying the accumulated w_sum by d = exp(-lambda) every frame selects frame i with
    probability w_i d^(N-1-i) / sum_j w_j d^(N-1-j): the memory-less damping of every past weight."""
    spec, px, py = varied_pixel
    n_frames = 60
    rgb, lev, gaze, w = _pixel_stream(oracle_mod, spec, px, py, n_frames)
    p = oracle_mod.default_params(spec.width, fovea_radius_px=spec.fovea_radius_px,
                                  bias_mode=oracle_mod.BIAS_MEMORYLESS, lambda_decay=lam)
    d = float(oracle_mod.Oracle(spec.width, spec.height, 1, p).decay)
    idx, _ = oracle_mod.trials(spec.width, spec.height, 4, p, px, py, 21, 100_000, rgb, lev, gaze)
    counts = np.bincount(idx.reshape(-1), minlength=n_frames)
    assert _chi2_pvalue(counts, _memoryless_law(w, d)) > P_REJECT


def test_memoryless_with_zero_rate_is_plain_alg2(oracle_mod):
    spec = synth.StreamSpec(64, 48, 4, 10, 8.0, 20.0, 1.0, 4, 3.0)
    src = synth.FrameSource(spec)
    frames = [(c.numpy(), l.numpy(), gx, gy) for (c, l, gx, gy) in src]
    states = []
    for bias, lam in [(oracle_mod.BIAS_NONE, 0.0231), (oracle_mod.BIAS_MEMORYLESS, 0.0)]:
        p = oracle_mod.default_params(spec.width, fovea_radius_px=spec.fovea_radius_px, bias_mode=bias,
                                      lambda_decay=lam)
        o = oracle_mod.Oracle(spec.width, spec.height, spec.k, p)
        for f in frames:
            o.push(*f)
        states.append(o.state())
    for name in ("wsum", "idx", "wt", "col"):
        np.testing.assert_array_equal(getattr(states[0], name), getattr(states[1], name), err_msg=name)


def test_aes_pipeline_invariants(oracle_mod):
    """Whole images: the first frame fills every slot, kept samples are the frame's colour and
    weight at their index, keys are log2(u)/w <= 0 and never decrease."""
    spec = synth.StreamSpec(64, 48, 4, 12, 8.0, 20.0, 1.0, 4, 3.0)
    src = synth.FrameSource(spec)
    frames = [(c.numpy(), l.numpy(), gx, gy) for (c, l, gx, gy) in src]
    p = oracle_mod.default_params(spec.width, fovea_radius_px=spec.fovea_radius_px, bias_mode=oracle_mod.AES)
    o = oracle_mod.Oracle(spec.width, spec.height, spec.k, p)
    prev = None
    for t, f in enumerate(frames):
        o.push(*f)
        st = o.state()
        if t == 0:
            assert np.all(st.idx == 0)
        if prev is not None:
            assert np.all(st.wslot >= prev)
        prev = st.wslot.copy()
    assert np.all(st.wslot <= 0.0)
    for j in range(spec.k):
        for t in range(len(frames)):
            m = st.idx[j] == t
            c, l, gx, gy = frames[t]
            np.testing.assert_array_equal(st.col[j][:, m], c[m].T)
            np.testing.assert_array_equal(st.wt[j][m], o.weight_image(l, gx, gy)[m])
