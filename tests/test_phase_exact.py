"""The float form of the sinusoid phase is exact.

A sinusoid term's phase is (p x + q y + j) mod W in revolutions of W.  The
kernels evaluate it as fract(p'/W x + (q'/W y + j'/W)) in float32, with p', q'
the residues of p, q mod W in [-W/2, W/2) and j' = j mod W (the texture is
built with W <= 4096).  Every product and sum there is exactly representable
(|p' x + q' y + j'| < W^2 <= 2^24), so the float form equals the integer
form's (v mod W) / W exactly, and both feed the same value to the sine.  This
checks that claim with float32 operations that round after every step: any
inexact step would show as a mismatch.
"""
import numpy as np
import pytest


def centred(v, W):
    r = np.mod(v, W)
    return np.where(r >= W // 2, r - W, r)


@pytest.mark.parametrize("W", [64, 256, 2048, 4096])
def test_float_phase_equals_integer_phase(W):
    rng = np.random.default_rng(W)
    n = 200_000
    p = rng.integers(-(1 << 23) + 1, 1 << 23, n)
    q = rng.integers(-(1 << 23) + 1, 1 << 23, n)
    j = rng.integers(0, 1 << 31, n)
    x = rng.integers(0, W, n)
    y = rng.integers(0, W, n)
    # the extremes of the bound: largest |p'|, |q'|, x, y and j'
    p[:4] = [W // 2, -W // 2, W // 2 - 1, -W // 2]
    q[:4] = [W // 2, -W // 2, -W // 2, W // 2 - 1]
    j[:4] = [W - 1, 0, W - 1, 3 * W - 1]
    x[:4] = W - 1
    y[:4] = W - 1
    f32 = np.float32
    pw = (centred(p, W) / W).astype(f32)
    qw = (centred(q, W) / W).astype(f32)
    jw = (np.mod(j, W) / W).astype(f32)
    inner = qw * y.astype(f32) + jw
    ph = pw * x.astype(f32) + inner
    frac = ph - np.floor(ph)
    want = np.mod(p * x + q * y + j, W) / W   # exact in float64
    assert np.array_equal(frac.astype(np.float64), want)
    # each step was exact, so a fused multiply-add gives the same value
    assert np.array_equal((qw.astype(np.float64) * y + jw), inner.astype(np.float64))
    assert np.array_equal(pw.astype(np.float64) * x + inner, ph.astype(np.float64))


def test_bound_fails_past_4096():
    """The kernels keep the integer form above W = 4096: there the float
    products can round (the bound W^2 <= 2^24 no longer holds)."""
    W = 8192
    p, q, j, x, y = W // 2 - 1, W // 2 - 1, W - 1, W - 1, W - 1
    v = p * x + q * y + j
    assert v >= 1 << 24
