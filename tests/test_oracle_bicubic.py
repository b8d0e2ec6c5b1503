"""Pins of the oracle's bicubic filters (Section 5: uniform cubic B-spline and
Catmull-Rom, 4x4 footprints) against facts the mathematics fixes.

* B-spline colours equal scipy's cubic spline evaluation of the same texel
  lattice used as spline coefficients (``map_coordinates`` order 3, no
  prefilter, periodic), an independent library routine.
* Catmull-Rom reproduces every polynomial of degree <= 2 per axis and
  interpolates (texel centres return the texel itself).
* Both weight sets sum to one (constants survive every method and fallback).
* One-tap draws pick tap (i, j) with probability |wx_i| |wy_j| / sums, and
  never a zero-weight tap.
* Unique sets, boxes and 16x16 masks of 4x4 footprints equal a brute-force
  numpy construction.
"""
import numpy as np
import pytest

import ctf_synth as cs
import oracle as O

INT_MIN = np.iinfo(np.int32).min
CUBICS = [O.FILTER_BSPLINE, O.FILTER_CATMULL_ROM]


def _grid_uv(W, n, rng, lo=0.0, hi=None, step=2.0**-10):
    """uv whose texel positions fx = u W - 1/2 are exact binary fractions."""
    hi = W if hi is None else hi
    fx = np.round(rng.uniform(lo, hi, (n, n)) / step) * step
    fy = np.round(rng.uniform(lo, hi, (n, n)) / step) * step
    uv = np.stack([(fx + 0.5) / W, (fy + 0.5) / W], -1).astype(np.float32)
    assert np.array_equal(uv[..., 0].astype(np.float64) * W - 0.5, fx)
    return uv, fx, fy


def test_bspline_equals_scipy_cubic_spline_evaluation():
    from scipy.ndimage import map_coordinates
    W = 32
    rng = np.random.default_rng(0)
    table = rng.uniform(0, 1, (W, W, 4)).astype(np.float32)
    uv, fx, fy = _grid_uv(W, 24, rng)
    duv = np.zeros(uv.shape[:2] + (4,), np.float32)
    r = O.filter(uv, duv, O.table_texture(table), O.method(O.BILINEAR4, filter=O.FILTER_BSPLINE))
    for c in range(4):
        want = map_coordinates(table[..., c].astype(np.float64), [fy.ravel(), fx.ravel()], order=3,
                               mode="grid-wrap", prefilter=False).reshape(fx.shape)
        np.testing.assert_allclose(r["out"][..., c], want, rtol=0, atol=1e-13)
    # and the bilinear filter is scipy's order-1 evaluation
    rb = O.filter(uv, duv, O.table_texture(table), O.method(O.BILINEAR4))
    want = map_coordinates(table[..., 0].astype(np.float64), [fy.ravel(), fx.ravel()], order=1,
                           mode="grid-wrap").reshape(fx.shape)
    np.testing.assert_allclose(rb["out"][..., 0], want, rtol=0, atol=1e-13)


def test_catmull_rom_reproduces_quadratics():
    """f = sum of monomials x^a y^b with a, b <= 2 is reproduced exactly
    (positions kept two texels away from the repeat seam)."""
    W = 64
    rng = np.random.default_rng(1)
    ys, xs = np.mgrid[0:W, 0:W].astype(np.float64)
    coef = rng.uniform(-1, 1, (4, 3, 3))
    table = np.zeros((W, W, 4))
    for c in range(4):
        for a in range(3):
            for b in range(3):
                table[..., c] += coef[c, a, b] * (xs / W) ** a * (ys / W) ** b
    uv, fx, fy = _grid_uv(W, 24, rng, lo=3.0, hi=W - 4.0)
    duv = np.zeros(uv.shape[:2] + (4,), np.float32)
    tab32 = table.astype(np.float32)
    r = O.filter(uv, duv, O.table_texture(tab32), O.method(O.BILINEAR4, filter=O.FILTER_CATMULL_ROM))
    # the same polynomial through the float32-rounded table: compare with the
    # exact polynomial at (fx, fy) within the table's rounding (sum |w| < 1.6)
    for c in range(4):
        want = sum(coef[c, a, b] * (fx / W) ** a * (fy / W) ** b for a in range(3) for b in range(3))
        assert np.abs(r["out"][..., c] - want).max() < 1.6 * 1.6 * 4 * 2.0**-24 * 4
    # the B-spline only reproduces degree <= 1 (a quadratic is smoothed)
    rb = O.filter(uv, duv, O.table_texture(tab32), O.method(O.BILINEAR4, filter=O.FILTER_BSPLINE))
    want = sum(coef[0, a, b] * (fx / W) ** a * (fy / W) ** b for a in range(3) for b in range(3))
    assert np.abs(rb["out"][..., 0] - want).max() > 1e-5


@pytest.mark.parametrize("flt", CUBICS)
def test_affine_reproduced_by_both_cubics(flt):
    W = 64
    rng = np.random.default_rng(2)
    coef = cs.affine_params(3)
    uv, fx, fy = _grid_uv(W, 24, rng, lo=-200.0, hi=200.0)
    duv = np.zeros(uv.shape[:2] + (4,), np.float32)
    r = O.filter(uv, duv, O.affine_texture(W, W, coef), O.method(O.BILINEAR4, filter=flt))
    for c in range(4):
        want = coef[c, 0] + coef[c, 1] * fx + coef[c, 2] * fy
        np.testing.assert_allclose(r["out"][..., c], want, rtol=0, atol=1e-9)


def test_texel_centres_catmull_rom_interpolates_bspline_smooths():
    W = 64
    pqj, amp = cs.sinusoid_params(W, 8, 8, seed=0)
    tex = O.sinusoid_texture(W, pqj, amp)
    rng = np.random.default_rng(3)
    xs = rng.integers(0, W, (16, 16))
    ys = rng.integers(0, W, (16, 16))
    uv = np.stack([(xs + 0.5) / W, (ys + 0.5) / W], -1).astype(np.float32)
    duv = np.zeros((16, 16, 4), np.float32)
    ev = lambda dx, dy: tex.eval(np.stack([(xs + dx).ravel(), (ys + dy).ravel()], -1)).reshape(16, 16, 4)
    r = O.filter(uv, duv, tex, O.method(O.BILINEAR4, filter=O.FILTER_CATMULL_ROM))
    np.testing.assert_allclose(r["out"], ev(0, 0), rtol=0, atol=1e-15)
    # B-spline at a lattice point: the separable [1 4 1] / 6 stencil
    r = O.filter(uv, duv, tex, O.method(O.BILINEAR4, filter=O.FILTER_BSPLINE))
    k = {-1: 1 / 6, 0: 4 / 6, 1: 1 / 6}
    want = sum(k[dx] * k[dy] * ev(dx, dy) for dx in (-1, 0, 1) for dy in (-1, 0, 1))
    np.testing.assert_allclose(r["out"], want, rtol=0, atol=1e-14)


@pytest.mark.parametrize("flt", CUBICS)
@pytest.mark.parametrize("kind", [O.BILINEAR4, O.STF1, O.LIST, O.BOX, O.MASK])
def test_constant_texture_every_method_and_fallback(flt, kind):
    uv, duv = cs.lowmag_quads_scene(60, seed=5, tex_w=64, mag=(1.0, 4.0))
    tex = O.constant_texture(64, 64, (0.3, 0.6, 0.9, 1.0))
    for fb in (O.FB_STF1, O.FB_C, O.FB_CPLUS):
        r = O.filter(uv, duv, tex, O.method(kind, k=2, fallback=fb, filter=flt), seed=3)
        np.testing.assert_allclose(r["out"], np.broadcast_to([0.3, 0.6, 0.9, 1.0], r["out"].shape),
                                   rtol=0, atol=2e-15)


def _taps(flt, x):
    x = np.float64(x)
    if flt == O.FILTER_BSPLINE:
        return np.array([(1 - x) ** 3, 3 * x**3 - 6 * x**2 + 4, -3 * x**3 + 3 * x**2 + 3 * x + 1, x**3]) / 6
    return np.array([-x**3 + 2 * x**2 - x, 3 * x**3 - 5 * x**2 + 2, -3 * x**3 + 4 * x**2 + x, x**3 - x**2]) / 2


@pytest.mark.parametrize("flt", CUBICS)
def test_cubic_stf_draws_follow_absolute_weights(flt):
    from scipy.stats import chisquare
    W = 64
    s, t = 0.3, 0.8
    n = 320
    uv = np.empty((n, n, 2), np.float32)
    uv[..., 0] = (10 + s + 0.5) / W
    uv[..., 1] = (20 + t + 0.5) / W
    duv = np.full((n, n, 4), 1.0, np.float32)     # minifying: every lane draws
    tex = O.constant_texture(W, W, (0, 0, 0, 0))
    r = O.filter(uv, duv, tex, O.method(O.LIST, filter=flt), seed=777, stf=True)
    pick = r["stf"].reshape(-1, 2)
    i, j = pick[:, 0] - 9, pick[:, 1] - 19
    assert i.min() >= 0 and i.max() <= 3 and j.min() >= 0 and j.max() <= 3
    ss = float(np.float32(uv[0, 0, 0] * np.float32(W) - np.float32(0.5))) - 10
    tt = float(np.float32(uv[0, 0, 1] * np.float32(W) - np.float32(0.5))) - 20
    p = np.outer(np.abs(_taps(flt, tt)), np.abs(_taps(flt, ss))).ravel()
    p /= p.sum()
    counts = np.bincount(4 * j + i, minlength=16)
    assert chisquare(counts, p * counts.sum()).pvalue > 1e-3
    # at s = t = 0 the zero-weight taps are never drawn
    uv[..., 0] = (10 + 0.5) / W
    uv[..., 1] = (20 + 0.5) / W
    r = O.filter(uv, duv, tex, O.method(O.LIST, filter=flt), seed=9, stf=True)
    pick = r["stf"].reshape(-1, 2)
    if flt == O.FILTER_CATMULL_ROM:          # weights (0, 1, 0, 0) per axis
        assert np.all(pick == np.array([10, 20]))
    else:                                      # weights (1, 4, 1, 0) / 6 per axis
        assert pick[:, 0].max() <= 11 and pick[:, 1].max() <= 21
        assert pick[:, 0].min() == 9 and pick[:, 1].min() == 19


@pytest.mark.parametrize("flt", CUBICS)
def test_cubic_lists_masks_boxes_against_numpy(flt):
    uv, duv = cs.lowmag_quads_scene(300, seed=8, tex_w=64, mag=(0.8, 6.0))
    # a few minifying lanes so that A is not always full
    duv[::3, ::7] = 2.0 / 64
    W = 64
    tex = O.constant_texture(W, W, (0, 0, 0, 0))
    rl = O.filter(uv, duv, tex, O.method(O.LIST, k=4, filter=flt), lists=True)
    rm = O.filter(uv, duv, tex, O.method(O.MASK, k=4, filter=flt), lists=True)
    rb = O.filter(uv, duv, tex, O.method(O.BOX, k=4, filter=flt), lists=True)
    f = (uv.astype(np.float64) * W - 0.5).astype(np.float32)
    x0y0 = np.floor(f).astype(np.int64)
    ok = 0
    for t in range(len(rl["stats"])):
        S = rl["stats"][t]
        lanes = [l for l in range(64) if (int(S["part"]) >> l) & 1]
        pts = set()
        for l in lanes:
            x0, y0 = x0y0[l // 8, 8 * t + l % 8]
            pts |= {(x0 + dx, y0 + dy) for dx in (-1, 0, 1, 2) for dy in (-1, 0, 1, 2)}
        U = sorted(pts, key=lambda p: (p[1], p[0]))
        assert S["unique"] == len(U)
        if not lanes:
            continue
        xs, ys = [p[0] for p in U], [p[1] for p in U]
        assert (S["xmin"], S["ymin"], S["bbw"], S["bbh"]) == (
            min(xs), min(ys), max(xs) - min(xs) + 1, max(ys) - min(ys) + 1)
        assert bool(S["flags"] & O.TILE_OK) == (len(U) <= 4 * len(lanes))
        if S["flags"] & O.TILE_OK:
            assert [tuple(e) for e in rl["lists"][t, :S["n"]]] == U
            ok += 1
        Sm = rm["stats"][t]
        if S["bbw"] <= 16 and S["bbh"] <= 16:
            bits = np.zeros(256, bool)
            for (x, y) in U:
                bits[16 * (y - S["ymin"]) + (x - S["xmin"])] = True
            words = [int(sum(1 << b for b in range(64) if bits[64 * w + b])) for w in range(4)]
            assert [int(w) for w in Sm["mask"]] == words
            if Sm["flags"] & O.TILE_OK:
                assert [tuple(e) for e in rm["lists"][t, :Sm["n"]]] == U
        else:
            assert not (Sm["flags"] & O.TILE_OK)
        Sb = rb["stats"][t]
        assert Sb["n"] == S["bbw"] * S["bbh"]
    assert ok > 50


@pytest.mark.parametrize("flt", CUBICS)
def test_cubic_fallback_eq1_cases(flt):
    """Eq. 1 with 16-tap footprints on failing waves: C+ is closer to exact
    filtering than C, and C closer than the one-tap draw."""
    uv, duv = cs.lowmag_quads_scene(200, seed=9, tex_w=64, mag=(1.0, 1.8))
    pqj, amp = cs.sinusoid_params(64, 8, 8, seed=4)
    tex = O.sinusoid_texture(64, pqj, amp)
    ex = O.filter(uv, duv, tex, O.method(O.BILINEAR4, filter=flt))["out"]
    mse = {}
    for name, fb in (("stf", O.FB_STF1), ("c", O.FB_C), ("cplus", O.FB_CPLUS)):
        r = O.filter(uv, duv, tex, O.method(O.MASK, fallback=fb, filter=flt), seed=2, stf=True)
        failed = (r["stats"]["flags"] & O.TILE_OK) == 0
        assert failed.mean() > 0.5
        mse[name] = ((r["out"] - ex) ** 2).mean()
    assert mse["cplus"] < mse["c"] < mse["stf"], mse
