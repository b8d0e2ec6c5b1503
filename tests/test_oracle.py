"""Pins of the CPU oracle against what the paper and mathematics fix.

Nothing here touches the GPU.  Each test checks the oracle against an
independent fact: a value the paper prints, a closed form, a library
routine, or brute force written separately in numpy.
"""
import json
import math
import os

import numpy as np
import pytest

import ctf_synth as cs
import oracle as O

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_pins.json")))


# ---------------------------------------------------------------------------
# Figure 3: the bijection h and its inverse
# ---------------------------------------------------------------------------

def _mask_from_bits(bits):
    B = np.zeros(4, np.uint64)
    for b in bits:
        B[b >> 6] |= np.uint64(1) << np.uint64(b & 63)
    return B


def test_figure3_worked_example():
    g = GOLD["figure3_bijection"]
    B = _mask_from_bits(g["set_bits"])
    for i, t in g["h"]:
        assert O.bit_select(B, i) == t
    for t, i in g["h_inv"]:
        assert O.bit_rank(B, t) == i


def test_bijection_against_numpy_random_masks():
    rng = np.random.default_rng(3)
    for _ in range(200):
        bits = np.flatnonzero(rng.random(256) < rng.uniform(0.02, 0.6))
        B = _mask_from_bits(bits)
        for i, t in enumerate(bits):
            assert O.bit_select(B, i) == t
            assert O.bit_rank(B, int(t)) == i          # round trip
        assert O.bit_select(B, len(bits)) == -1
        for t in rng.integers(0, 256, 20):
            assert O.bit_rank(B, int(t)) == int((bits < t).sum())


# ---------------------------------------------------------------------------
# procedural texture
# ---------------------------------------------------------------------------

def test_sinusoid_texture_matches_fft_spectrum():
    """The 2-D DFT of one channel has exactly the drawn (p, q, j, a) lines.

    sin(2 pi (p x + q y + j)/W) contributes (W^2 / 2i) e^{2 pi i j / W} at
    frequency (kx, ky) = (p, q) mod W and the conjugate at (-p, -q).
    """
    W, K = 64, 8
    pqj, amp = cs.sinusoid_params(W, K, 8, seed=5)
    tex = O.sinusoid_texture(W, pqj, amp)
    ys, xs = np.mgrid[0:W, 0:W]
    vals = tex.eval(np.stack([xs.ravel(), ys.ravel()], -1)).reshape(W, W, 4)
    for c in range(4):
        F = np.fft.fft2(vals[..., c])          # F[ky, kx] = sum f e^{-2pi i (kx x + ky y)/W}
        expect = np.zeros((W, W), complex)
        expect[0, 0] += 0.5 * W * W
        for (p, q, j), a in zip(pqj[c], amp[c]):
            coef = 0.5 * float(a) * W * W / 2j
            expect[q % W, p % W] += coef * np.exp(2j * np.pi * j / W)
            expect[(-q) % W, (-p) % W] += np.conj(coef * np.exp(2j * np.pi * j / W))
        np.testing.assert_allclose(F, expect, atol=1e-8 * W * W)


def test_sinusoid_texture_periodic_and_in_range():
    W = 2048
    pqj, amp = cs.sinusoid_params(W, 32, 64, seed=2)
    tex = O.sinusoid_texture(W, pqj, amp)
    rng = np.random.default_rng(0)
    xy = rng.integers(-5000, 5000, (2000, 2)).astype(np.int32)
    a = tex.eval(xy)
    for shift in ((W, 0), (0, W), (-W, 3 * W)):
        b = tex.eval(xy + np.array(shift, np.int32))
        assert np.array_equal(a, b)
    assert a.min() >= 0.0 and a.max() <= 1.0


# ---------------------------------------------------------------------------
# footprint and weights: closed forms
# ---------------------------------------------------------------------------

ALL = [O.BILINEAR4, O.LIST, O.BOX, O.MASK]


@pytest.fixture(scope="module")
def c0_scene():
    return cs.tilted_plane_scene()


@pytest.mark.parametrize("kind", ALL)
def test_affine_texture_reproduced_exactly(c0_scene, kind):
    """Bilinear filtering reproduces an affine function of the texel lattice.

    With f = a + b x + c y, the filtered value at the lane's filter position
    (x0 + s, y0 + t) is a + b (x0 + s) + c (y0 + t), for every exactly
    filtered lane.
    """
    sc = c0_scene
    coef = cs.affine_params(1)
    tex = O.affine_texture(64, 64, coef)
    r = O.filter(sc.uv, sc.duv, tex, O.method(kind, box=(4, 4)), seed=0, stf=True)
    # float32 texel position (one rounding, as the method's fma), then the
    # filter position x0 + s with s = fx - x0 taken in float32 as the paper's
    # code does (inexact for -1 < fx < 0)
    def pos(c):
        f = (sc.uv[..., c].astype(np.float64) * 64 - 0.5).astype(np.float32)
        f0 = np.floor(f)
        return f0.astype(np.float64) + (f - f0).astype(np.float64)
    fx, fy = pos(0), pos(1)
    exact = r["stf"][..., 0] == np.iinfo(np.int32).min
    assert exact.sum() > 1000
    for ch in range(4):
        want = coef[ch, 0] + coef[ch, 1] * fx + coef[ch, 2] * fy
        np.testing.assert_allclose(r["out"][..., ch][exact], want[exact], rtol=0, atol=1e-12)


@pytest.mark.parametrize("kind", ALL + [O.STF1])
def test_constant_texture(c0_scene, kind):
    sc = c0_scene
    rgba = (0.25, 0.5, 0.75, 1.0)
    tex = O.constant_texture(64, 64, rgba)
    r = O.filter(sc.uv, sc.duv, tex, O.method(kind, box=(4, 4)), seed=7)
    act = np.isfinite(sc.uv).all(-1)
    assert np.all(r["out"][act] == np.array(rgba))


def test_texel_centres_return_texel_values():
    """uv at texel centres gives s = t = 0: the output is f(x, y) itself."""
    W = 64
    pqj, amp = cs.sinusoid_params(W, 8, 8, seed=0)
    tex = O.sinusoid_texture(W, pqj, amp)
    rng = np.random.default_rng(1)
    xs = rng.integers(0, W, (16, 16))
    ys = rng.integers(0, W, (16, 16))
    uv = np.stack([(xs + 0.5) / W, (ys + 0.5) / W], -1).astype(np.float32)
    duv = np.zeros((16, 16, 4), np.float32)
    want = tex.eval(np.stack([xs.ravel(), ys.ravel()], -1)).reshape(16, 16, 4)
    for kind in ALL + [O.STF1]:
        r = O.filter(uv, duv, tex, O.method(kind), seed=3)
        np.testing.assert_array_equal(r["out"], want)


# ---------------------------------------------------------------------------
# unique sets, masks, boxes
# ---------------------------------------------------------------------------

def _numpy_footprints(uv, W):
    """Independent float32 footprint: floor(u*W - 0.5) with one rounding."""
    f = (uv.astype(np.float64) * W - 0.5).astype(np.float32)
    return np.floor(f).astype(np.int64)


def test_lists_and_masks_against_numpy(c0_scene):
    sc = c0_scene
    W = 64
    pqj, amp = cs.sinusoid_params(W, 8, 8, seed=0)
    tex = O.sinusoid_texture(W, pqj, amp)
    rl = O.filter(sc.uv, sc.duv, tex, O.method(O.LIST), lists=True)
    rm = O.filter(sc.uv, sc.duv, tex, O.method(O.MASK), lists=True)
    rb = O.filter(sc.uv, sc.duv, tex, O.method(O.BOX), lists=True)
    x0y0 = _numpy_footprints(sc.uv, W)
    tiles_x = sc.width // 8
    checked = 0
    for t in range(len(rl["stats"])):
        S = rl["stats"][t]
        ty, tx = divmod(t, tiles_x)
        lanes = [l for l in range(64) if (int(S["part"]) >> l) & 1]
        pts = set()
        for l in lanes:
            x0, y0 = x0y0[ty * 8 + l // 8, tx * 8 + l % 8]
            pts |= {(x0 + dx, y0 + dy) for dx in (0, 1) for dy in (0, 1)}
        U = sorted(pts, key=lambda p: (p[1], p[0]))
        assert S["unique"] == len(U)
        if not lanes:
            continue
        xs = [p[0] for p in U]
        ys = [p[1] for p in U]
        assert (S["xmin"], S["ymin"]) == (min(xs), min(ys))
        assert (S["bbw"], S["bbh"]) == (max(xs) - min(xs) + 1, max(ys) - min(ys) + 1)
        if S["flags"] & O.TILE_OK:
            got = [tuple(e) for e in rl["lists"][t, :S["n"]]]
            assert got == U
            checked += 1
        Sm = rm["stats"][t]
        if S["bbw"] <= 16 and S["bbh"] <= 16:
            # invariant: popcount of the 16x16 mask is the exact unique count
            pc = sum(bin(int(w)).count("1") for w in Sm["mask"])
            assert pc == len(U) == Sm["n"]
            # Mask and List succeed on the same waves
            assert bool(Sm["flags"] & O.TILE_OK) == bool(S["flags"] & O.TILE_OK)
            if Sm["flags"] & O.TILE_OK:
                assert [tuple(e) for e in rm["lists"][t, :Sm["n"]]] == U
        Sb = rb["stats"][t]
        assert Sb["n"] == S["bbw"] * S["bbh"]
        if Sb["flags"] & O.TILE_OK:
            cells = [(S["xmin"] + i % S["bbw"], S["ymin"] + i // S["bbw"]) for i in range(Sb["n"])]
            assert [tuple(e) for e in rb["lists"][t, :Sb["n"]]] == cells
    assert checked > 500


def _quad_tiles(tile, mags, angles, offsets):
    """One head-on rotated-quad tile per (mag, angle, offset), side by side."""
    tw, th = tile
    n = len(mags)
    uv = np.zeros((th, tw * n, 2), np.float32)
    duv = np.zeros((th, tw * n, 4), np.float32)
    for i in range(n):
        u, d = cs.head_on_quad_uv(tw, th, mags[i], angles[i], offsets[i])
        uv[:, i * tw:(i + 1) * tw] = u
        duv[:, i * tw:(i + 1) * tw] = d
    return uv, duv


def _quad_stats(tile, mags, angles, offsets, meth):
    uv, duv = _quad_tiles(tile, mags, angles, offsets)
    tex = O.constant_texture(4096, 4096, (0, 0, 0, 0))
    return O.filter(uv, duv, tex, meth, tile=tile)["stats"]


@pytest.mark.slow
def test_paper_max_unique_54_at_mag1():
    g = GOLD["max_unique_8x4_mag1"]
    rng = np.random.default_rng(11)
    angs = np.concatenate([np.radians(np.arange(0, 90.01, 0.5)),
                           np.radians(rng.uniform(28, 32, 4000)),
                           np.radians(rng.uniform(58, 62, 4000))])
    angs = np.repeat(angs, 40)
    offs = rng.uniform(0, 64, (len(angs), 2)) + 1000
    st = _quad_stats(tuple(g["tile"]), np.full(len(angs), g["magnification"]), angs, offs,
                     O.method(O.LIST))
    u = st["unique"]
    assert u.max() == g["max_unique"]
    best = np.degrees(angs[u == u.max()]) % 90
    assert np.all((np.abs(best - 30) < 5) | (np.abs(best - 60) < 5))


@pytest.mark.slow
def test_paper_exact_set_threshold_159():
    g = GOLD["exact_set_threshold_8x4"]
    rng = np.random.default_rng(12)
    angs = np.repeat(np.radians(np.arange(0, 90.01, 0.25)), 60)
    offs = rng.uniform(0, 64, (len(angs), 2)) + 1000
    for meth in (O.method(O.LIST), O.method(O.MASK)):
        above = _quad_stats(tuple(g["tile"]), np.full(len(angs), 1.595), angs, offs, meth)
        assert np.all(above["flags"] & O.TILE_OK)
        below = _quad_stats(tuple(g["tile"]), np.full(len(angs), 1.575), angs, offs, meth)
        assert np.any((below["flags"] & O.TILE_OK) == 0)


@pytest.mark.slow
def test_paper_box_threshold_235_at_45deg():
    """Box succeeds for every offset iff the rotated tile's span stays below 3 texels.

    At 45 degrees an 8x4 tile spans (7 + 3)/(sqrt 2 m) texels per axis, so
    success is guaranteed from m = 10 / (3 sqrt 2) = 2.357 (the paper's 2.35).
    """
    g = GOLD["box_threshold_8x4_45deg"]
    rng = np.random.default_rng(13)
    n = 20000
    angs = np.full(n, math.radians(g["angle_deg"]))
    offs = rng.uniform(0, 64, (n, 2)) + 1000
    m_star = 10 / (3 * math.sqrt(2))
    assert abs(m_star - g["magnification"]) < 0.01
    ok = _quad_stats(tuple(g["tile"]), np.full(n, m_star * 1.001), angs, offs, O.method(O.BOX))
    assert np.all(ok["flags"] & O.TILE_OK)
    bad = _quad_stats(tuple(g["tile"]), np.full(n, 2.30), angs, offs, O.method(O.BOX))
    assert np.any((bad["flags"] & O.TILE_OK) == 0)


# ---------------------------------------------------------------------------
# stochastic draw
# ---------------------------------------------------------------------------

def _pcg_inverse(y):
    """Independent inverse of the published pcg hash (each step is a bijection)."""
    M32 = 0xFFFFFFFF
    x = y ^ (y >> 22)                       # undo word ^ (word >> 22)
    w = (x * pow(277803737, -1, 2**32)) & M32
    sh = (w >> 28) + 4                      # top 4 bits survive the xorshift
    s = w
    for _ in range(8):
        s = w ^ (s >> sh)
    return ((s - 2891336453) * pow(747796405, -1, 2**32)) & M32


def test_pcg_hash_is_the_published_permutation():
    rng = np.random.default_rng(4)
    for v in list(rng.integers(0, 2**32, 3000)) + [0, 1, 2**31, 2**32 - 1]:
        v = int(v)
        assert _pcg_inverse(O.pcg_hash(v)) == v
    # avalanche: flipping one input bit flips about half the output bits
    flips = []
    for v in rng.integers(0, 2**32, 300):
        h = O.pcg_hash(int(v))
        for b in range(32):
            flips.append(bin(h ^ O.pcg_hash(int(v) ^ (1 << b))).count("1"))
    assert 14.5 < np.mean(flips) < 17.5


def test_stf_draw_frequencies_match_weights():
    """P(texel k) = bilinear weight k (chi-square over many pixels)."""
    from scipy.stats import chisquare
    W = 64
    s, t = 0.3, 0.8
    n = 256
    uv = np.empty((n, n, 2), np.float32)
    uv[..., 0] = (10 + s + 0.5) / W
    uv[..., 1] = (20 + t + 0.5) / W
    duv = np.full((n, n, 4), 1.0, np.float32)     # minifying: every lane draws
    tex = O.constant_texture(W, W, (0, 0, 0, 0))
    r = O.filter(uv, duv, tex, O.method(O.LIST), seed=12345, stf=True)
    pick = r["stf"].reshape(-1, 2)
    assert pick[:, 0].min() >= 10 and pick[:, 0].max() <= 11
    k = (pick[:, 0] - 10) + 2 * (pick[:, 1] - 20)
    counts = np.bincount(k, minlength=4)
    ss = float(np.float32(uv[0, 0, 0] * np.float32(W) - np.float32(0.5))) - 10
    tt = float(np.float32(uv[0, 0, 1] * np.float32(W) - np.float32(0.5))) - 20
    w = np.array([(1 - ss) * (1 - tt), ss * (1 - tt), (1 - ss) * tt, ss * tt])
    w /= w.sum()
    assert chisquare(counts, w * counts.sum()).pvalue > 1e-3
    # s = t = 0: the draw is always the upper-left texel
    uv[..., 0] = (10 + 0.5) / W
    uv[..., 1] = (20 + 0.5) / W
    r = O.filter(uv, duv, tex, O.method(O.LIST), seed=9, stf=True)
    assert np.all(r["stf"].reshape(-1, 2) == np.array([10, 20]))


def test_minify_lanes_draw_and_magnify_lanes_do_not(c0_scene):
    sc = c0_scene
    tex = O.constant_texture(64, 64, (1, 1, 1, 1))
    r = O.filter(sc.uv, sc.duv, tex, O.method(O.LIST), stf=True)
    ratio = cs.texel_ratio(sc.duv, 64, 64)
    drew = r["stf"][..., 0] != np.iinfo(np.int32).min
    ok = np.zeros(sc.uv.shape[:2], bool)
    tiles_x = sc.width // 8
    for t, S in enumerate(r["stats"]):
        if S["flags"] & O.TILE_OK:
            ty, tx = divmod(t, tiles_x)
            ok[ty * 8:(ty + 1) * 8, tx * 8:(tx + 1) * 8] = True
    # in successful tiles, a lane draws iff its footprint spans more than a texel
    # (away from ties at exactly one texel, which float32 rounding decides)
    clear = ok & (np.abs(ratio - 1) > 1e-5)
    assert np.array_equal(drew[clear], ratio[clear] > 1)


# ---------------------------------------------------------------------------
# decoder (float64)
# ---------------------------------------------------------------------------

def test_decoder_identity_network_is_bilinear_latents():
    """A network that passes features through reduces to latent interpolation.

    With H = 16, W1 = W2 = identity on the 16 features, W3 summing feature c
    (level 0) and feature 8 + c (level 1) into output c, zero biases and
    positive latents, the output equals the sum of the two levels' bilinear
    samples with repeat addressing -- scipy's map_coordinates (order 1,
    mode 'grid-wrap') computes those independently.
    """
    from scipy.ndimage import map_coordinates
    tex_w, l0, l1, H, C = 32, 8, 4, 16, 8
    lay = cs.decoder_layout(l0, l1, H, C)
    rng = np.random.default_rng(2)
    p = np.zeros(lay["total"][1])
    o, n = lay["lat0"]; p[o:o + n] = rng.uniform(0.1, 1, n)
    o, n = lay["lat1"]; p[o:o + n] = rng.uniform(0.1, 1, n)
    o, n = lay["W1"]; p[o:o + n] = np.eye(16).ravel()
    o, n = lay["W2"]; p[o:o + n] = np.eye(16).ravel()
    W3 = np.zeros((16, 4))
    for c in range(4):
        W3[c, c] = 1
        W3[8 + c, c] = 1
    o, n = lay["W3"]; p[o:o + n] = W3.ravel()
    tex = O.decoder_texture(tex_w, l0, l1, H, p)
    xy = rng.integers(-40, 80, (300, 2)).astype(np.int32)
    got = tex.eval(xy)
    want = np.zeros_like(got)
    for name, L in (("lat0", l0), ("lat1", l1)):
        o, n = lay[name]
        grid = p[o:o + n].reshape(L, L, C)
        gx = (xy[:, 0] + 0.5) * L / tex_w - 0.5
        gy = (xy[:, 1] + 0.5) * L / tex_w - 0.5
        for c in range(4):
            want[:, c] += map_coordinates(grid[..., c], [gy, gx], order=1, mode="grid-wrap")
    np.testing.assert_allclose(got, want, atol=1e-12)


def test_decoder_gradient_finite_differences_4x4_width4():
    """Analytic float64 gradient vs central differences (4x4 latent grid, 4-wide MLP)."""
    tex_w, l0, l1, H = 16, 4, 2, 4
    p = cs.decoder_init(l0, l1, H, seed=1, latent_range=0.5).astype(np.float64)
    rng = np.random.default_rng(5)
    xy = rng.integers(0, tex_w, (64, 2)).astype(np.int32)
    target = rng.uniform(0, 1, (64, 4)).astype(np.float32)
    loss, g = O.decoder_loss_grad(p, xy, target, l0, l1, H, tex_w)
    eps = 1e-6
    fd = np.empty_like(p)
    for i in range(p.size):
        q = p.copy(); q[i] += eps
        lp, _ = O.decoder_loss_grad(q, xy, target, l0, l1, H, tex_w, grad=False)
        q[i] -= 2 * eps
        lm, _ = O.decoder_loss_grad(q, xy, target, l0, l1, H, tex_w, grad=False)
        fd[i] = (lp - lm) / (2 * eps)
    np.testing.assert_allclose(g, fd, rtol=1e-5, atol=1e-8)
    assert np.abs(g).max() > 1e-3


def test_layer_transform_identity_and_power_of_two_scale(c0_scene):
    """The layer transform is a float32 map: the identity changes nothing,
    and a power-of-two scale equals filtering pre-scaled coordinates."""
    sc = c0_scene
    pqj, amp = cs.sinusoid_params(64, 8, 8, seed=0)
    tex = O.sinusoid_texture(64, pqj, amp)
    m = O.method(O.LIST, k=2)
    base = O.filter(sc.uv, sc.duv, tex, m, seed=4, stf=True)
    ident = O.filter(sc.uv, sc.duv, tex, m, seed=4, stf=True, xform=np.eye(2))
    assert np.array_equal(base["out"], ident["out"]) and np.array_equal(base["stf"], ident["stf"])
    two = O.filter(sc.uv, sc.duv, tex, m, seed=4, stf=True, xform=2 * np.eye(2))
    pre = O.filter(sc.uv * np.float32(2), sc.duv * np.float32(2), tex, m, seed=4, stf=True)
    assert np.array_equal(two["out"], pre["out"]) and np.array_equal(two["stf"], pre["stf"])
    for f in ("part", "mask", "n", "evals"):
        assert np.array_equal(two["stats"][f], pre["stats"][f])


# ---------------------------------------------------------------------------
# fallbacks C and C+ (Section 3.4)
# ---------------------------------------------------------------------------

def test_eq2_lane_mapping_pins():
    g = GOLD["fallback_eq2"]
    for nA, ns, c, want in g["cases"]:
        assert O.cplus_target(nA, ns, c) == want, (nA, ns, c)
    # the paper's formula written with exact rationals, round half up
    from fractions import Fraction
    for nA in (8, 32, 64):
        for ns in range(nA):
            for c in range(ns, nA):
                want = 0 if nA - 1 - ns == 0 else int(Fraction((nA - 1) * (c - ns), nA - 1 - ns) + Fraction(1, 2))
                assert O.cplus_target(nA, ns, c) == want
            if nA - ns >= 2:
                assert O.cplus_target(nA, ns, ns) == 0 and O.cplus_target(nA, ns, nA - 1) == nA - 1


def _lowmag_scene():
    """Exact sets overflow one texel per lane: the fallback runs on most tiles."""
    return cs.lowmag_quads_scene(600, seed=21, tex_w=64)


@pytest.mark.parametrize("fb", [O.FB_C, O.FB_CPLUS])
def test_eq1_special_cases(fb):
    g = GOLD["fallback_eq1"]
    assert g
    uv, duv = _lowmag_scene()
    pqj, amp = cs.sinusoid_params(64, 8, 8, seed=7)
    tex = O.sinusoid_texture(64, pqj, amp)
    fbr = O.filter(uv, duv, tex, O.method(O.MASK, fallback=fb), seed=5, stf=True)
    ex = O.filter(uv, duv, tex, O.method(O.BILINEAR4), seed=5)
    st = O.filter(uv, duv, tex, O.method(O.MASK), seed=5, stf=True)
    failed = (fbr["stats"]["flags"] & O.TILE_OK) == 0
    assert failed.mean() > 0.5
    # constant textures stay constant under Eq. 1
    ct = O.filter(uv, duv, O.constant_texture(64, 64, (0.3, 0.6, 0.9, 1.0)),
                  O.method(O.MASK, fallback=fb), seed=5)
    assert np.allclose(ct["out"], [0.3, 0.6, 0.9, 1.0], atol=1e-15)
    # lanes whose output equals the exact filter or the one-tap value
    close_exact = np.abs(fbr["out"] - ex["out"]).max(-1) < 1e-12
    close_stf = np.abs(fbr["out"] - st["out"]).max(-1) < 1e-12
    drew = fbr["stf"][..., 0] != np.iinfo(np.int32).min
    assert np.all(close_exact | close_stf | drew)
    assert close_exact[drew].mean() > 0.05 and close_stf[drew].mean() > 0.005
    # the draws themselves are the one-tap draws
    assert np.array_equal(fbr["stf"], st["stf"])


def test_fallback_quality_order():
    """C+ is closer to exact filtering than C, and C closer than one-tap STF."""
    assert GOLD["fallback_quality_order"]
    uv, duv = _lowmag_scene()
    pqj, amp = cs.sinusoid_params(64, 8, 8, seed=8)
    tex = O.sinusoid_texture(64, pqj, amp)
    ex = O.filter(uv, duv, tex, O.method(O.BILINEAR4))["out"]
    mse = {}
    for name, fb in (("stf", O.FB_STF1), ("c", O.FB_C), ("cplus", O.FB_CPLUS)):
        errs = []
        for seed in range(4):
            o = O.filter(uv, duv, tex, O.method(O.MASK, fallback=fb), seed=seed)["out"]
            errs.append(((o - ex) ** 2).mean())
        mse[name] = np.mean(errs)
    assert mse["cplus"] < mse["c"] < mse["stf"], mse


# ---------------------------------------------------------------------------
# decoder: where the ReLUs sit (hidden pre-activations of both signs)
# ---------------------------------------------------------------------------

def _signed_network(tex_w=32, l0=8, l1=4, C=8, seed=12):
    """A hand-built decoder whose hidden units split each feature f into its
    positive and negative parts.

    Layer 1 (2C -> H = 4C): unit i = f_i, unit 2C + i = -f_i (W1 = [I, -I],
    no bias), so its ReLU yields (max(f, 0), max(-f, 0)).  Layer 2: unit
    j = a_j - a_{2C+j} + beta_p, unit 2C + j = -(a_j - a_{2C+j}) + beta_n,
    i.e. f_j + beta_p and -f_j + beta_n before its ReLU.  Output c:
    1 x unit c + 2 x unit 2C + c + 3 x unit C + c + 4 x unit 3C + c of the
    second layer's activations, plus b3_c.  Latents are drawn from U(-1, 1),
    so every pre-activation takes both signs.
    """
    H = 4 * C
    lay = cs.decoder_layout(l0, l1, H, C)
    rng = np.random.default_rng(seed)
    p = np.zeros(lay["total"][1])
    o, n = lay["lat0"]; p[o:o + n] = rng.uniform(-1, 1, n)
    o, n = lay["lat1"]; p[o:o + n] = rng.uniform(-1, 1, n)
    F = 2 * C
    W1 = np.zeros((F, H))
    W1[np.arange(F), np.arange(F)] = 1
    W1[np.arange(F), F + np.arange(F)] = -1
    W2 = np.zeros((H, H))
    for j in range(F):
        W2[j, j], W2[F + j, j] = 1, -1
        W2[j, F + j], W2[F + j, F + j] = -1, 1
    beta_p, beta_n = 0.125, -0.25
    b2 = np.concatenate([np.full(F, beta_p), np.full(F, beta_n)])
    W3 = np.zeros((H, 4))
    for c in range(4):
        W3[c, c], W3[F + c, c] = 1, 2              # level 0, channel c
        W3[C + c, c], W3[F + C + c, c] = 3, 4      # level 1, channel c
    b3 = np.array([-1.0, -0.5, 0.25, -2.0])
    for name, v in (("W1", W1), ("W2", W2), ("b2", b2), ("W3", W3), ("b3", b3)):
        o, n = lay[name]
        p[o:o + n] = v.ravel()
    return dict(p=p, lay=lay, tex_w=tex_w, l0=l0, l1=l1, H=H, C=C,
                beta_p=beta_p, beta_n=beta_n, b3=b3)


def _bilinear_corners(xy, L, tex_w):
    """Corner cells and weights of the repeat-addressed bilinear sample at
    g = (x + 1/2) L / W - 1/2, per sample: ([n][4] flat cell index, [n][4] weight)."""
    g = (xy.astype(np.float64) + 0.5) * L / tex_w - 0.5
    c = np.floor(g)
    f = g - c
    cx, cy = c[:, 0].astype(np.int64), c[:, 1].astype(np.int64)
    fx, fy = f[:, 0], f[:, 1]
    idx = np.stack([(cy % L) * L + cx % L, (cy % L) * L + (cx + 1) % L,
                    ((cy + 1) % L) * L + cx % L, ((cy + 1) % L) * L + (cx + 1) % L], 1)
    w = np.stack([(1 - fx) * (1 - fy), fx * (1 - fy), (1 - fx) * fy, fx * fy], 1)
    return idx, w


def _signed_features(net, xy):
    """Level-0 and level-1 features by scipy's map_coordinates (order 1, grid-wrap)."""
    from scipy.ndimage import map_coordinates
    lay, C = net["lay"], net["C"]
    feats = []
    for name, L in (("lat0", net["l0"]), ("lat1", net["l1"])):
        o, n = lay[name]
        grid = net["p"][o:o + n].reshape(L, L, C)
        gx = (xy[:, 0] + 0.5) * L / net["tex_w"] - 0.5
        gy = (xy[:, 1] + 0.5) * L / net["tex_w"] - 0.5
        feats.append(np.stack([map_coordinates(grid[..., c], [gy, gx], order=1, mode="grid-wrap")
                               for c in range(C)], 1))
    return feats


def test_decoder_relu_placement_closed_form():
    """Forward pass of the signed network against its closed form:
    out_c = max(f0+bp, 0) + 2 max(-f0+bn, 0) + 3 max(f1+bp, 0) + 4 max(-f1+bn, 0) + b3_c
    with f0, f1 the level-0 and level-1 features of channel c.  A missing,
    extra (output) or moved ReLU changes the result."""
    net = _signed_network()
    tex = O.decoder_texture(net["tex_w"], net["l0"], net["l1"], net["H"], net["p"])
    rng = np.random.default_rng(4)
    xy = rng.integers(-50, 90, (400, 2)).astype(np.int32)
    got = tex.eval(xy)
    f0, f1 = _signed_features(net, xy)
    bp, bn = net["beta_p"], net["beta_n"]
    relu = lambda v: np.maximum(v, 0.0)
    want = np.stack([relu(f0[:, c] + bp) + 2 * relu(-f0[:, c] + bn)
                     + 3 * relu(f1[:, c] + bp) + 4 * relu(-f1[:, c] + bn) + net["b3"][c]
                     for c in range(4)], 1)
    # both signs and both inactive bands are exercised, and outputs go negative
    for f in (f0[:, :4], f1[:, :4]):
        assert (f > -bp).mean() > 0.2 and (f < bn).mean() > 0.2
        assert ((f < -bp) & (f > bn)).any()
    assert (want < 0).mean() > 0.1
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)


def test_decoder_relu_gradients_closed_form():
    """Backward pass of the signed network against its closed form.

    With e = y - target and dy = 2 e / (4 n): dL/db3 = sum dy; dL/dW3 rows
    are the second layer's activations times dy; dL/db2_j = sum dy_c times
    the coefficient of unit j (1, 2, 3, 4) where that unit is active; the
    latent gradient of channel c < 4 is dy_c times phi'(f) times the
    corner weight, phi'(f) = [f > -bp] - 2 [f < bn] (level 0) and
    3 [f > -bp] - 4 [f < bn] (level 1); channels 4..7 feed no output and get
    no gradient."""
    net = _signed_network()
    lay, C, H = net["lay"], net["C"], net["H"]
    rng = np.random.default_rng(6)
    n = 300
    xy = rng.integers(0, net["tex_w"], (n, 2)).astype(np.int32)
    target = rng.uniform(-1, 1, (n, 4)).astype(np.float32)
    loss, g = O.decoder_loss_grad(net["p"], xy, target, net["l0"], net["l1"], H, net["tex_w"])
    f0, f1 = _signed_features(net, xy)
    bp, bn = net["beta_p"], net["beta_n"]
    relu = lambda v: np.maximum(v, 0.0)
    F = 2 * C
    f = np.concatenate([f0, f1], 1)                       # [n][2C]
    a2 = np.concatenate([relu(f + bp), relu(-f + bn)], 1)  # [n][H]
    y = np.stack([a2[:, c] + 2 * a2[:, F + c] + 3 * a2[:, C + c] + 4 * a2[:, F + C + c]
                  + net["b3"][c] for c in range(4)], 1)
    e = y - target.astype(np.float64)
    assert loss == pytest.approx((e ** 2).mean(), rel=1e-12)
    dy = 2 * e / (4 * n)

    o, m = lay["b3"]
    np.testing.assert_allclose(g[o:o + m], dy.sum(0), atol=1e-12)
    o, m = lay["W3"]
    np.testing.assert_allclose(g[o:o + m].reshape(H, 4), a2.T @ dy, atol=1e-12)
    coef = np.zeros((H, 4))
    for c in range(4):
        coef[c, c], coef[F + c, c], coef[C + c, c], coef[F + C + c, c] = 1, 2, 3, 4
    active2 = np.concatenate([f + bp > 0, -f + bn > 0], 1)
    o, m = lay["b2"]
    np.testing.assert_allclose(g[o:o + m], (active2 * (dy @ coef.T)).sum(0), atol=1e-12)
    for lev, (name, L, fl, kp, kn) in enumerate((("lat0", net["l0"], f0, 1, 2),
                                                 ("lat1", net["l1"], f1, 3, 4))):
        idx, w = _bilinear_corners(xy, L, net["tex_w"])
        dphi = kp * (fl[:, :4] > -bp) - kn * (fl[:, :4] < bn)     # [n][4 channels]
        want = np.zeros((L * L, C))
        for q in range(4):
            np.add.at(want[:, :4], idx[:, q], (w[:, q:q + 1] * dy * dphi))
        o, m = lay[name]
        np.testing.assert_allclose(g[o:o + m].reshape(L * L, C), want, atol=1e-12)
        assert np.abs(want).max() > 1e-3


# ---------------------------------------------------------------------------
# fallback C+ (Section 3.4, Eq. 2): what each spare lane produces
# ---------------------------------------------------------------------------

def _f32_footprints(uv, W):
    """Bilinear footprint per pixel in float32 (W a power of two, so the
    fused multiply-add of the footprint equals the rounded product and sum):
    (x0, y0, s, t)."""
    uv = uv.astype(np.float32)
    fx = uv[..., 0] * np.float32(W) - np.float32(0.5)
    fy = uv[..., 1] * np.float32(W) - np.float32(0.5)
    x0, y0 = np.floor(fx), np.floor(fy)
    return x0.astype(np.int64), y0.astype(np.int64), (fx - x0).astype(np.float32), (fy - y0).astype(np.float32)


def _cplus_waves(seed):
    uv, duv = _lowmag_scene()
    W = 64
    pqj, amp = cs.sinusoid_params(W, 8, 8, seed=7)
    tex = O.sinusoid_texture(W, pqj, amp)
    r = O.filter(uv, duv, tex, O.method(O.MASK, fallback=O.FB_CPLUS), seed=seed, stf=True,
                 fb_items=True)
    return uv, W, r


@pytest.mark.parametrize("seed", [5, 6])
def test_cplus_spare_lanes_follow_eq2(seed):
    """Per failed wave, independently of the oracle's own steps:
    the first |S| produced texels are the distinct one-tap draws of A in
    mask (row-major) order, made by the lanes of rank 0..|S|-1; every other
    produced texel is made by a spare lane of rank c >= |S| and lies in the
    footprint of the lane of rank round((nA-1)(c-|S|)/(nA-1-|S|)) (Eq. 2,
    exact rationals, ties up), with a nonzero float32 weight there, outside
    S; a spare lane produces nothing only when that footprint has no such
    texel; the tile's evaluation count is |S| + the spare texels + the draws
    of the minifying lanes."""
    from fractions import Fraction
    uv, W, r = _cplus_waves(seed)
    x0, y0, s, t = _f32_footprints(uv, W)
    n_tiles = uv.shape[1] // 8
    checked = spare_total = idle_total = 0
    for tile in range(n_tiles):
        S_rec = r["stats"][tile]
        if S_rec["flags"] & O.TILE_OK or S_rec["part"] == 0:
            continue
        assert S_rec["bbw"] <= 16 and S_rec["bbh"] <= 16
        A = int(S_rec["part"])
        lanes = [l for l in range(64) if (A >> l) & 1]
        nA = len(lanes)
        sl = np.s_[:, 8 * tile:8 * tile + 8]
        tx0, ty0, ts, tt = (a[sl].reshape(64) for a in (x0, y0, s, t))
        picks = r["stf"][sl].reshape(64, 2)
        S = sorted({(int(picks[l, 1]), int(picks[l, 0])) for l in lanes})   # (y, x) order
        ns = len(S)
        items = r["fb_items"][tile]
        items = items[items[:, 2] != np.iinfo(np.int32).min]
        assert [(int(i[1]), int(i[0])) for i in items[:ns]] == S
        assert list(items[:ns, 2]) == list(range(ns))
        spare = items[ns:]
        ranks = list(spare[:, 2])
        assert ranks == sorted(set(ranks)) and all(ns <= c < nA for c in ranks)
        Sset = set(S)
        for c in range(ns, nA):
            span = nA - 1 - ns
            tr = 0 if span == 0 else int(Fraction((nA - 1) * (c - ns), span) + Fraction(1, 2))
            L = lanes[tr]
            wx = (np.float32(1) - ts[L], ts[L])
            wy = (np.float32(1) - tt[L], tt[L])
            cand = {(int(ty0[L] + j), int(tx0[L] + i)) for j in range(2) for i in range(2)
                    if np.float32(wx[i] * wy[j]) != 0 and (int(ty0[L] + j), int(tx0[L] + i)) not in Sset}
            row = spare[spare[:, 2] == c]
            if row.size:
                assert (int(row[0, 1]), int(row[0, 0])) in cand, (tile, c)
                spare_total += 1
            else:
                assert not cand, (tile, c)
                idle_total += 1
        minify_draws = bin(int(S_rec["active"]) & ~A).count("1")
        assert S_rec["evals"] == ns + len(spare) + minify_draws
        checked += 1
    assert checked > 300 and spare_total > 3000 and idle_total > 0


def test_cplus_spare_draws_follow_abs_weights():
    """A spare lane draws among its candidates with probability |w| / sum |w|:
    the randomised probability-integral transform of every draw (a uniform
    point inside the drawn candidate's interval of the cumulative |w|
    distribution, candidates in row-major order) is uniform on [0, 1)."""
    from fractions import Fraction
    from scipy.stats import chisquare
    pit = []
    rng = np.random.default_rng(11)
    for seed in range(4):
        uv, W, r = _cplus_waves(seed)
        x0, y0, s, t = _f32_footprints(uv, W)
        for tile in range(uv.shape[1] // 8):
            S_rec = r["stats"][tile]
            if S_rec["flags"] & O.TILE_OK or S_rec["part"] == 0:
                continue
            A = int(S_rec["part"])
            lanes = [l for l in range(64) if (A >> l) & 1]
            nA = len(lanes)
            sl = np.s_[:, 8 * tile:8 * tile + 8]
            tx0, ty0, ts, tt = (a[sl].reshape(64) for a in (x0, y0, s, t))
            picks = r["stf"][sl].reshape(64, 2)
            Sset = {(int(picks[l, 1]), int(picks[l, 0])) for l in lanes}
            ns = len(Sset)
            items = r["fb_items"][tile]
            for x, y, c in items[items[:, 2] != np.iinfo(np.int32).min][ns:]:
                span = nA - 1 - ns
                tr = 0 if span == 0 else int(Fraction((nA - 1) * (int(c) - ns), span) + Fraction(1, 2))
                L = lanes[tr]
                wx = (1.0 - float(ts[L]), float(ts[L]))
                wy = (1.0 - float(tt[L]), float(tt[L]))
                cw = [(int(ty0[L] + j), int(tx0[L] + i), abs(wx[i] * wy[j]))
                      for j in range(2) for i in range(2)]
                cw = [e for e in cw if e[2] > 0 and (e[0], e[1]) not in Sset]
                tot = sum(e[2] for e in cw)
                lo = 0.0
                for yy, xx, w in cw:
                    if (yy, xx) == (int(y), int(x)):
                        pit.append((lo + rng.uniform() * w) / tot)
                        break
                    lo += w
                else:
                    raise AssertionError("spare texel not among the candidates")
    pit = np.array(pit)
    assert pit.size > 10000
    counts = np.histogram(pit, bins=20, range=(0, 1))[0]
    assert chisquare(counts).pvalue > 1e-4, counts


def test_filter_parallel_equals_one_call():
    """The threaded whole-frame helper the full-frame GPU tests use gives
    the single call's outputs bit for bit (8x8 and 8x4 tiles, a fallback)."""
    sc = cs.random_planes_scene(203, 77, 64, 64, seed=4)
    pqj, amp = cs.sinusoid_params(64, 8, 8, seed=1)
    tex = O.sinusoid_texture(64, pqj, amp)
    for m, t in ((O.method(O.LIST, k=2), (8, 8)), (O.method(O.MASK, fallback=O.FB_CPLUS), (8, 4)),
                 (O.method(O.BILINEAR4, filter=O.FILTER_CATMULL_ROM), (8, 8))):
        a = O.filter(sc.uv, sc.duv, tex, m, seed=3, stf=True, tile=t)
        b = O.filter_parallel(sc.uv, sc.duv, tex, m, seed=3, tile=t, threads=5)
        for k in ("out", "stats", "stf"):
            assert np.array_equal(a[k], b[k]), k
