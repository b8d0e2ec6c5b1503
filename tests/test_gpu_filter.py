"""GPU filter parity: HIP kernels (through the C ABI) vs the CPU oracle.

Bar: per-tile decisions (masks, boxes, counts, flags), item lists and STF
draws bit-exact; colours within 1e-6 absolute of the float64 oracle.
"""
import math

import numpy as np
import pytest

import ctf_synth as cs
import oracle as O

pytestmark = pytest.mark.gpu

TOL = 1e-6
INT_MIN = np.iinfo(np.int32).min
METHODS = [  # (name, gpu kind, oracle kind, box budget, k)
    ("bilinear4", 0, O.BILINEAR4, (0, 0), 1),
    ("stf1", 1, O.STF1, (0, 0), 1),
    ("list", 2, O.LIST, (0, 0), 1),
    ("box4x4", 3, O.BOX, (4, 4), 1),
    ("box6x6", 3, O.BOX, (6, 6), 1),
    ("box", 3, O.BOX, (0, 0), 1),
    ("mask", 4, O.MASK, (0, 0), 1),
    ("list_k2", 2, O.LIST, (0, 0), 2),
    ("mask_k4", 4, O.MASK, (0, 0), 4),
    ("box_k3", 3, O.BOX, (0, 0), 3),
]
STAT_FIELDS = ["active", "part", "stf", "mask", "xmin", "ymin", "bbw", "bbh", "n", "unique",
               "evals", "flags"]


@pytest.fixture(scope="module")
def G():
    import torch
    import paper_2506_17770_amd as ctf
    ctx = ctf.Context(0)
    yield ctf, ctx, torch
    ctx.close()


def run_gpu(G, uv, duv, tex, meth, seed=0):
    ctf, ctx, torch = G
    sh, sw = uv.shape[:2]
    uv_t = torch.from_numpy(np.ascontiguousarray(uv)).cuda()
    duv_t = torch.from_numpy(np.ascontiguousarray(duv)).cuda()
    ts = ctf.tile_stats_buffer(sw, sh)
    fs = ctf.frame_stats_buffer()
    li = ctf.lists_buffer(sw, sh)
    sx = ctf.stf_buffer(sw, sh)
    out = ctx.filter(uv_t, duv_t, tex, meth, seed=seed, tile_stats=ts, frame_stats=fs, lists=li, stf=sx)
    torch.cuda.synchronize()
    return dict(out=out.cpu().numpy(), stats=ctf.tile_stats_numpy(ts), frame=ctf.frame_stats_dict(fs),
                lists=li.cpu().numpy(), stf=sx.cpu().numpy())


def compare(g, o, what="", tol=TOL):
    """Full parity of one frame: decisions exact, colours within tol."""
    for f in STAT_FIELDS:
        a, b = g["stats"][f], o["stats"][f]
        bad = np.flatnonzero((a != b).reshape(len(a), -1).any(-1))
        assert bad.size == 0, f"{what}: tile field {f} differs at tiles {bad[:8]}: gpu {a[bad[:3]]} oracle {b[bad[:3]]}"
    ok = (o["stats"]["flags"] & O.TILE_OK) != 0
    for t in np.flatnonzero(ok):
        n = o["stats"]["n"][t]
        assert np.array_equal(g["lists"][t, :n], o["lists"][t, :n]), f"{what}: list of tile {t}"
    assert np.array_equal(g["stf"], o["stf"]), f"{what}: STF draws differ"
    err = np.abs(g["out"].astype(np.float64) - o["out"])
    print(f"colour error {what}: {err.max():.3e}", flush=True)
    assert err.max() <= tol, f"{what}: max colour error {err.max():.3e} at {np.unravel_index(err.argmax(), err.shape)}"
    st = o["stats"]
    fr = g["frame"]
    assert fr["evals"] == int(st["evals"].sum())
    assert fr["active"] == sum(bin(int(a)).count("1") for a in st["active"])
    assert fr["stf"] == sum(bin(int(a)).count("1") for a in st["stf"])
    return err.max()


def _method(G, kind, box, k):
    ctf = G[0]
    return ctf.method(kind, box=box, k=k)


@pytest.fixture(scope="module")
def c0():
    sc = cs.tilted_plane_scene()
    pqj, amp = cs.sinusoid_params(64, 8, 8, seed=0)
    return sc, pqj, amp


@pytest.mark.parametrize("name,gk,ok,box,k", METHODS)
def test_tiny_plane_parity(G, c0, name, gk, ok, box, k):
    """256x256 plane, 64x64 sinusoid texture (K=8): every output compared."""
    ctf, ctx, _ = G
    sc, pqj, amp = c0
    tex = ctx.sinusoid_texture(64, pqj, amp)
    otex = O.sinusoid_texture(64, pqj, amp)
    g = run_gpu(G, sc.uv, sc.duv, tex, _method(G, gk, box, k), seed=0)
    o = O.filter(sc.uv, sc.duv, otex, O.method(ok, box=box, k=k), seed=0, lists=True, stf=True)
    compare(g, o, name)
    tex.close()


@pytest.mark.parametrize("name,gk,ok,box,k", [m for m in METHODS if m[1] >= 2])
def test_collaborative_equals_bilinear4_bitwise(G, c0, name, gk, ok, box, k):
    """On successful waves, shared texels give exactly the 4-tap result."""
    ctf, ctx, _ = G
    sc, pqj, amp = c0
    tex = ctx.sinusoid_texture(64, pqj, amp)
    g4 = run_gpu(G, sc.uv, sc.duv, tex, _method(G, 0, (0, 0), 1))
    gc = run_gpu(G, sc.uv, sc.duv, tex, _method(G, gk, box, k))
    exact = gc["stf"][..., 0] == INT_MIN
    assert exact.sum() > 10000
    assert np.array_equal(g4["out"][exact], gc["out"][exact])
    tex.close()


@pytest.mark.parametrize("K", [62, 63, 64])
@pytest.mark.parametrize("name,gk,ok,box,k", [METHODS[0], METHODS[2], METHODS[6]])
def test_term_count_staging_boundary(G, c0, K, name, gk, ok, box, k):
    """Up to 62 terms per channel the per-lane kernels read the texture's
    terms from workgroup LDS, beyond that from memory: both forms give the
    oracle's result."""
    ctf, ctx, _ = G
    sc = c0[0]
    pqj, amp = cs.sinusoid_params(64, K, 8, seed=12)
    tex = ctx.sinusoid_texture(64, pqj, amp)
    otex = O.sinusoid_texture(64, pqj, amp)
    g = run_gpu(G, sc.uv, sc.duv, tex, _method(G, gk, box, k), seed=5)
    o = O.filter(sc.uv, sc.duv, otex, O.method(ok, box=box, k=k), seed=5, lists=True, stf=True)
    compare(g, o, f"{name} K={K}")
    tex.close()


def test_texel_eval_matches_float64(G):
    ctf, ctx, torch = G
    W = 2048
    pqj, amp = cs.sinusoid_params(W, 32, 64, seed=2)
    tex = ctx.sinusoid_texture(W, pqj, amp)
    rng = np.random.default_rng(0)
    xy = rng.integers(-(2**24), 2**24, (100000, 2)).astype(np.int32)
    got = tex.eval(torch.from_numpy(xy).cuda()).cpu().numpy()
    want = O.sinusoid_texture(W, pqj, amp).eval(xy)
    err = np.abs(got - want).max()
    assert err < 3e-7, err
    tex.close()


@pytest.mark.parametrize("W", [64, 4096, 8192])
def test_texel_eval_extreme_frequencies(G, W):
    """Frequencies and phases far outside [0, W) (up to the API's 2^23): the
    float phase form (W <= 4096, residues prepared at texture creation) and
    the integer form (W > 4096) both reduce them exactly; a wrong residue
    would give errors of order 1."""
    ctf, ctx, torch = G
    rng = np.random.default_rng(W)
    K = 16
    pqj = np.stack([rng.integers(-(1 << 23) + 1, 1 << 23, (4, K)), rng.integers(-(1 << 23) + 1, 1 << 23, (4, K)),
                    rng.integers(0, 1 << 31, (4, K))], axis=-1).astype(np.int32)
    pqj[0, 0] = (W // 2, -W // 2, W - 1)          # the residues' extremes
    pqj[0, 1] = (-W // 2 - 1, W // 2 - 1, 3 * W)
    a = rng.uniform(0.5, 1.5, (4, K))
    amp = (a / a.sum(axis=1, keepdims=True)).astype(np.float32)
    tex = ctx.sinusoid_texture(W, pqj, amp)
    xy = rng.integers(-(2**24), 2**24, (50000, 2)).astype(np.int32)
    xy[:4] = [(W - 1, W - 1), (0, 0), (-1, -1), (2**24 - 1, -(2**24))]
    got = tex.eval(torch.from_numpy(xy).cuda()).cpu().numpy()
    want = O.sinusoid_texture(W, pqj, amp).eval(xy)
    err = np.abs(got - want).max()
    print(f"texel error W={W}: {err:.3g}")
    assert err < 1e-6, err
    tex.close()


def test_affine_and_constant_textures(G, c0):
    ctf, ctx, _ = G
    sc = c0[0]
    coef = cs.affine_params(1)
    for kind in (0, 2, 3, 4):
        tex = ctx.affine_texture(64, 64, coef)
        g = run_gpu(G, sc.uv, sc.duv, tex, _method(G, kind, (4, 4), 1))
        o = O.filter(sc.uv, sc.duv, O.affine_texture(64, 64, coef),
                     O.method([O.BILINEAR4, 1, O.LIST, O.BOX, O.MASK][kind], box=(4, 4)), stf=True)
        assert np.array_equal(g["stf"], o["stf"])
        # float32 coefficients and arithmetic vs float64: relative 1e-6 of the magnitude
        assert np.abs(g["out"] - o["out"]).max() < 1e-6 * max(1.0, np.abs(o["out"]).max()) * 8
        tex.close()
        ctex = ctx.constant_texture(64, 64, (0.25, 0.5, 0.75, 1.0))
        g = run_gpu(G, sc.uv, sc.duv, ctex, _method(G, kind, (4, 4), 1))
        act = np.isfinite(sc.uv).all(-1)
        assert np.all(g["out"][act] == np.float32([0.25, 0.5, 0.75, 1.0]))
        assert np.all(g["out"][~act] == 0)
        ctex.close()


def _edge_scene():
    """Ragged 203x77 screen mixing every hard case, tile by tile."""
    rng = np.random.default_rng(7)
    sh, sw = 77, 203
    W = 64
    uv = np.zeros((sh, sw, 2), np.float32)
    duv = np.zeros((sh, sw, 4), np.float32)
    ys, xs = np.mgrid[0:sh, 0:sw]
    tiles_x = (sw + 7) // 8
    for ty in range((sh + 7) // 8):
        for tx in range(tiles_x):
            sl = (slice(ty * 8, ty * 8 + 8), slice(tx * 8, tx * 8 + 8))
            case = (ty * tiles_x + tx) % 9
            m = rng.uniform(0.6, 6.0)
            ang = rng.uniform(0, 2 * math.pi)
            off = rng.uniform(-200, 200, 2)
            c, s = math.cos(ang), math.sin(ang)
            px, py = xs[sl] + 0.5, ys[sl] + 0.5
            tu = (c * px - s * py) / m + off[0]
            tv = (s * px + c * py) / m + off[1]
            uv[sl] = np.stack([tu / W, tv / W], -1)
            duv[sl] = np.array([c / m / W, s / m / W, -s / m / W, c / m / W], np.float32)
            if case == 1:      # some lanes inactive (NaN, inf, huge)
                mask = rng.random(uv[sl].shape[:2]) < 0.4
                bad = uv[sl]
                bad[mask] = np.nan
                bad[rng.random(bad.shape[:2]) < 0.1] = np.array([np.inf, 0.5], np.float32)
                bad[rng.random(bad.shape[:2]) < 0.1] = np.array([1e9, 0.5], np.float32)
                uv[sl] = bad
            elif case == 2:    # all lanes minify
                duv[sl] = 3.0 / W
            elif case == 3:    # a single active lane
                u2 = uv[sl].copy()
                u2[...] = np.nan
                u2[0, 0] = uv[sl][0, 0]
                uv[sl] = u2
            elif case == 4:    # two surfaces in one tile: a large box (List sorts)
                part = uv[sl].copy()
                part[:, 4:] += np.float32(37.0 / W)
                uv[sl] = part
            elif case == 5:    # half minify, half magnify
                d = duv[sl].copy()
                d[::2] = 2.0 / W
                duv[sl] = d
            elif case == 6:    # exactly one texel per pixel: ties of the minify test
                duv[sl] = np.array([1.0 / W, 0, 0, 1.0 / W], np.float32)
            elif case == 7:    # texel centres (s = t = 0)
                u2 = uv[sl]
                uv[sl] = (np.floor(u2 * W) + 0.5) / W
            elif case == 8:    # strong magnification: one texel box
                uv[sl] = (uv[sl][0, 0] + (np.stack([px, py], -1) - px.min()) * 1e-3 / W).astype(np.float32)
    return uv, duv


@pytest.mark.parametrize("name,gk,ok,box,k", METHODS)
def test_edge_cases_ragged_screen(G, name, gk, ok, box, k):
    ctf, ctx, _ = G
    uv, duv = _edge_scene()
    pqj, amp = cs.sinusoid_params(64, 8, 8, seed=3)
    tex = ctx.sinusoid_texture(64, pqj, amp)
    g = run_gpu(G, uv, duv, tex, _method(G, gk, box, k), seed=99)
    o = O.filter(uv, duv, O.sinusoid_texture(64, pqj, amp), O.method(ok, box=box, k=k), seed=99,
                 lists=True, stf=True)
    compare(g, o, name)
    if gk == 2:   # the sort path of List was exercised
        st = o["stats"]
        assert np.any((st["bbw"] > 16) & ((st["flags"] & O.TILE_OK) != 0))
    tex.close()


def test_stf_seed_changes_draws(G, c0):
    ctf, ctx, _ = G
    sc, pqj, amp = c0
    tex = ctx.sinusoid_texture(64, pqj, amp)
    a = run_gpu(G, sc.uv, sc.duv, tex, _method(G, 1, (0, 0), 1), seed=1)
    b = run_gpu(G, sc.uv, sc.duv, tex, _method(G, 1, (0, 0), 1), seed=2 + (5 << 32))
    o = O.filter(sc.uv, sc.duv, O.sinusoid_texture(64, pqj, amp), O.method(O.STF1),
                 seed=2 + (5 << 32), stf=True)
    assert np.array_equal(b["stf"], o["stf"])
    assert not np.array_equal(a["stf"], b["stf"])
    tex.close()


@pytest.fixture(scope="module")
def c1():
    sc = cs.random_planes_scene(1920, 1080, seed=1)
    pqj, amp = cs.sinusoid_params(2048, 32, 64, seed=2)
    return sc, pqj, amp


@pytest.mark.parametrize("name,gk,ok,box,k", [m for m in METHODS if m[0] in
                                              ("bilinear4", "list", "box4x4", "box6x6", "mask")])
def test_1080p_four_planes_sampled_parity(G, c1, name, gk, ok, box, k):
    """Full 1920x1080 frame, K=32 on 2048^2: sampled tile ranges vs the oracle."""
    ctf, ctx, _ = G
    sc, pqj, amp = c1
    tex = ctx.sinusoid_texture(2048, pqj, amp)
    g = run_gpu(G, sc.uv, sc.duv, tex, _method(G, gk, box, k), seed=0)
    otex = O.sinusoid_texture(2048, pqj, amp)
    ntiles = 240 * 135
    rng = np.random.default_rng(1)
    starts = rng.integers(0, ntiles - 240, 6)
    for b in starts:
        e = b + 240
        o = O.filter(sc.uv, sc.duv, otex, O.method(ok, box=box, k=k), seed=0, tiles=(b, e),
                     lists=True, stf=True)
        for f in STAT_FIELDS:
            assert np.array_equal(g["stats"][f][b:e], o["stats"][f][b:e]), f"{name} {f} tiles {b}:{e}"
        tx0 = np.arange(b, e)
        rows = set(int(t // 240) for t in tx0)
        for t in tx0:
            ty, tx = divmod(int(t), 240)
            sl = (slice(ty * 8, ty * 8 + 8), slice(tx * 8, tx * 8 + 8))
            assert np.abs(g["out"][sl] - o["out"][sl]).max() <= TOL
            assert np.array_equal(g["stf"][sl], o["stf"][sl])
            if o["stats"]["flags"][t] & O.TILE_OK:
                n = o["stats"]["n"][t]
                assert np.array_equal(g["lists"][t, :n], o["lists"][t, :n])
    tex.close()


def _split_rule(st):
    """Tiles the library evaluates channel by channel over all 64 lanes:
    successful, no draws, ceil(n / 16) < 4 ceil(n / |A|)."""
    nA = np.array([bin(int(x)).count("1") for x in st["part"]], np.int64)
    n = st["n"].astype(np.int64)
    ok = ((st["flags"] & O.TILE_OK) != 0) & (st["stf"] == 0) & (nA > 0)
    per_lane = 4 * ((n + np.maximum(nA, 1) - 1) // np.maximum(nA, 1))
    return ok & ((n + 15) // 16 < per_lane), n


@pytest.mark.parametrize("name,gk,ok,box,k", [m for m in METHODS if m[1] >= 2])
def test_split_texel_production_is_bitwise_identical(G, c0, name, gk, ok, box, k):
    """Split-texel production (the 4n channels of a wave's texels spread
    over all 64 lanes) gives the same bits, lists and counts as one lane per
    texel: on the tilted plane (mostly n <= 32) and on head-on quads from
    0.45x (n up to 4 |A|)."""
    ctf, ctx, _ = G
    sc, pqj, amp = c0
    tex = ctx.sinusoid_texture(64, pqj, amp)
    quads = cs.lowmag_quads_scene(300, seed=5, tex_w=64, mag=(0.45, 4.0))
    total, wide = 0, 0
    for uv, duv in ((sc.uv, sc.duv), quads):
        on = run_gpu(G, uv, duv, tex, ctf.method(gk, box=box, k=k, split=ctf.SPLIT_AUTO), seed=4)
        off = run_gpu(G, uv, duv, tex, ctf.method(gk, box=box, k=k, split=ctf.SPLIT_OFF), seed=4)
        split_tiles, n = _split_rule(on["stats"])
        total += int(split_tiles.sum())
        wide += int((split_tiles & (n > 32)).sum())
        assert np.array_equal(on["out"], off["out"])
        assert np.array_equal(on["lists"], off["lists"])
        for f in STAT_FIELDS:
            assert np.array_equal(on["stats"][f], off["stats"][f]), f
    assert total > 20
    if box != (4, 4):
        assert wide > 0, "no split wave with more than 32 texels"
    tex.close()
