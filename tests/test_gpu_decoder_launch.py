"""The filter in the launch configuration the benchmark times.

With no per-tile records or item lists requested the library runs its
kernels without statistics: on the decoder path the batched List / Box /
Mask kernel (rows of two tiles decoded per pass, the 16x16 window test of
List and Mask) and the per-tile kernel of the other methods; on the
procedural path the per-lane kernels (split texels on, fallbacks, bicubic,
8x4 waves).  They are checked against the oracle (on the decoder path
filtering the GPU-decoded texel lattice): one-tap draws and frame counts
exact, colours within 1e-6 (the cubics too) -- on the small scenes in
full, and at the benchmark's sizes on sampled rows of tiles: 3840x2160 with
the 2048^2 decoder (bilinear and both bicubics), six layers at 3840x2160 in
one launch, and every procedural configuration at 1920x1080 with 32
sinusoids per channel on 2048^2.
"""
import numpy as np
import pytest

import ctf_synth as cs
import oracle as O

pytestmark = pytest.mark.gpu

TOL = 1e-6
FP16, BF16 = 0, 1
METHODS = [  # (name, gpu kind, oracle kind, box budget, k)
    ("bilinear4", 0, O.BILINEAR4, (0, 0), 1),
    ("stf1", 1, O.STF1, (0, 0), 1),
    ("list_k4", 2, O.LIST, (0, 0), 4),
    ("list", 2, O.LIST, (0, 0), 1),
    ("box4x4", 3, O.BOX, (4, 4), 1),
    ("box_k4", 3, O.BOX, (0, 0), 4),
    ("mask", 4, O.MASK, (0, 0), 1),
    ("mask_k2", 4, O.MASK, (0, 0), 2),
]


@pytest.fixture(scope="module")
def G():
    import torch
    import paper_2506_17770_amd as ctf
    ctx = ctf.Context(0)
    yield ctf, ctx, torch
    ctx.close()


def run_launch(G, uv, duv, tex, meth, seed):
    """The filter with frame totals and draws only (no per-tile outputs)."""
    ctf, ctx, torch = G
    sh, sw = uv.shape[:2]
    fs = ctf.frame_stats_buffer()
    sx = ctf.stf_buffer(sw, sh)
    out = ctx.filter(torch.from_numpy(np.ascontiguousarray(uv)).cuda(),
                     torch.from_numpy(np.ascontiguousarray(duv)).cuda(), tex, meth, seed=seed,
                     frame_stats=fs, stf=sx)
    torch.cuda.synchronize()
    return dict(out=out.cpu().numpy(), frame=ctf.frame_stats_dict(fs), stf=sx.cpu().numpy())


def lattice_table(tex, tex_w, torch):
    ys, xs = np.mgrid[0:tex_w, 0:tex_w]
    xy = np.stack([xs.ravel(), ys.ravel()], -1).astype(np.int32)
    return tex.eval(torch.from_numpy(xy).cuda()).cpu().numpy().reshape(tex_w, tex_w, 4)


def popcount(a):
    return sum(bin(int(v)).count("1") for v in a)


def check_frame(g, o, collaborative, what, tol=TOL):
    assert np.array_equal(g["stf"], o["stf"]), f"{what}: draws differ"
    err = np.abs(g["out"].astype(np.float64) - o["out"])
    print(f"colour error {what}: {err.max():.3e}", flush=True)
    assert err.max() <= tol, f"{what}: colour error {err.max():.3e}"
    st, fr = o["stats"], g["frame"]
    assert fr["evals"] == int(st["evals"].sum()), what
    assert fr["active"] == popcount(st["active"]), what
    assert fr["stf"] == popcount(st["stf"]), what
    assert fr["minify"] == popcount(st["active"] & ~st["part"]), what
    assert fr["tiles"] == int((st["active"] != 0).sum()), what
    if collaborative:
        ok = (st["flags"] & O.TILE_OK) != 0
        assert fr["tiles_ok"] == int(ok.sum()), what
        assert fr["tiles_fail"] == int(((st["part"] != 0) & ~ok).sum()), what


def small_scenes():
    from test_gpu_filter import _edge_scene
    sc = cs.tilted_plane_scene()
    # head-on quads from 0.45x (boxes past 16x16: the sorted List) to 4x
    low_uv, low_duv = cs.lowmag_quads_scene(300, seed=5, tex_w=64, mag=(0.45, 4.0))
    return [("edge", *_edge_scene()), ("tilted", sc.uv, sc.duv), ("quads", low_uv, low_duv)]


@pytest.mark.parametrize("prec", [FP16, BF16])
@pytest.mark.parametrize("name,gk,ok,box,k", METHODS)
def test_launch_configuration_parity_small(G, prec, name, gk, ok, box, k):
    ctf, ctx, torch = G
    dec = ctx.decoder(16, 4, 64, 64, cs.decoder_init(16, 4, 64, seed=5, latent_range=0.5))
    tex = ctx.decoder_texture(dec, prec)
    otex = O.table_texture(lattice_table(tex, 64, torch))
    for sname, uv, duv in small_scenes():
        g = run_launch(G, uv, duv, tex, ctf.method(gk, box=box, k=k), seed=13)
        o = O.filter(uv, duv, otex, O.method(ok, box=box, k=k), seed=13, stf=True)
        check_frame(g, o, gk >= 2, f"{name} {sname}")
    tex.close()
    dec.close()


@pytest.fixture(scope="module")
def c4k(G):
    ctf, ctx, torch = G
    sc = cs.random_planes_scene(3840, 2160, 2048, 2048, seed=1)
    dec = ctx.decoder(512, 128, 64, 2048, cs.decoder_init(512, 128, 64, seed=3, latent_range=0.5))
    tex = ctx.decoder_texture(dec, FP16)
    otex = O.table_texture(lattice_table(tex, 2048, torch))
    yield sc, tex, otex
    tex.close()
    dec.close()


def sampled_tile_rows(tiles_y, n, seed):
    """First and last tile rows plus n - 2 seeded ones."""
    mid = np.random.default_rng(seed).choice(np.arange(1, tiles_y - 1), n - 2, replace=False)
    return [0, tiles_y - 1] + [int(t) for t in mid]


def check_tile_rows(g_out, g_stf, o_for_rows, rows, tiles_x, tile_h, tol, what):
    """Colours and draws of whole tile rows against the oracle run on them."""
    for ty in rows:
        o = o_for_rows((ty * tiles_x, (ty + 1) * tiles_x))
        sl = slice(tile_h * ty, tile_h * ty + tile_h)
        err = np.abs(g_out[sl].astype(np.float64) - o["out"][sl]).max()
        assert err <= tol, f"{what}: tile row {ty} colour error {err:.3e}"
        assert np.array_equal(g_stf[sl], o["stf"][sl]), f"{what}: tile row {ty} draws"


@pytest.mark.parametrize("name,gk,ok,box,k,filt", [
    ("bilinear4", 0, O.BILINEAR4, (0, 0), 1, 0),
    ("list_k4", 2, O.LIST, (0, 0), 4, 0),
    ("box_k4", 3, O.BOX, (0, 0), 4, 0),
    ("mask_k2", 4, O.MASK, (0, 0), 2, 0),
    ("bspline_list_k4", 2, O.LIST, (0, 0), 4, 1),
    ("bspline_full16", 0, O.BILINEAR4, (0, 0), 1, 1),
    ("catmull_rom_list_k4", 2, O.LIST, (0, 0), 4, 2),
    ("catmull_rom_full16", 0, O.BILINEAR4, (0, 0), 1, 2),
])
def test_launch_configuration_4k_sampled(G, c4k, name, gk, ok, box, k, filt):
    """3840x2160, fp16 decoder on 2048^2 (latents 512^2 + 128^2), bilinear
    and the two bicubics: the whole frame on the GPU, eight rows of 480
    tiles (first, last, six seeded) on the oracle."""
    ctf, ctx, torch = G
    sc, tex, otex = c4k
    g = run_launch(G, sc.uv, sc.duv, tex, ctf.method(gk, box=box, k=k, filter=filt), seed=0)
    om = O.method(ok, box=box, k=k, filter=filt)
    check_tile_rows(g["out"], g["stf"],
                    lambda tr: O.filter(sc.uv, sc.duv, otex, om, seed=0, tiles=tr, stf=True),
                    sampled_tile_rows(270, 8, 7), 480, 8, TOL, name)


@pytest.mark.parametrize("prec", [FP16, BF16])
def test_launch_configuration_layers_4k_sampled(G, prec):
    """Six material layers at 3840x2160 in one launch, each with its own
    2048^2 decoder (latents 512^2 + 128^2) and uv_l = s_l R(theta_l) uv:
    List k=4 and 4-tap, four tile rows per layer on the oracle."""
    ctf, ctx, torch = G
    n = 6
    sc = cs.random_planes_scene(3840, 2160, 2048, 2048, seed=1)
    mats = np.array([cs.layer_params(11, l)[2] for l in range(n)], np.float32)
    decs = [ctx.decoder(512, 128, 64, 2048, cs.decoder_init(512, 128, 64, seed=100 + l, latent_range=0.5))
            for l in range(n)]
    texs = [ctx.decoder_texture(d, prec) for d in decs]
    otexs = [O.table_texture(lattice_table(t, 2048, torch)) for t in texs]
    uv, duv = torch.from_numpy(sc.uv).cuda(), torch.from_numpy(sc.duv).cuda()
    for gk, ok, k in ((2, O.LIST, 4), (0, O.BILINEAR4, 1)):
        sx = torch.full((n, 2160, 3840, 2), -2**31, dtype=torch.int32, device="cuda")
        out = ctx.filter_layers(uv, duv, texs, mats, ctf.method(gk, k=k), seed=0, stf=sx)
        torch.cuda.synchronize()
        out, sx = out.cpu().numpy(), sx.cpu().numpy()
        for l in range(n):
            check_tile_rows(out[l], sx[l],
                            lambda tr: O.filter(sc.uv, sc.duv, otexs[l], O.method(ok, k=k), seed=0, layer=l,
                                                xform=mats[l], tiles=tr, stf=True),
                            sampled_tile_rows(270, 4, 30 + l), 480, 8, TOL, f"layer {l} kind {gk}")
    for t in texs:
        t.close()
    for d in decs:
        d.close()


PROCEDURAL = [  # (name, gpu kind, oracle kind, box, k, fallback, filter, 8x4 waves)
    ("bilinear4", 0, O.BILINEAR4, (0, 0), 1, 0, 0, False),
    ("stf1", 1, O.STF1, (0, 0), 1, 0, 0, False),
    ("list", 2, O.LIST, (0, 0), 1, 0, 0, False),
    ("list_k2", 2, O.LIST, (0, 0), 2, 0, 0, False),
    ("box4x4", 3, O.BOX, (4, 4), 1, 0, 0, False),
    ("mask", 4, O.MASK, (0, 0), 1, 0, 0, False),
    ("mask_fbC", 4, O.MASK, (0, 0), 1, 1, 0, False),
    ("mask_fbCplus", 4, O.MASK, (0, 0), 1, 2, 0, False),
    ("list_bspline_k4", 2, O.LIST, (0, 0), 4, 0, 1, False),
    ("mask_catmull_rom_k4", 4, O.MASK, (0, 0), 4, 0, 2, False),
    ("bilinear4_8x4", 0, O.BILINEAR4, (0, 0), 1, 0, 0, True),
    ("list_8x4", 2, O.LIST, (0, 0), 1, 0, 0, True),
    ("box4x4_8x4", 3, O.BOX, (4, 4), 1, 0, 0, True),
    ("mask_8x4", 4, O.MASK, (0, 0), 1, 0, 0, True),
]


@pytest.mark.parametrize("name,gk,ok,box,k,fb,filt,w84", PROCEDURAL)
def test_launch_configuration_procedural_small(G, name, gk, ok, box, k, fb, filt, w84):
    ctf, ctx, torch = G
    pqj, amp = cs.sinusoid_params(64, 8, 8, seed=0)
    tex = ctx.sinusoid_texture(64, pqj, amp)
    otex = O.sinusoid_texture(64, pqj, amp)
    gm = ctf.method(gk, box=box, k=k, fallback=fb, filter=filt,
                    wave_shape=ctf.WAVE_8X4 if w84 else ctf.WAVE_8X8)
    om = O.method(ok, box=box, k=k, fallback=fb, filter=filt)
    for sname, uv, duv in small_scenes():
        g = run_launch(G, uv, duv, tex, gm, seed=13)
        o = O.filter(uv, duv, otex, om, seed=13, stf=True, tile=(8, 4) if w84 else (8, 8))
        check_frame(g, o, gk >= 2, f"{name} {sname}", tol=TOL)
    tex.close()


@pytest.fixture(scope="module")
def c1080(G):
    ctf, ctx, torch = G
    sc = cs.random_planes_scene(1920, 1080, 2048, 2048, seed=1)
    pqj, amp = cs.sinusoid_params(2048, 32, 64, seed=2)
    tex = ctx.sinusoid_texture(2048, pqj, amp)
    yield sc, tex, O.sinusoid_texture(2048, pqj, amp)
    tex.close()


@pytest.mark.parametrize("name,gk,ok,box,k,fb,w84,split", [
    ("bilinear4", 0, O.BILINEAR4, (0, 0), 1, 0, False, 0),
    ("stf1", 1, O.STF1, (0, 0), 1, 0, False, 0),
    ("list", 2, O.LIST, (0, 0), 1, 0, False, 0),
    ("box4x4", 3, O.BOX, (4, 4), 1, 0, False, 0),
    ("box6x6", 3, O.BOX, (6, 6), 1, 0, False, 0),
    ("mask", 4, O.MASK, (0, 0), 1, 0, False, 0),
    ("mask_fbC", 4, O.MASK, (0, 0), 1, 1, False, 0),
    ("mask_fbCplus", 4, O.MASK, (0, 0), 1, 2, False, 0),
    ("list_k2", 2, O.LIST, (0, 0), 2, 0, False, 0),
    ("list_no_split", 2, O.LIST, (0, 0), 1, 0, False, 1),
    ("mask_no_split", 4, O.MASK, (0, 0), 1, 0, False, 1),
    ("bilinear4_8x4", 0, O.BILINEAR4, (0, 0), 1, 0, True, 0),
    ("list_8x4", 2, O.LIST, (0, 0), 1, 0, True, 0),
    ("box4x4_8x4", 3, O.BOX, (4, 4), 1, 0, True, 0),
    ("mask_8x4", 4, O.MASK, (0, 0), 1, 0, True, 0),
    ("mask_fbCplus_8x4", 4, O.MASK, (0, 0), 1, 2, True, 0),
])
def test_launch_configuration_procedural_1080p_sampled(G, c1080, name, gk, ok, box, k, fb, w84, split):
    """1920x1080, 32 sinusoids per channel on 2048^2, every configuration
    the benchmark times, without per-tile records: six tile rows on the
    oracle (8x8 tiles: rows of 240; 8x4 tiles: rows of 240 four pixels
    high)."""
    ctf, ctx, torch = G
    sc, tex, otex = c1080
    split_mode = ctf.SPLIT_OFF if split else ctf.SPLIT_AUTO
    gm = ctf.method(gk, box=box, k=k, fallback=fb, split=split_mode,
                    wave_shape=ctf.WAVE_8X4 if w84 else ctf.WAVE_8X8)
    g = run_launch(G, sc.uv, sc.duv, tex, gm, seed=0)
    om = O.method(ok, box=box, k=k, fallback=fb)
    th = 4 if w84 else 8
    check_tile_rows(g["out"], g["stf"],
                    lambda tr: O.filter(sc.uv, sc.duv, otex, om, seed=0, tiles=tr, stf=True, tile=(8, th)),
                    sampled_tile_rows(1080 // th, 6, 11), 240, th, TOL, name)


@pytest.mark.parametrize("name,gk,ok,box", [("bilinear4", 0, O.BILINEAR4, (0, 0)), ("stf1", 1, O.STF1, (0, 0)),
                                            ("list", 2, O.LIST, (0, 0)), ("box6x6", 3, O.BOX, (6, 6)),
                                            ("mask", 4, O.MASK, (0, 0))])
def test_launch_configuration_constant_texture(G, name, gk, ok, box):
    """The constant texture the benchmark uses to time the dedup machinery
    alone, through the same statistics-free kernels."""
    ctf, ctx, torch = G
    rgba = (0.25, 0.5, 0.75, 1.0)
    tex = ctx.constant_texture(2048, 2048, rgba)
    otex = O.constant_texture(2048, 2048, rgba)
    for sname, uv, duv in small_scenes():
        g = run_launch(G, uv, duv, tex, ctf.method(gk, box=box), seed=13)
        o = O.filter(uv, duv, otex, O.method(ok, box=box), seed=13, stf=True)
        check_frame(g, o, gk >= 2, f"{name} {sname}")
    tex.close()
