"""The filter in the launch configuration the benchmark times.

With no per-tile records or item lists requested the library runs its
kernels without statistics: on the decoder path the batched List / Box /
Mask kernel (rows of two tiles decoded per pass, the 16x16 window test of
List and Mask) and the per-tile kernel of the other methods; on the
procedural path the per-lane kernels (split texels on, fallbacks, bicubic,
8x4 waves).  They are checked against the oracle (on the decoder path
filtering the GPU-decoded texel lattice): one-tap draws and frame counts
exact, colours within 1e-6 (2e-6 for the cubics) -- on the small scenes in
full, and at 3840x2160 with the 2048^2 decoder of the benchmark on sampled
rows of tiles.
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


@pytest.mark.parametrize("name,gk,ok,box,k", [m for m in METHODS if m[0] in
                                              ("bilinear4", "list_k4", "box_k4", "mask_k2")])
def test_launch_configuration_4k_sampled(G, c4k, name, gk, ok, box, k):
    """3840x2160, fp16 decoder on 2048^2 (latents 512^2 + 128^2): the whole
    frame on the GPU, eight rows of 480 tiles (first, last, six seeded) on
    the oracle."""
    ctf, ctx, torch = G
    sc, tex, otex = c4k
    g = run_launch(G, sc.uv, sc.duv, tex, ctf.method(gk, box=box, k=k), seed=0)
    tiles_x, tiles_y = 480, 270
    rows = [0, tiles_y - 1] + list(np.random.default_rng(7).choice(np.arange(1, tiles_y - 1), 6, replace=False))
    for ty in rows:
        b, e = ty * tiles_x, (ty + 1) * tiles_x
        o = O.filter(sc.uv, sc.duv, otex, O.method(ok, box=box, k=k), seed=0, tiles=(b, e), stf=True)
        sl = slice(8 * ty, 8 * ty + 8)
        err = np.abs(g["out"][sl].astype(np.float64) - o["out"][sl]).max()
        assert err <= TOL, f"{name}: tile row {ty} colour error {err:.3e}"
        assert np.array_equal(g["stf"][sl], o["stf"][sl]), f"{name}: tile row {ty} draws"


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
        check_frame(g, o, gk >= 2, f"{name} {sname}", tol=2e-6 if filt else TOL)
    tex.close()
