"""Whole frames at the benchmark's sizes against the oracle.

The kernels the benchmark times (no per-tile records requested) run on the
full 3840x2160 decoder frame, the six-layer 3840x2160 launch and every
procedural 1920x1080 configuration; the oracle runs the same whole frames on
the host's threads.  Compared: every pixel's one-tap draw (exact), every
pixel's colour (1e-6, bilinear and cubic) and the frame
counters -- texel evaluations, active, not-exact and minifying pixels, tiles,
successful and failed tiles -- against the sums of the oracle's tile
records (exact).  "Texel evaluations per pixel", half of the benchmark's
metric, is exactly such a frame counter.

Decoder textures: the oracle filters the GPU-decoded 2048^2 lattice as a
table (the decode itself is checked against the float64 network elsewhere).
Procedural textures: the oracle filters its own float64 lattice rounded to
float32 (2^-25 from float64, far inside the colour bound).
"""
import os

import numpy as np
import pytest

import ctf_synth as cs
import oracle as O
from test_gpu_decoder_launch import check_frame, lattice_table, run_launch

pytestmark = pytest.mark.gpu

FP16 = 0
# Cubic filters: the kernel takes the cubic weights in float32 (the op order
# of the one-tap draw); their rounding stays within the same 1e-6 bar
# (largest measured on these frames: 4.4e-7).
TOL_BILINEAR, TOL_CUBIC = 1e-6, 1e-6


@pytest.fixture(scope="module")
def G():
    import torch
    import paper_2506_17770_amd as ctf
    ctx = ctf.Context(0)
    yield ctf, ctx, torch
    ctx.close()


@pytest.fixture(scope="module")
def frame4k(G):
    ctf, ctx, torch = G
    sc = cs.random_planes_scene(3840, 2160, 2048, 2048, seed=1)
    dec = ctx.decoder(512, 128, 64, 2048, cs.decoder_init(512, 128, 64, seed=3, latent_range=0.5))
    tex = ctx.decoder_texture(dec, FP16)
    otex = O.table_texture(lattice_table(tex, 2048, torch))
    yield sc, tex, otex
    tex.close()
    dec.close()


@pytest.mark.parametrize("name,gk,ok,box,k,filt", [
    ("bilinear4", 0, O.BILINEAR4, (0, 0), 1, 0),
    ("list_k4", 2, O.LIST, (0, 0), 4, 0),
    ("box_k4", 3, O.BOX, (0, 0), 4, 0),
    ("mask_k2", 4, O.MASK, (0, 0), 2, 0),
    ("stf1", 1, O.STF1, (0, 0), 1, 0),
    ("bspline_list_k4", 2, O.LIST, (0, 0), 4, 1),
    ("bspline_full16", 0, O.BILINEAR4, (0, 0), 1, 1),
    ("catmull_rom_list_k4", 2, O.LIST, (0, 0), 4, 2),
    ("catmull_rom_full16", 0, O.BILINEAR4, (0, 0), 1, 2),
])
def test_full_frame_4k_decoder(G, frame4k, name, gk, ok, box, k, filt):
    """3840x2160, four planes, fp16 decoder on 2048^2 (latents 512^2 + 128^2):
    the whole frame, every pixel and every frame counter."""
    ctf, ctx, torch = G
    sc, tex, otex = frame4k
    print(f"case 4k {name}", flush=True)
    g = run_launch(G, sc.uv, sc.duv, tex, ctf.method(gk, box=box, k=k, filter=filt), seed=0)
    o = O.filter_parallel(sc.uv, sc.duv, otex, O.method(ok, box=box, k=k, filter=filt), seed=0)
    err = float(np.abs(g["out"].astype(np.float64) - o["out"]).max())
    print(f"4k {name}: max colour error {err:.3e}, evals/px {g['frame']['evals'] / (3840 * 2160):.4f}",
          flush=True)
    check_frame(g, o, gk >= 2, f"4k {name}", tol=TOL_CUBIC if filt else TOL_BILINEAR)


@pytest.mark.parametrize("prec", [0, 1])
def test_full_frame_layers_4k(G, prec):
    """Six material layers at 3840x2160 in one launch, List k=4 and 4-tap:
    every layer's whole frame, and the launch's frame counters against the
    oracle's tile records summed over all six layers."""
    ctf, ctx, torch = G
    n = 6
    print(f"case layers 4k precision {prec}", flush=True)
    sc = cs.random_planes_scene(3840, 2160, 2048, 2048, seed=1)
    mats = np.array([cs.layer_params(11, l)[2] for l in range(n)], np.float32)
    decs = [ctx.decoder(512, 128, 64, 2048, cs.decoder_init(512, 128, 64, seed=100 + l, latent_range=0.5))
            for l in range(n)]
    texs = [ctx.decoder_texture(d, prec) for d in decs]
    tables = [lattice_table(t, 2048, torch) for t in texs]
    uv, duv = torch.from_numpy(sc.uv).cuda(), torch.from_numpy(sc.duv).cuda()
    for gk, ok, k in ((2, O.LIST, 4), (0, O.BILINEAR4, 1)):
        sx = torch.full((n, 2160, 3840, 2), -2**31, dtype=torch.int32, device="cuda")
        fs = ctf.frame_stats_buffer()
        out = ctx.filter_layers(uv, duv, texs, mats, ctf.method(gk, k=k), seed=0, stf=sx, frame_stats=fs)
        torch.cuda.synchronize()
        out, sx, fr = out.cpu().numpy(), sx.cpu().numpy(), ctf.frame_stats_dict(fs)
        stats = []
        for l in range(n):
            o = O.filter_parallel(sc.uv, sc.duv, O.table_texture(tables[l]), O.method(ok, k=k), seed=0, layer=l,
                                  xform=mats[l])
            err = float(np.abs(out[l].astype(np.float64) - o["out"]).max())
            assert err <= TOL_BILINEAR, f"layer {l} kind {gk}: colour error {err:.3e}"
            assert np.array_equal(sx[l], o["stf"]), f"layer {l} kind {gk}: draws differ"
            stats.append(o["stats"])
        st = np.concatenate(stats)
        pc = lambda a: int(np.unpackbits(np.ascontiguousarray(a).view(np.uint8)).sum())
        assert fr["evals"] == int(st["evals"].sum())
        assert fr["active"] == pc(st["active"]) and fr["stf"] == pc(st["stf"])
        assert fr["minify"] == pc(st["active"] & ~st["part"])
        assert fr["tiles"] == int((st["active"] != 0).sum())
        if gk >= 2:
            okm = (st["flags"] & O.TILE_OK) != 0
            assert fr["tiles_ok"] == int(okm.sum())
            assert fr["tiles_fail"] == int(((st["part"] != 0) & ~okm).sum())
    for t in texs:
        t.close()
    for d in decs:
        d.close()


@pytest.fixture(scope="module")
def frame1080(G):
    """The 1920x1080 four-plane frame and the 2048^2 procedural texture (32
    sinusoids per channel); the oracle's float64 lattice, rounded to float32,
    evaluated on the host's threads."""
    import threading
    ctf, ctx, torch = G
    sc = cs.random_planes_scene(1920, 1080, 2048, 2048, seed=1)
    pqj, amp = cs.sinusoid_params(2048, 32, 64, seed=2)
    tex = ctx.sinusoid_texture(2048, pqj, amp)
    osin = O.sinusoid_texture(2048, pqj, amp)
    ys, xs = np.mgrid[0:2048, 0:2048]
    xy = np.ascontiguousarray(np.stack([xs.ravel(), ys.ravel()], -1).astype(np.int32))
    table = np.empty((xy.shape[0], 4), np.float32)
    parts = np.array_split(np.arange(xy.shape[0]), min(16, os.cpu_count() or 1))

    def work(ix):
        table[ix] = osin.eval(xy[ix])

    ths = [threading.Thread(target=work, args=(ix,)) for ix in parts]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    yield sc, tex, O.table_texture(table.reshape(2048, 2048, 4))
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
def test_full_frame_procedural_1080p(G, frame1080, name, gk, ok, box, k, fb, w84, split):
    """Every procedural configuration the benchmark times, whole frame."""
    ctf, ctx, torch = G
    sc, tex, otab = frame1080
    print(f"case 1080p {name}", flush=True)
    gm = ctf.method(gk, box=box, k=k, fallback=fb, split=ctf.SPLIT_OFF if split else ctf.SPLIT_AUTO,
                    wave_shape=ctf.WAVE_8X4 if w84 else ctf.WAVE_8X8)
    g = run_launch(G, sc.uv, sc.duv, tex, gm, seed=0)
    o = O.filter_parallel(sc.uv, sc.duv, otab, O.method(ok, box=box, k=k, fallback=fb), seed=0,
                          tile=(8, 4) if w84 else (8, 8))
    check_frame(g, o, gk >= 2, f"1080p {name}", tol=TOL_BILINEAR)
