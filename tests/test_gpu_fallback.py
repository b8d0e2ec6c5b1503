"""GPU parity of fallbacks C (Eq. 1) and C+ (Eq. 2) against the oracle.

Scenes where most waves fail: head-on quads near magnification 1 (exact sets
overflow one evaluation per lane) and the ragged edge-case screen (inactive
lanes, mixed minification, boxes past 16x16 where C+ reduces to C).  Same bar
as the other filter tests: decisions, draws and evaluation counts exact,
colours within 1e-6 of the float64 oracle.
"""
import numpy as np
import pytest

import ctf_synth as cs
import oracle as O

pytestmark = pytest.mark.gpu

FP16, BF16 = 0, 1
FALLBACKS = [("C", O.FB_C), ("Cplus", O.FB_CPLUS)]
METHODS = [("list", 2, O.LIST, (0, 0), 1), ("box", 3, O.BOX, (0, 0), 1),
           ("box4x4", 3, O.BOX, (4, 4), 1), ("mask", 4, O.MASK, (0, 0), 1),
           ("list_k2", 2, O.LIST, (0, 0), 2)]


@pytest.fixture(scope="module")
def G():
    import torch
    import paper_2506_17770_amd as ctf
    ctx = ctf.Context(0)
    yield ctf, ctx, torch
    ctx.close()


def _scenes():
    from test_gpu_filter import _edge_scene
    return [("lowmag", cs.lowmag_quads_scene(600, seed=21, tex_w=64)), ("edge", _edge_scene())]


def _check_fallback_ran(o, uv):
    st = o["stats"]
    failed = (st["part"] != 0) & ((st["flags"] & O.TILE_OK) == 0)
    assert failed.sum() >= 20


@pytest.mark.parametrize("fbname,fb", FALLBACKS)
@pytest.mark.parametrize("name,gk,ok,box,k", METHODS)
def test_fallback_parity_procedural(G, fbname, fb, name, gk, ok, box, k):
    from test_gpu_filter import compare, run_gpu
    ctf, ctx, _ = G
    pqj, amp = cs.sinusoid_params(64, 8, 8, seed=3)
    tex = ctx.sinusoid_texture(64, pqj, amp)
    otex = O.sinusoid_texture(64, pqj, amp)
    for sname, (uv, duv) in _scenes():
        g = run_gpu(G, uv, duv, tex, ctf.method(gk, box=box, k=k, fallback=fb), seed=17)
        o = O.filter(uv, duv, otex, O.method(ok, box=box, k=k, fallback=fb), seed=17, lists=True,
                     stf=True)
        if sname == "lowmag" and k == 1:
            _check_fallback_ran(o, uv)
        compare(g, o, f"{name} {fbname} {sname}")
    tex.close()


@pytest.mark.parametrize("fb", [O.FB_C, O.FB_CPLUS])
def test_fallback_leaves_successful_waves_bitwise(G, fb):
    """Waves that succeed give the same bits whatever the fallback."""
    from test_gpu_filter import run_gpu
    ctf, ctx, _ = G
    pqj, amp = cs.sinusoid_params(64, 8, 8, seed=4)
    tex = ctx.sinusoid_texture(64, pqj, amp)
    uv, duv = cs.lowmag_quads_scene(600, seed=22, tex_w=64, mag=(1.0, 2.0))
    a = run_gpu(G, uv, duv, tex, ctf.method(ctf.MASK), seed=3)
    b = run_gpu(G, uv, duv, tex, ctf.method(ctf.MASK, fallback=fb), seed=3)
    ok = (a["stats"]["flags"] & O.TILE_OK) != 0
    assert ok.sum() > 50 and (~ok).sum() > 50
    okpx = np.repeat(ok, 8)[None, :].repeat(8, 0)
    assert np.array_equal(a["out"][okpx], b["out"][okpx])
    assert not np.array_equal(a["out"][~okpx], b["out"][~okpx])
    tex.close()


@pytest.mark.parametrize("prec", [FP16, BF16])
@pytest.mark.parametrize("fbname,fb", FALLBACKS)
@pytest.mark.parametrize("name,gk,ok,box,k", [m for m in METHODS if m[0] in ("list", "box4x4", "mask")])
def test_fallback_parity_decoder(G, prec, fbname, fb, name, gk, ok, box, k):
    """Decoder producer: the oracle filters the GPU-decoded texel lattice."""
    from test_gpu_decoder import _decoder_case, _lattice_table
    from test_gpu_filter import compare, run_gpu
    ctf, ctx, torch = G
    dec, _ = _decoder_case(ctx)
    tex = ctx.decoder_texture(dec, prec)
    otex = O.table_texture(_lattice_table(tex, 64, torch))
    for sname, (uv, duv) in _scenes():
        g = run_gpu(G, uv, duv, tex, ctf.method(gk, box=box, k=k, fallback=fb), seed=23)
        o = O.filter(uv, duv, otex, O.method(ok, box=box, k=k, fallback=fb), seed=23, lists=True,
                     stf=True)
        compare(g, o, f"decoder {name} {fbname} {sname}")
    tex.close()
    dec.close()


def test_fallback_parity_layers(G):
    """Two material layers in one launch with fallback C+."""
    from test_gpu_filter import STAT_FIELDS
    ctf, ctx, torch = G
    n = 2
    decs = [ctx.decoder(16, 4, 64, 64, cs.decoder_init(16, 4, 64, seed=40 + i, latent_range=0.5))
            for i in range(n)]
    texs = [ctx.decoder_texture(d, FP16) for d in decs]
    ys, xs = np.mgrid[0:64, 0:64]
    lattice = torch.from_numpy(np.stack([xs.ravel(), ys.ravel()], -1).astype(np.int32)).cuda()
    tables = [t.eval(lattice).cpu().numpy().reshape(64, 64, 4) for t in texs]
    xf = np.array([np.eye(2), [[0.0, -1.0], [1.0, 0.0]]], np.float32)   # identity, 90 degrees
    uv, duv = cs.lowmag_quads_scene(300, seed=23, tex_w=64)
    sh, sw = uv.shape[:2]
    tiles = ((sw + 7) // 8) * ((sh + 7) // 8)
    ts = torch.zeros((n, tiles, 128), dtype=torch.uint8, device="cuda")
    sx = torch.full((n, sh, sw, 2), -2**31, dtype=torch.int32, device="cuda")
    m = ctf.method(ctf.LIST, fallback=ctf.FB_CPLUS)
    out = ctx.filter_layers(torch.from_numpy(uv).cuda(), torch.from_numpy(duv).cuda(), texs, xf, m,
                            seed=4, tile_stats=ts, stf=sx)
    torch.cuda.synchronize()
    out = out.cpu().numpy()
    for l in range(n):
        o = O.filter(uv, duv, O.table_texture(tables[l]), O.method(O.LIST, fallback=O.FB_CPLUS), seed=4,
                     layer=l, xform=xf[l], stf=True)
        st = ctf.tile_stats_numpy(ts[l])
        for f in STAT_FIELDS:
            assert np.array_equal(st[f], o["stats"][f]), (l, f)
        assert np.array_equal(sx[l].cpu().numpy(), o["stf"]), l
        assert np.abs(out[l] - o["out"]).max() <= 1e-6, l
    for t in texs:
        t.close()
    for d in decs:
        d.close()
