"""GPU parity of the bicubic filters (Section 5: B-spline, Catmull-Rom; 4x4
footprints) on the per-lane and the decoder producers, against the oracle.

Decisions, lists, draws and counts exact.  Colours within 1e-6 of the
float64 oracle, the bar of the bilinear path.  The cubic weighting takes
16 float32 weights (each within half an ulp of its float64 value) and 16
float32 products and sums; with procedural texels within 3e-7 of float64
and sum |w| <= 1.27 (Catmull-Rom's largest) the error stays below 1e-6
(largest measured over every case here: 5.9e-7).
"""
import numpy as np
import pytest

import ctf_synth as cs
import oracle as O

pytestmark = pytest.mark.gpu

TOL_CUBIC = 1e-6
FILTERS = [("bspline", O.FILTER_BSPLINE), ("catmull_rom", O.FILTER_CATMULL_ROM)]
METHODS = [("full", 0, O.BILINEAR4, (0, 0), 1), ("stf1", 1, O.STF1, (0, 0), 1),
           ("list", 2, O.LIST, (0, 0), 1), ("list_k2", 2, O.LIST, (0, 0), 2),
           ("box", 3, O.BOX, (0, 0), 1), ("box6x6_k2", 3, O.BOX, (6, 6), 2),
           ("mask", 4, O.MASK, (0, 0), 1), ("mask_k4", 4, O.MASK, (0, 0), 4)]


@pytest.fixture(scope="module")
def G():
    import torch
    import paper_2506_17770_amd as ctf
    ctx = ctf.Context(0)
    yield ctf, ctx, torch
    ctx.close()


def _scenes():
    from test_gpu_filter import _edge_scene
    sc = cs.tilted_plane_scene()
    return [("plane", (sc.uv, sc.duv)), ("edge", _edge_scene()),
            ("quads", cs.lowmag_quads_scene(300, seed=31, tex_w=64, mag=(0.9, 4.0)))]


@pytest.mark.parametrize("fname,flt", FILTERS)
@pytest.mark.parametrize("name,gk,ok,box,k", METHODS)
def test_bicubic_parity(G, fname, flt, name, gk, ok, box, k):
    from test_gpu_filter import compare, run_gpu
    ctf, ctx, _ = G
    pqj, amp = cs.sinusoid_params(64, 8, 8, seed=5)
    tex = ctx.sinusoid_texture(64, pqj, amp)
    otex = O.sinusoid_texture(64, pqj, amp)
    for sname, (uv, duv) in _scenes():
        g = run_gpu(G, uv, duv, tex, ctf.method(gk, box=box, k=k, filter=flt), seed=13)
        o = O.filter(uv, duv, otex, O.method(ok, box=box, k=k, filter=flt), seed=13, lists=True, stf=True)
        compare(g, o, f"{fname} {name} {sname}", tol=TOL_CUBIC)
        if gk == 2 and k == 2 and sname == "edge":   # the sorted (past 16x16) List path ran
            st = o["stats"]
            assert np.any((st["bbw"] > 16) & ((st["flags"] & O.TILE_OK) != 0))
    tex.close()


@pytest.mark.parametrize("fname,flt", FILTERS)
@pytest.mark.parametrize("gk,k", [(2, 2), (3, 4), (4, 2)])
def test_bicubic_collaborative_equals_full_bitwise(G, fname, flt, gk, k):
    from test_gpu_filter import run_gpu
    ctf, ctx, _ = G
    pqj, amp = cs.sinusoid_params(64, 8, 8, seed=6)
    tex = ctx.sinusoid_texture(64, pqj, amp)
    sc = cs.tilted_plane_scene()
    full = run_gpu(G, sc.uv, sc.duv, tex, ctf.method(0, filter=flt))
    col = run_gpu(G, sc.uv, sc.duv, tex, ctf.method(gk, k=k, filter=flt))
    exact = col["stf"][..., 0] == np.iinfo(np.int32).min
    assert exact.sum() > 5000
    assert np.array_equal(full["out"][exact], col["out"][exact])
    assert col["frame"]["evals"] < full["frame"]["evals"] / 3
    tex.close()


@pytest.mark.parametrize("fname,flt", FILTERS)
@pytest.mark.parametrize("fb", [O.FB_C, O.FB_CPLUS])
@pytest.mark.parametrize("gk,ok,box", [(2, O.LIST, (0, 0)), (3, O.BOX, (0, 0)), (4, O.MASK, (0, 0))])
def test_bicubic_fallback_parity(G, fname, flt, fb, gk, ok, box):
    from test_gpu_filter import compare, run_gpu
    ctf, ctx, _ = G
    pqj, amp = cs.sinusoid_params(64, 8, 8, seed=7)
    tex = ctx.sinusoid_texture(64, pqj, amp)
    otex = O.sinusoid_texture(64, pqj, amp)
    for sname, (uv, duv) in _scenes()[1:]:
        g = run_gpu(G, uv, duv, tex, ctf.method(gk, box=box, fallback=fb, filter=flt), seed=21)
        o = O.filter(uv, duv, otex, O.method(ok, box=box, fallback=fb, filter=flt), seed=21, lists=True,
                     stf=True)
        compare(g, o, f"{fname} fb{fb} {sname}", tol=TOL_CUBIC)
    tex.close()


DEC_METHODS = [("full", 0, O.BILINEAR4, (0, 0), 1), ("stf1", 1, O.STF1, (0, 0), 1),
               ("list_k4", 2, O.LIST, (0, 0), 4), ("list", 2, O.LIST, (0, 0), 1),
               ("box_k4", 3, O.BOX, (0, 0), 4), ("mask_k2", 4, O.MASK, (0, 0), 2)]


@pytest.mark.parametrize("prec", [0, 1])
@pytest.mark.parametrize("fname,flt", FILTERS)
@pytest.mark.parametrize("name,gk,ok,box,k", DEC_METHODS)
def test_bicubic_decoder_parity(G, prec, fname, flt, name, gk, ok, box, k):
    """Decoder producer: the oracle filters the GPU-decoded texel lattice."""
    from test_gpu_decoder import _decoder_case, _lattice_table
    from test_gpu_filter import compare, run_gpu
    ctf, ctx, torch = G
    dec, _ = _decoder_case(ctx)
    tex = ctx.decoder_texture(dec, prec)
    otex = O.table_texture(_lattice_table(tex, 64, torch))
    for sname, (uv, duv) in _scenes():
        g = run_gpu(G, uv, duv, tex, ctf.method(gk, box=box, k=k, filter=flt), seed=29)
        o = O.filter(uv, duv, otex, O.method(ok, box=box, k=k, filter=flt), seed=29, lists=True, stf=True)
        compare(g, o, f"decoder {fname} {name} {sname}", tol=TOL_CUBIC)
    tex.close()
    dec.close()


@pytest.mark.parametrize("fname,flt", FILTERS)
@pytest.mark.parametrize("fb", [O.FB_C, O.FB_CPLUS])
def test_bicubic_decoder_fallback_parity(G, fname, flt, fb):
    from test_gpu_decoder import _decoder_case, _lattice_table
    from test_gpu_filter import compare, run_gpu
    ctf, ctx, torch = G
    dec, _ = _decoder_case(ctx)
    tex = ctx.decoder_texture(dec, 0)
    otex = O.table_texture(_lattice_table(tex, 64, torch))
    for sname, (uv, duv) in _scenes()[1:]:
        for gk, ok in ((2, O.LIST), (4, O.MASK)):
            g = run_gpu(G, uv, duv, tex, ctf.method(gk, fallback=fb, filter=flt), seed=31)
            o = O.filter(uv, duv, otex, O.method(ok, fallback=fb, filter=flt), seed=31, lists=True, stf=True)
            compare(g, o, f"decoder {fname} fb{fb} {gk} {sname}", tol=TOL_CUBIC)
    tex.close()
    dec.close()


@pytest.mark.parametrize("fname,flt", FILTERS)
def test_bicubic_decoder_collaborative_equals_full_bitwise(G, fname, flt):
    from test_gpu_decoder import _decoder_case
    from test_gpu_filter import run_gpu
    ctf, ctx, torch = G
    dec, _ = _decoder_case(ctx)
    tex = ctx.decoder_texture(dec, 0)
    sc = cs.tilted_plane_scene()
    full = run_gpu(G, sc.uv, sc.duv, tex, ctf.method(0, filter=flt))
    col = run_gpu(G, sc.uv, sc.duv, tex, ctf.method(2, k=4, filter=flt))
    exact = col["stf"][..., 0] == np.iinfo(np.int32).min
    assert exact.sum() > 5000
    assert np.array_equal(full["out"][exact], col["out"][exact])
    assert col["frame"]["evals"] < full["frame"]["evals"] / 6
    tex.close()
    dec.close()


@pytest.mark.parametrize("records", [True, False], ids=["records", "no_records"])
@pytest.mark.parametrize("fname,filt", [("bspline", 1), ("catmull_rom", 2)])
@pytest.mark.parametrize("gk,ok,k", [(2, O.LIST, 4), (4, O.MASK, 2), (0, O.BILINEAR4, 1)])
def test_bicubic_layered_launch_matches_oracle_per_layer(G, fname, filt, gk, ok, k, records):
    """The layered launch with the cubic filters: every layer against the
    oracle on its own GPU-decoded lattice and transform."""
    from test_gpu_filter import STAT_FIELDS, _edge_scene
    ctf, ctx, torch = G
    n = 2
    decs = [ctx.decoder(16, 4, 64, 64, cs.decoder_init(16, 4, 64, seed=60 + i, latent_range=0.5)) for i in range(n)]
    texs = [ctx.decoder_texture(d, 0) for d in decs]
    ys, xs = np.mgrid[0:64, 0:64]
    lattice = torch.from_numpy(np.stack([xs.ravel(), ys.ravel()], -1).astype(np.int32)).cuda()
    tables = [t.eval(lattice).cpu().numpy().reshape(64, 64, 4) for t in texs]
    xf = np.array([[[1.3, -0.4], [0.4, 1.3]], [[0.6, 0.2], [-0.2, 0.6]]], np.float32)
    for uv, duv in ((cs.tilted_plane_scene().uv, cs.tilted_plane_scene().duv), _edge_scene()):
        sh, sw = uv.shape[:2]
        tiles = ((sw + 7) // 8) * ((sh + 7) // 8)
        ts = torch.zeros((n, tiles, 128), dtype=torch.uint8, device="cuda")
        sx = torch.full((n, sh, sw, 2), -2**31, dtype=torch.int32, device="cuda")
        fs = ctf.frame_stats_buffer()
        out = ctx.filter_layers(torch.from_numpy(uv).cuda(), torch.from_numpy(duv).cuda(), texs, xf,
                                ctf.method(gk, k=k, filter=filt), seed=9, tile_stats=ts if records else None,
                                frame_stats=fs, stf=sx)
        torch.cuda.synchronize()
        out = out.cpu().numpy()
        evals = 0
        for l in range(n):
            o = O.filter(uv, duv, O.table_texture(tables[l]), O.method(ok, k=k, filter=filt), seed=9, layer=l,
                         xform=xf[l], stf=True)
            if records:
                st = ctf.tile_stats_numpy(ts[l])
                for f in STAT_FIELDS:
                    assert np.array_equal(st[f], o["stats"][f]), (l, f)
            assert np.array_equal(sx[l].cpu().numpy(), o["stf"]), l
            assert np.abs(out[l] - o["out"]).max() <= TOL_CUBIC, l
            evals += int(o["stats"]["evals"].sum())
        assert ctf.frame_stats_dict(fs)["evals"] == evals
    for t in texs:
        t.close()
    for d in decs:
        d.close()
