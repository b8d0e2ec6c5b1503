"""Multi-layer material filter in one launch (ctf_filter_layers) vs the oracle.

Each layer samples its own decoder at uv_l = M_l uv; the oracle applies the
same float32 transform and filters the layer's GPU-decoded texel lattice.
"""
import math

import numpy as np
import pytest

import ctf_synth as cs
import oracle as O

pytestmark = pytest.mark.gpu

FP16, BF16 = 0, 1


@pytest.fixture(scope="module")
def G():
    import torch
    import paper_2506_17770_amd as ctf
    ctx = ctf.Context(0)
    yield ctf, ctx, torch
    ctx.close()


def _xforms(n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        s = rng.uniform(0.25, 4.0)
        th = rng.uniform(0, 2 * math.pi)
        out.append(s * np.array([[math.cos(th), -math.sin(th)], [math.sin(th), math.cos(th)]]))
    return np.array(out, np.float32)


@pytest.mark.parametrize("records", [True, False], ids=["records", "no_records"])
@pytest.mark.parametrize("prec", [FP16, BF16])
@pytest.mark.parametrize("kind,ok,k", [(2, O.LIST, 4), (3, O.BOX, 1), (0, O.BILINEAR4, 1), (4, O.MASK, 2)])
def test_layers_match_oracle_per_layer(G, prec, kind, ok, k, records):
    """Per layer against the oracle; without per-tile records the kernels
    the benchmark times run (draws, colours and frame counts checked)."""
    from test_gpu_filter import STAT_FIELDS, _edge_scene
    ctf, ctx, torch = G
    n = 3
    decs = [ctx.decoder(16, 4, 64, 64, cs.decoder_init(16, 4, 64, seed=20 + i, latent_range=0.5))
            for i in range(n)]
    texs = [ctx.decoder_texture(d, prec) for d in decs]
    ys, xs = np.mgrid[0:64, 0:64]
    lattice = torch.from_numpy(np.stack([xs.ravel(), ys.ravel()], -1).astype(np.int32)).cuda()
    tables = [t.eval(lattice).cpu().numpy().reshape(64, 64, 4) for t in texs]
    xf = _xforms(n, 5)
    for uv, duv in (cs.tilted_plane_scene().uv, cs.tilted_plane_scene().duv), _edge_scene():
        sh, sw = uv.shape[:2]
        tiles = ((sw + 7) // 8) * ((sh + 7) // 8)
        ts = torch.zeros((n, tiles, 128), dtype=torch.uint8, device="cuda")
        sx = torch.full((n, sh, sw, 2), -2**31, dtype=torch.int32, device="cuda")
        fs = ctf.frame_stats_buffer()
        out = ctx.filter_layers(torch.from_numpy(uv).cuda(), torch.from_numpy(duv).cuda(), texs, xf,
                                ctf.method(kind, k=k), seed=9, tile_stats=ts if records else None,
                                frame_stats=fs, stf=sx)
        torch.cuda.synchronize()
        out = out.cpu().numpy()
        evals = 0
        for l in range(n):
            o = O.filter(uv, duv, O.table_texture(tables[l]), O.method(ok, k=k), seed=9, layer=l,
                         xform=xf[l], stf=True)
            if records:
                st = ctf.tile_stats_numpy(ts[l])
                for f in STAT_FIELDS:
                    assert np.array_equal(st[f], o["stats"][f]), (l, f)
            assert np.array_equal(sx[l].cpu().numpy(), o["stf"]), l
            assert np.abs(out[l] - o["out"]).max() <= 1e-6, l
            evals += int(o["stats"]["evals"].sum())
        assert ctf.frame_stats_dict(fs)["evals"] == evals
    for t in texs:
        t.close()
    for d in decs:
        d.close()


def test_identity_layer_equals_single_filter(G):
    ctf, ctx, torch = G
    dec = ctx.decoder(16, 4, 64, 64, cs.decoder_init(16, 4, 64, seed=1, latent_range=0.5))
    tex = ctx.decoder_texture(dec, FP16)
    sc = cs.tilted_plane_scene()
    uv, duv = torch.from_numpy(sc.uv).cuda(), torch.from_numpy(sc.duv).cuda()
    m = ctf.method(ctf.LIST, k=4)
    single = ctx.filter(uv, duv, tex, m, seed=3)
    layered = ctx.filter_layers(uv, duv, [tex], np.eye(2, dtype=np.float32)[None], m, seed=3)
    torch.cuda.synchronize()
    assert torch.equal(single, layered[0])
    tex.close()
    dec.close()
