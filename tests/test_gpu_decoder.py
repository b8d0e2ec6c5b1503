"""Learned texel producer on the GPU: decode, filter parity, gradients, training.

Decode accuracy is checked against the float64 oracle evaluated on the
same 16-bit parameter values; the filter on the decoder path is checked
against the oracle filtering the GPU-decoded texel lattice (decisions
bit-exact, colours within 1e-6); the hand-written backward pass against
the float64 chain rule and central differences.
"""
import numpy as np
import pytest

import ctf_synth as cs
import oracle as O

pytestmark = pytest.mark.gpu

FP16, BF16 = 0, 1
# unit roundoff of the operand formats
U = {FP16: 2.0 ** -11, BF16: 2.0 ** -8}


@pytest.fixture(scope="module")
def G():
    import torch
    import paper_2506_17770_amd as ctf
    ctx = ctf.Context(0)
    yield ctf, ctx, torch
    ctx.close()


def round_params(p, l0, l1, H, prec):
    """The 16-bit values the kernels read: latents and weights rounded, biases float32."""
    import torch
    lay = cs.decoder_layout(l0, l1, H)
    q = p.astype(np.float64).copy()
    dt = torch.float16 if prec == FP16 else torch.bfloat16
    for name in ("lat0", "lat1", "W1", "W2", "W3"):
        o, n = lay[name]
        q[o:o + n] = torch.from_numpy(p[o:o + n].astype(np.float32)).to(dt).to(torch.float64).numpy()
    return q


def trained_like_params(l0, l1, H, seed):
    """Parameters with the magnitudes of a trained decoder (latents ~0.5)."""
    p = cs.decoder_init(l0, l1, H, seed=seed, latent_range=0.5)
    return p


@pytest.mark.parametrize("prec", [FP16, BF16])
def test_decode_matches_float64(G, prec):
    ctf, ctx, torch = G
    tex_w, l0, l1, H = 2048, 512, 128, 64
    p = trained_like_params(l0, l1, H, seed=3)
    dec = ctx.decoder(l0, l1, H, tex_w, p)
    tex = ctx.decoder_texture(dec, prec)
    rng = np.random.default_rng(1)
    xy = rng.integers(-5000, 5000, (50000, 2)).astype(np.int32)
    got = tex.eval(torch.from_numpy(xy).cuda()).cpu().numpy().astype(np.float64)
    want = O.decoder_texture(tex_w, l0, l1, H, round_params(p, l0, l1, H, prec)).eval(xy)
    err = np.abs(got - want)
    scale = np.abs(want).max()
    # three rounding points (features, two hidden layers) of relative size u,
    # each propagated through 64-wide layers: allow 16 u of the output scale
    assert err.max() <= 16 * U[prec] * max(scale, 1.0), (err.max(), scale)
    tex.close()
    dec.close()


def _decoder_case(ctx, tex_w=64, l0=16, l1=4, H=64, seed=5):
    p = trained_like_params(l0, l1, H, seed)
    return ctx.decoder(l0, l1, H, tex_w, p), p


def _lattice_table(tex, tex_w, torch):
    ys, xs = np.mgrid[0:tex_w, 0:tex_w]
    xy = np.stack([xs.ravel(), ys.ravel()], -1).astype(np.int32)
    return tex.eval(torch.from_numpy(xy).cuda()).cpu().numpy().reshape(tex_w, tex_w, 4)


METHODS = [("bilinear4", 0, O.BILINEAR4, (0, 0), 1), ("stf1", 1, O.STF1, (0, 0), 1),
           ("list_k4", 2, O.LIST, (0, 0), 4), ("list", 2, O.LIST, (0, 0), 1),
           ("box4x4", 3, O.BOX, (4, 4), 1), ("box_k4", 3, O.BOX, (0, 0), 4),
           ("mask", 4, O.MASK, (0, 0), 1), ("mask_k2", 4, O.MASK, (0, 0), 2)]


@pytest.mark.parametrize("prec", [FP16, BF16])
@pytest.mark.parametrize("name,gk,ok,box,k", METHODS)
def test_decoder_filter_parity_tiny(G, prec, name, gk, ok, box, k):
    from test_gpu_filter import compare, run_gpu, _edge_scene
    ctf, ctx, torch = G
    dec, _ = _decoder_case(ctx)
    tex = ctx.decoder_texture(dec, prec)
    table = _lattice_table(tex, 64, torch)
    otex = O.table_texture(table)
    for uv, duv in (_edge_scene(), (cs.tilted_plane_scene().uv, cs.tilted_plane_scene().duv)):
        g = run_gpu(G, uv, duv, tex, ctf.method(gk, box=box, k=k), seed=11)
        o = O.filter(uv, duv, otex, O.method(ok, box=box, k=k), seed=11, lists=True, stf=True)
        compare(g, o, name)
    tex.close()
    dec.close()


def test_collaborative_decode_equals_4tap_bitwise(G):
    from test_gpu_filter import run_gpu
    ctf, ctx, torch = G
    dec, _ = _decoder_case(ctx)
    tex = ctx.decoder_texture(dec, FP16)
    sc = cs.tilted_plane_scene()
    g4 = run_gpu(G, sc.uv, sc.duv, tex, ctf.method(0))
    gl = run_gpu(G, sc.uv, sc.duv, tex, ctf.method(2, k=4))
    exact = gl["stf"][..., 0] == np.iinfo(np.int32).min
    assert np.array_equal(g4["out"][exact], gl["out"][exact])
    assert gl["frame"]["evals"] < g4["frame"]["evals"] / 3
    tex.close()
    dec.close()


@pytest.mark.parametrize("prec", [FP16, BF16])
def test_gradient_small_instance(G, prec):
    """4x4 latent grid, 4-wide MLP: GPU backward vs float64 chain rule and differences."""
    ctf, ctx, torch = G
    tex_w, l0, l1, H = 16, 4, 2, 4
    p = cs.decoder_init(l0, l1, H, seed=1, latent_range=0.5)
    rng = np.random.default_rng(5)
    n = 300
    xy = rng.integers(0, tex_w, (n, 2)).astype(np.int32)
    target = rng.uniform(0, 1, (n, 4)).astype(np.float32)
    dec = ctx.decoder(l0, l1, H, tex_w, p)
    loss, grad = dec.loss_grad(torch.from_numpy(xy).cuda(), torch.from_numpy(target).cuda(), precision=prec)
    loss = float(loss.cpu()[0])
    grad = grad.cpu().numpy().astype(np.float64)
    q = round_params(p, l0, l1, H, prec)
    lref, gref = O.decoder_loss_grad(q, xy, target, l0, l1, H, tex_w)
    # float64 chain rule pinned by central differences
    eps = 1e-6
    for i in rng.choice(q.size, 40, replace=False):
        a = q.copy(); a[i] += eps
        b = q.copy(); b[i] -= eps
        fd = (O.decoder_loss_grad(a, xy, target, l0, l1, H, tex_w, grad=False)[0] -
              O.decoder_loss_grad(b, xy, target, l0, l1, H, tex_w, grad=False)[0]) / (2 * eps)
        assert abs(fd - gref[i]) <= 1e-6 + 1e-5 * abs(gref[i])
    assert abs(loss - lref) <= 8 * U[prec] * lref
    # operand rounding of activations and back-propagated errors (relative u
    # each, a handful of stages): per component within 16 u of the largest
    gmax = np.abs(gref).max()
    err = np.abs(grad - gref)
    assert err.max() <= 16 * U[prec] * gmax, (err.max(), gmax)
    assert np.linalg.norm(grad - gref) <= 4 * U[prec] * np.linalg.norm(gref)
    dec.close()


def test_gradient_full_size_bf16(G):
    ctf, ctx, torch = G
    tex_w, l0, l1, H = 2048, 512, 128, 64
    p = trained_like_params(l0, l1, H, seed=7)
    pqj, amp = cs.sinusoid_params(tex_w, 32, 64, seed=2)
    rng = np.random.default_rng(6)
    n = 2000
    xy = rng.integers(0, tex_w, (n, 2)).astype(np.int32)
    target = O.sinusoid_texture(tex_w, pqj, amp).eval(xy).astype(np.float32)
    dec = ctx.decoder(l0, l1, H, tex_w, p)
    loss, grad = dec.loss_grad(torch.from_numpy(xy).cuda(), torch.from_numpy(target).cuda(), precision=BF16)
    grad = grad.cpu().numpy().astype(np.float64)
    q = round_params(p, l0, l1, H, BF16)
    lref, gref = O.decoder_loss_grad(q, xy, target, l0, l1, H, tex_w)
    assert abs(float(loss.cpu()[0]) - lref) <= 8 * U[BF16] * lref
    # The residual y - t is formed from a forward pass with three bf16
    # roundings, so its relative error is u |y| / |y - t|, larger than u when
    # the fit is close; the back-propagated signals add three more roundings.
    # 16 u in norm per parameter group; a wrong index, sign or transposition
    # gives errors of order 1.
    lay = cs.decoder_layout(l0, l1, H)
    for name in ("lat0", "lat1", "W1", "b1", "W2", "b2", "W3", "b3"):
        o, m = lay[name]
        a, b = grad[o:o + m], gref[o:o + m]
        rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        print(f"full-size bf16 gradient {name}: relative error {rel:.2e} ({rel / U[BF16]:.1f} u)")
        assert rel <= 16 * U[BF16], name
    dec.close()


def test_training_reduces_loss_and_checkpoint_resumes(G):
    ctf, ctx, torch = G
    tex_w, l0, l1, H = 256, 64, 16, 64
    pqj, amp = cs.sinusoid_params(tex_w, 8, 8, seed=4)
    target = ctx.sinusoid_texture(tex_w, pqj, amp)
    p = cs.decoder_init(l0, l1, H, seed=2)
    dec = ctx.decoder(l0, l1, H, tex_w, p)
    trace = torch.zeros(300, device="cuda")
    dec.train(target, 300, batch=4096, lr=1e-2, seed=1, loss_trace=trace)
    torch.cuda.synchronize()
    tr = trace.cpu().numpy()
    assert np.all(np.isfinite(tr))
    assert tr[-20:].mean() < 0.2 * tr[:5].mean(), (tr[:5], tr[-20:])
    # checkpoint / resume: the same steps from a restored state give the
    # same parameters bit for bit (fixed-order MLP reduction, fixed-point
    # latent gradient sums)
    blob = dec.state()
    dec.train(target, 50, batch=4096, lr=1e-2, seed=1)
    a = dec.params()
    dec.set_state(blob)
    dec.train(target, 50, batch=4096, lr=1e-2, seed=1)
    b = dec.params()
    assert np.array_equal(a, b)
    dec.close()
    target.close()


def test_trained_decoder_reaches_40db_against_float64(G):
    """Full training run (20k Adam steps of 65536 texels, bf16): PSNR vs the
    float64 procedural texture on 200k random texels, and the gain over the
    untrained network."""
    ctf, ctx, torch = G
    tex_w, l0, l1, H = 2048, 512, 128, 64
    pqj, amp = cs.sinusoid_params(tex_w, 32, 64, seed=2)
    target = ctx.sinusoid_texture(tex_w, pqj, amp)
    init = cs.decoder_init(l0, l1, H, seed=3)
    dec = ctx.decoder(l0, l1, H, tex_w, init)
    untrained = ctx.decoder_texture(dec, FP16)
    dec.train(target, 20000, batch=65536, lr=1e-3, seed=7, precision=BF16)
    trained = ctx.decoder_texture(dec, FP16)
    rng = np.random.default_rng(9)
    xy = rng.integers(0, tex_w, (200000, 2)).astype(np.int32)
    ref = O.sinusoid_texture(tex_w, pqj, amp).eval(xy)
    xt = torch.from_numpy(xy).cuda()

    def psnr(tex):
        v = tex.eval(xt).cpu().numpy().astype(np.float64)
        return 10 * np.log10(1.0 / np.mean((v - ref) ** 2)), np.abs(v - ref).max()

    p1, m1 = psnr(trained)
    p0, _ = psnr(untrained)
    print(f"decoder PSNR vs float64: trained {p1:.2f} dB (max abs {m1:.4f}), untrained {p0:.2f} dB")
    assert p1 >= 40.0
    assert p1 - p0 >= 15.0
    for t in (trained, untrained, target):
        t.close()
    dec.close()
