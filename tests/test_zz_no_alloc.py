"""The allocation-free loss/gradient entry point (ctf_decoder_loss_grad_noalloc).

It runs the same kernels as ctf_decoder_loss_grad with the library's fixed
per-device scratch array instead of the decoder's batch buffers, so its
loss and gradient must equal that call's bit for bit.  Two calls in a row
(the largest batch the array takes, then a smaller one) check that nothing
carries over from one call to the next; the device's free memory is the
same before and after them.
"""
import numpy as np
import pytest

import ctf_synth as cs

pytestmark = pytest.mark.gpu

FP16, BF16 = 0, 1


@pytest.mark.parametrize("prec", [BF16, FP16])
def test_noalloc_loss_grad_matches_the_allocating_call(prec):
    import torch
    import paper_2506_17770_amd as ctf
    print(f"case noalloc loss/grad precision {prec}", flush=True)
    ctx = ctf.Context(0)
    tex_w, l0, l1, H = 2048, 512, 128, 64
    dec = ctx.decoder(l0, l1, H, tex_w, cs.decoder_init(l0, l1, H, seed=11, latent_range=0.5))
    rng = np.random.default_rng(21 + prec)
    nmax = 16384
    sizes = (nmax, 3000)
    xys = [torch.from_numpy(rng.integers(-4096, 4096, (n, 2)).astype(np.int32)).cuda() for n in sizes]
    tgts = [torch.from_numpy(rng.uniform(0, 1, (n, 4)).astype(np.float32)).cuda() for n in sizes]
    outs = [(torch.zeros(1, dtype=torch.float32, device="cuda"),
             torch.zeros(dec.count, dtype=torch.float32, device="cuda")) for _ in sizes]
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    for xy, tg, (loss, grad) in zip(xys, tgts, outs):
        dec.loss_grad_noalloc(xy, tg, loss, grad, precision=prec)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    assert free1 == free0, (free0, free1)
    for i, (xy, tg, (loss, grad)) in enumerate(zip(xys, tgts, outs)):
        lref, gref = dec.loss_grad(xy, tg, precision=prec)
        torch.cuda.synchronize()
        a, b = grad.cpu().numpy(), gref.cpu().numpy()
        assert np.isfinite(a).all() and np.abs(a).max() > 0
        assert float(loss.cpu()[0]) == float(lref.cpu()[0]), f"call {i}: loss differs"
        assert np.array_equal(a, b), f"call {i}: gradient differs (max {np.abs(a - b).max():.3e})"
    # a batch past the array's size is refused before any device work
    big = torch.zeros((nmax + 1, 2), dtype=torch.int32, device="cuda")
    with pytest.raises(ctf.CtfError):
        dec.loss_grad_noalloc(big, torch.zeros((nmax + 1, 4), dtype=torch.float32, device="cuda"),
                              outs[0][0], outs[0][1], precision=prec)
    dec.close()
    ctx.close()
