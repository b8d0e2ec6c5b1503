"""Data-dependent LDS extents of the decoder List kernels on the 4K frames.

The decoder kernels keep a wave's texels in fixed LDS arrays: 256 value
slots, 256 row slots, a 256-entry byte rank table (positions of a 16x16
window) and, for a List wave whose footprints do not fit a 16x16 window, a
sort buffer of F^2 x 64 keys (1024 for the bicubic filters, laid over the
value, row and key arrays).  What goes into them depends on the frame: the
unique texel count n, the row count R = n + (one-tap draws) of a successful
wave, the draws alone of a failed one, and the window positions.  For every
tile of the benchmark's 3840x2160 four-plane frame (seed 1) under List k = 4
with each reconstruction filter, the oracle's tile records give those
quantities (its decisions do not depend on texel values, so a constant
texture stands in for the decoder) and this checks them against the array
sizes, including the bicubic B-spline launch.
"""
import numpy as np
import pytest

import ctf_synth as cs
import oracle as O

MAX_ITEMS = O.MAX_ITEMS   # value and row slots per wave; byte ranks index < 256


def popcount64(a):
    a = np.asarray(a, dtype=np.uint64)
    return np.array([bin(int(v)).count("1") for v in a], dtype=np.int64)


@pytest.fixture(scope="module")
def frame4k():
    return cs.random_planes_scene(3840, 2160, 2048, 2048, seed=1)


@pytest.mark.parametrize("filt,F", [(O.FILTER_BILINEAR, 2), (O.FILTER_BSPLINE, 4), (O.FILTER_CATMULL_ROM, 4)])
def test_list_k4_extents_4k(frame4k, filt, F):
    sc = frame4k
    tex = O.constant_texture(2048, 2048, (0.25, 0.5, 0.75, 1.0))
    o = O.filter_parallel(sc.uv, sc.duv, tex, O.method(O.LIST, k=4, filter=filt), seed=0)
    st = o["stats"]
    nA = popcount64(st["part"])
    nact = popcount64(st["active"])
    ndraw = popcount64(st["stf"])
    n = st["n"].astype(np.int64)
    ok = (st["flags"] & O.TILE_OK) != 0
    assert ok.sum() > 90000 and (nA == 0).sum() > 30000   # collaborative and all-draw waves occur

    # a successful wave: n <= k |A| <= 256 value and row slots, byte ranks
    # 0..n-1, and its rows (unique texels, then the one-tap draws of the
    # lanes outside A) fit the row list
    assert (n[ok] <= 4 * nA[ok]).all()
    assert n[ok].max() <= MAX_ITEMS
    R_ok = n[ok] + ndraw[ok]
    assert R_ok.max() <= MAX_ITEMS
    assert (ndraw[ok] <= nact[ok] - nA[ok]).all()
    # a failed or empty wave decodes its draws only
    assert ndraw[~ok].max() <= 64 and (ndraw[~ok] <= nact[~ok]).all()

    # window positions: 16 (y - ymin) + (x - xmin) < 256 whenever the
    # byte tables are used (the box fits 16x16); larger boxes take the sort
    # buffer of F^2 keys per lane, 64 F^2 in all
    fits = (st["bbw"] <= 16) & (st["bbh"] <= 16) & (nA > 0)
    assert (16 * (st["bbh"][fits].astype(np.int64) - 1) + st["bbw"][fits] - 1 < 256).all()
    sorted_waves = (nA > 0) & ~fits
    assert (F * F * nA[sorted_waves] <= 64 * F * F).all()
    # the unique set of a sorted wave is its compaction: at most F^2 |A| keys
    assert (st["unique"][sorted_waves] <= F * F * nA[sorted_waves]).all()
    print(f"F={F}: tiles {len(st)}, ok {int(ok.sum())}, sorted {int(sorted_waves.sum())}, "
          f"max n {int(n[ok].max())}, max R {int(R_ok.max())}", flush=True)
