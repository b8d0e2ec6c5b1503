"""CPU oracle for collaborative texture filtering -- TEST INFRASTRUCTURE ONLY.

Python access to ``libctf_oracle.so`` (plain C, ``ctf_oracle.c``).  Only the
test-suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package; the HIP library never does, and this
package never imports the HIP library.

Paper: "Collaborative Texture Filtering" (Akenine-Moller et al., HPG 2025).
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "ctf_oracle.c")
LIB_PATH = os.path.join(HERE, "libctf_oracle.so")

BILINEAR4, STF1, LIST, BOX, MASK = 0, 1, 2, 3, 4
FB_STF1, FB_C, FB_CPLUS = 0, 1, 2
FILTER_BILINEAR, FILTER_BSPLINE, FILTER_CATMULL_ROM = 0, 1, 2
TEX_SINUSOIDS, TEX_AFFINE, TEX_CONSTANT, TEX_TABLE, TEX_DECODER = 0, 1, 2, 3, 4
TILE_OK, TILE_CAP, TILE_OVERFLOW, TILE_EMPTY = 1, 2, 4, 8
MAX_ITEMS = 256
MAX_FB_ITEMS = 128


def build() -> str:
    """Compile the oracle with gcc (no contraction of a*b+c into fma)."""
    tmp = LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off",
                           "-fno-fast-math", "-Wall", "-fPIC", "-shared",
                           "-o", tmp, SRC, "-lm"])
    os.replace(tmp, LIB_PATH)
    return LIB_PATH


class Decoder(ctypes.Structure):
    _fields_ = [("l0", ctypes.c_int32), ("l1", ctypes.c_int32),
                ("hidden", ctypes.c_int32), ("channels", ctypes.c_int32),
                ("tex_w", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("params", ctypes.POINTER(ctypes.c_double))]


class Texture(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("width", ctypes.c_int32),
                ("height", ctypes.c_int32), ("n_terms", ctypes.c_int32),
                ("pqj", ctypes.POINTER(ctypes.c_int32)),
                ("amp", ctypes.POINTER(ctypes.c_float)),
                ("affine", (ctypes.c_double * 3) * 4),
                ("constant", ctypes.c_double * 4),
                ("table", ctypes.POINTER(ctypes.c_float)),
                ("dec", ctypes.POINTER(Decoder))]


class Method(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("box_w", ctypes.c_int32),
                ("box_h", ctypes.c_int32), ("mask_side", ctypes.c_int32),
                ("max_evals_per_lane", ctypes.c_int32), ("fallback", ctypes.c_int32),
                ("filter", ctypes.c_int32)]


TILE_STATS_DTYPE = np.dtype([
    ("active", "<u8"), ("part", "<u8"), ("stf", "<u8"), ("mask", "<u8", (4,)),
    ("xmin", "<i4"), ("ymin", "<i4"), ("bbw", "<i4"), ("bbh", "<i4"),
    ("n", "<i4"), ("unique", "<i4"), ("evals", "<i4"), ("flags", "<i4"),
    ("reserved", "<i4", (10,))])
assert TILE_STATS_DTYPE.itemsize == 128

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH) or os.path.getmtime(LIB_PATH) < os.path.getmtime(SRC):
            build()
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        L.ctfo_pcg_hash.argtypes = [ctypes.c_uint32]
        L.ctfo_pcg_hash.restype = ctypes.c_uint32
        L.ctfo_bit_select.argtypes = [P, ctypes.c_int32]
        L.ctfo_bit_rank.argtypes = [P, ctypes.c_int32]
        L.ctfo_texel_eval.argtypes = [ctypes.POINTER(Texture), P, ctypes.c_int64, P]
        L.ctfo_filter.argtypes = [P, P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                  ctypes.c_int32, ctypes.POINTER(Texture),
                                  ctypes.POINTER(Method), ctypes.c_uint64, ctypes.c_int32,
                                  P, P, P, P, P, P, ctypes.c_int64, ctypes.c_int64]
        L.ctfo_cplus_target.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]
        L.ctfo_decoder_loss_grad.argtypes = [ctypes.POINTER(Decoder), P, P, ctypes.c_int64,
                                             P, P]
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


# ---------------------------------------------------------------------------
# small helpers
# ---------------------------------------------------------------------------

def pcg_hash(v: int) -> int:
    return lib().ctfo_pcg_hash(v & 0xFFFFFFFF)


def _mask4(B) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(B, dtype=np.uint64).reshape(4))


def cplus_target(nA: int, ns: int, c: int) -> int:
    """Eq. 2: rank of the lane whose footprint spare lane c draws from."""
    return lib().ctfo_cplus_target(nA, ns, c)


def bit_select(B, i: int) -> int:
    """h(i, B): position of the i-th set bit of the 256-bit mask B (words low first)."""
    return lib().ctfo_bit_select(_ptr(_mask4(B)), i)


def bit_rank(B, t: int) -> int:
    """h^-1(t, B): number of set bits of B below position t."""
    return lib().ctfo_bit_rank(_ptr(_mask4(B)), t)


# ---------------------------------------------------------------------------
# textures
# ---------------------------------------------------------------------------

class OracleTexture:
    """Holds a ``Texture`` struct and keeps its arrays alive."""

    def __init__(self, kind, width, height, **kw):
        self._keep = []
        t = Texture()
        t.kind, t.width, t.height = kind, width, height
        if kind == TEX_SINUSOIDS:
            pqj = np.ascontiguousarray(kw["pqj"], dtype=np.int32)
            amp = np.ascontiguousarray(kw["amp"], dtype=np.float32)
            t.n_terms = pqj.shape[1]
            t.pqj = pqj.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
            t.amp = amp.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
            self._keep += [pqj, amp]
        elif kind == TEX_AFFINE:
            coef = np.asarray(kw["coef"], dtype=np.float64).reshape(4, 3)
            for c in range(4):
                for j in range(3):
                    t.affine[c][j] = float(coef[c, j])
        elif kind == TEX_CONSTANT:
            for c in range(4):
                t.constant[c] = float(kw["rgba"][c])
        elif kind == TEX_TABLE:
            tab = np.ascontiguousarray(kw["table"], dtype=np.float32)
            assert tab.shape == (height, width, 4)
            t.table = tab.ctypes.data_as(ctypes.POINTER(ctypes.c_float))
            self._keep.append(tab)
        elif kind == TEX_DECODER:
            params = np.ascontiguousarray(kw["params"], dtype=np.float64)
            d = Decoder(kw["l0"], kw["l1"], kw["hidden"], kw.get("channels", 8), width, 0,
                        params.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
            self._keep += [params, d]
            t.dec = ctypes.pointer(d)
        else:
            raise ValueError(kind)
        self.struct = t

    def eval(self, xy) -> np.ndarray:
        xy = np.ascontiguousarray(xy, dtype=np.int32).reshape(-1, 2)
        out = np.empty((xy.shape[0], 4), np.float64)
        rc = lib().ctfo_texel_eval(ctypes.byref(self.struct), _ptr(xy), xy.shape[0], _ptr(out))
        if rc:
            raise RuntimeError("ctfo_texel_eval failed")
        return out


def sinusoid_texture(width, pqj, amp):
    return OracleTexture(TEX_SINUSOIDS, width, width, pqj=pqj, amp=amp)


def affine_texture(width, height, coef):
    return OracleTexture(TEX_AFFINE, width, height, coef=coef)


def constant_texture(width, height, rgba):
    return OracleTexture(TEX_CONSTANT, width, height, rgba=rgba)


def table_texture(table):
    h, w, _ = table.shape
    return OracleTexture(TEX_TABLE, w, h, table=table)


def decoder_texture(tex_w, l0, l1, hidden, params, channels=8):
    return OracleTexture(TEX_DECODER, tex_w, tex_w, l0=l0, l1=l1, hidden=hidden,
                         params=params, channels=channels)


# ---------------------------------------------------------------------------
# filter
# ---------------------------------------------------------------------------

def method(kind, box=(0, 0), mask_side=16, k=1, fallback=FB_STF1, filter=FILTER_BILINEAR) -> Method:
    return Method(kind, box[0], box[1], mask_side, k, fallback, filter)


def filter(uv, duv, tex: OracleTexture, meth: Method, seed=0, layer=0, tile=(8, 8),
           tiles=None, stats=True, lists=False, stf=False, xform=None, fb_items=False, into=None):
    """Run the oracle filter.  Returns dict(out f64 [H][W][4], stats, lists, stf, fb_items).

    ``tiles`` = (begin, end) restricts the work to a tile range (the other
    pixels of ``out`` are left zero).  ``xform`` = 2x2 matrix of a material
    layer applied (in float32) to uv and its derivatives.  ``fb_items``:
    return, per tile, the texels fallback C or C+ produced as rows
    (x, y, rank in A of the producing lane), padded with INT32_MIN.
    """
    xf = None if xform is None else np.ascontiguousarray(np.asarray(xform, np.float32).reshape(4))
    uv = np.ascontiguousarray(uv, dtype=np.float32)
    duv = np.ascontiguousarray(duv, dtype=np.float32)
    sh, sw = uv.shape[:2]
    tw, th = tile
    ntiles = ((sw + tw - 1) // tw) * ((sh + th - 1) // th)
    # preallocated outputs (filter_parallel): each call writes only its tiles
    out = into["out"] if into else np.zeros((sh, sw, 4), np.float64)
    st = (into["stats"] if into else np.zeros(ntiles, TILE_STATS_DTYPE)) if stats else None
    li = np.full((ntiles, MAX_ITEMS, 2), np.iinfo(np.int32).min, np.int32) if lists else None
    sx = (into["stf"] if into else np.full((sh, sw, 2), np.iinfo(np.int32).min, np.int32)) if stf else None
    fi = np.full((ntiles, MAX_FB_ITEMS, 3), np.iinfo(np.int32).min, np.int32) if fb_items else None
    b, e = tiles if tiles is not None else (0, ntiles)
    rc = lib().ctfo_filter(_ptr(uv), _ptr(duv), sw, sh, tw, th, ctypes.byref(tex.struct),
                           ctypes.byref(meth), seed & (2**64 - 1), layer, _ptr(xf), _ptr(out), _ptr(st),
                           _ptr(li), _ptr(sx), _ptr(fi), b, e)
    if rc:
        raise RuntimeError(f"ctfo_filter failed ({rc})")
    return dict(out=out, stats=st, lists=li, stf=sx, fb_items=fi)


def filter_parallel(uv, duv, tex: OracleTexture, meth: Method, seed=0, layer=0, tile=(8, 8),
                    stf=True, xform=None, threads=None):
    """The whole frame through ``filter`` on several host threads, each on a
    contiguous range of tiles (the C oracle releases the GIL; tiles are
    independent).  Returns dict(out, stats, stf) as ``filter`` does."""
    import threading
    sh, sw = np.asarray(uv).shape[:2]
    tw, th = tile
    ntiles = ((sw + tw - 1) // tw) * ((sh + th - 1) // th)
    into = {"out": np.zeros((sh, sw, 4), np.float64), "stats": np.zeros(ntiles, TILE_STATS_DTYPE),
            "stf": np.full((sh, sw, 2), np.iinfo(np.int32).min, np.int32)}
    uv = np.ascontiguousarray(uv, dtype=np.float32)
    duv = np.ascontiguousarray(duv, dtype=np.float32)
    n = max(1, min(threads or os.cpu_count() or 1, 16, ntiles))
    bounds = np.linspace(0, ntiles, n + 1).astype(np.int64)
    errs = []

    def work(b, e):
        try:
            filter(uv, duv, tex, meth, seed=seed, layer=layer, tile=tile, tiles=(int(b), int(e)), stats=True,
                   stf=stf, xform=xform, into=into)
        except Exception as ex:   # surfaced below
            errs.append(ex)

    ths = [threading.Thread(target=work, args=(bounds[i], bounds[i + 1])) for i in range(n)]
    for t in ths:
        t.start()
    for t in ths:
        t.join()
    if errs:
        raise errs[0]
    return dict(out=into["out"], stats=into["stats"], stf=into["stf"] if stf else None)


def decoder_loss_grad(params, xy, target, l0, l1, hidden, tex_w, channels=8, grad=True):
    """float64 MSE loss and its gradient w.r.t. the flat parameter vector."""
    params = np.ascontiguousarray(params, dtype=np.float64)
    xy = np.ascontiguousarray(xy, dtype=np.int32).reshape(-1, 2)
    target = np.ascontiguousarray(target, dtype=np.float32).reshape(-1, 4)
    d = Decoder(l0, l1, hidden, channels, tex_w, 0,
                params.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    loss = np.zeros(1, np.float64)
    g = np.zeros(params.size, np.float64) if grad else None
    rc = lib().ctfo_decoder_loss_grad(ctypes.byref(d), _ptr(xy), _ptr(target), xy.shape[0],
                                      _ptr(loss), _ptr(g))
    if rc:
        raise RuntimeError("ctfo_decoder_loss_grad failed")
    return float(loss[0]), g
