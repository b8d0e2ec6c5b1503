"""Collaborative texture filtering on MI355X (gfx950): Python binding.

A thin ctypes layer over ``libctf.so`` (the C ABI declared in
``include/ctf.h``).  It only marshals arguments: every step of the filter
runs in the library's HIP kernels.  Device buffers are torch tensors on a
ROCm device; streams are torch streams.  If the library has not been built
this module raises on import (no CPU fallback exists).

Paper: Akenine-Moller, Ebelin, Pharr, Wronski, "Collaborative Texture
Filtering", HPG 2025 (arXiv 2506.17770).
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libctf.so")

BILINEAR4, STF1, LIST, BOX, MASK = 0, 1, 2, 3, 4
FB_STF1, FB_C, FB_CPLUS = 0, 1, 2
FILTER_BILINEAR, FILTER_BSPLINE, FILTER_CATMULL_ROM = 0, 1, 2
SPLIT_AUTO, SPLIT_OFF = 0, 1
WAVE_8X8, WAVE_8X4 = 0, 1
TEX_SINUSOIDS, TEX_AFFINE, TEX_CONSTANT, TEX_TABLE, TEX_DECODER = 0, 1, 2, 3, 4
FP16, BF16 = 0, 1
TILE_OK, TILE_CAP, TILE_OVERFLOW, TILE_EMPTY = 1, 2, 4, 8
MAX_ITEMS = 256
METHOD_NAMES = {BILINEAR4: "bilinear4", STF1: "stf1", LIST: "list", BOX: "box", MASK: "mask"}

TILE_STATS_DTYPE = np.dtype([
    ("active", "<u8"), ("part", "<u8"), ("stf", "<u8"), ("mask", "<u8", (4,)),
    ("xmin", "<i4"), ("ymin", "<i4"), ("bbw", "<i4"), ("bbh", "<i4"),
    ("n", "<i4"), ("unique", "<i4"), ("evals", "<i4"), ("flags", "<i4"),
    ("reserved", "<i4", (10,))])
FRAME_STATS_FIELDS = ("evals", "active", "stf", "minify", "tiles", "tiles_ok", "tiles_fail", "rows")
FRAME_STATS_WORDS = 16   # ctf_frame_stats: 8 counters + 8 reserved uint64


class CtfError(RuntimeError):
    pass


class TextureDesc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("width", ctypes.c_int32), ("height", ctypes.c_int32),
                ("n_terms", ctypes.c_int32), ("pqj", ctypes.c_void_p), ("amp", ctypes.c_void_p),
                ("affine", (ctypes.c_float * 3) * 4), ("constant", ctypes.c_float * 4),
                ("table", ctypes.c_void_p), ("decoder", ctypes.c_void_p),
                ("precision", ctypes.c_int32), ("reserved_", ctypes.c_int32 * 3)]


class Method(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("box_w", ctypes.c_int32), ("box_h", ctypes.c_int32),
                ("mask_side", ctypes.c_int32), ("max_evals_per_lane", ctypes.c_int32),
                ("fallback", ctypes.c_int32), ("filter", ctypes.c_int32), ("split", ctypes.c_int32),
                ("wave_shape", ctypes.c_int32)]


class DecoderDesc(ctypes.Structure):
    _fields_ = [("l0", ctypes.c_int32), ("l1", ctypes.c_int32), ("hidden", ctypes.c_int32),
                ("channels", ctypes.c_int32), ("tex_w", ctypes.c_int32),
                ("reserved_", ctypes.c_int32 * 3)]


# every entry point of include/ctf.h: name -> (restype, argtypes)
_P = ctypes.c_void_p
_I32, _I64, _U64, _SZ, _F = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_size_t, ctypes.c_float
SIGNATURES = {
    "ctf_last_error": (ctypes.c_char_p, []),
    "ctf_create": (_I32, [ctypes.c_int, _P]),
    "ctf_destroy": (_I32, [_P]),
    "ctf_texture_create": (_I32, [_P, _P, _P]),
    "ctf_texture_destroy": (_I32, [_P]),
    "ctf_texture_eval": (_I32, [_P, _P, _I64, _P, _P]),
    "ctf_filter": (_I32, [_P, _P, _P, _I32, _I32, _P, _P, _U64, _P, _P, _P, _P, _P, _P]),
    "ctf_filter_layers": (_I32, [_P, _P, _P, _I32, _I32, _I32, _P, _P, _P, _U64, _P, _P, _P, _P, _P]),
    "ctf_decoder_param_count": (_SZ, [_P]),
    "ctf_decoder_create": (_I32, [_P, _P, _P, _P]),
    "ctf_decoder_destroy": (_I32, [_P]),
    "ctf_decoder_get_params": (_I32, [_P, _P, _SZ]),
    "ctf_decoder_set_params": (_I32, [_P, _P, _SZ]),
    "ctf_decoder_state_bytes": (_SZ, [_P]),
    "ctf_decoder_get_state": (_I32, [_P, _P, _SZ]),
    "ctf_decoder_set_state": (_I32, [_P, _P, _SZ]),
    "ctf_decoder_loss_grad": (_I32, [_P, _P, _P, _I32, _I32, _P, _P, _P]),
    "ctf_decoder_loss_grad_noalloc": (_I32, [_P, _P, _P, _I32, _I32, _P, _P, _P]),
    "ctf_decoder_train": (_I32, [_P, _P, _I64, _I32, _F, _U64, _I32, _P, _P]),
}


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with "
                          "`python paper_2506_17770_amd/build.py` (no CPU fallback exists)")
    L = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    return L


lib = _load()


def _check(rc):
    if rc != 0:
        raise CtfError(f"ctf error {rc}: {lib.ctf_last_error().decode()}")


def _dptr(t) -> Optional[int]:
    """Device pointer of a torch tensor (None passes NULL)."""
    if t is None:
        return None
    if not t.is_cuda:
        raise CtfError("expected a tensor in GPU memory")
    if not t.is_contiguous():
        raise CtfError("expected a contiguous tensor")
    return t.data_ptr()


def _buf(t, name: str, dtype, numel: int, device: int) -> Optional[int]:
    """Device pointer of a caller buffer after checking what the library will
    read or write through it: a contiguous tensor on the context's device,
    of ``dtype`` (None: any dtype, counted in bytes), holding at least
    ``numel`` elements (bytes when dtype is None).  None passes NULL."""
    if t is None:
        return None
    if not getattr(t, "is_cuda", False):
        raise CtfError(f"{name}: expected a tensor in GPU memory")
    if t.device.index != device:
        raise CtfError(f"{name}: tensor on cuda:{t.device.index}, the context is on cuda:{device}")
    if not t.is_contiguous():
        raise CtfError(f"{name}: expected a contiguous tensor")
    if dtype is not None and t.dtype != dtype:
        raise CtfError(f"{name}: dtype {t.dtype}, expected {dtype}")
    have = t.numel() if dtype is not None else t.numel() * t.element_size()
    if have < numel:
        unit = "elements" if dtype is not None else "bytes"
        raise CtfError(f"{name}: {have} {unit}, the call needs {numel}")
    return t.data_ptr()


def tile_height(meth: Optional[Method]) -> int:
    """Pixel rows per tile record: 4 for the paper's 8x4 waves, else 8."""
    return 4 if meth is not None and meth.wave_shape == WAVE_8X4 else 8


def n_tiles(sw: int, sh: int, meth: Optional[Method] = None) -> int:
    th = tile_height(meth)
    return ((sw + 7) // 8) * ((sh + th - 1) // th)


def _stream(stream) -> Optional[int]:
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def method(kind, box=(0, 0), mask_side=16, k=1, fallback=FB_STF1, filter=FILTER_BILINEAR,
           split=SPLIT_AUTO, wave_shape=WAVE_8X8) -> Method:
    return Method(kind, box[0], box[1], mask_side, k, fallback, filter, split, wave_shape)


class Context:
    """A library context on one GPU (owns its textures and decoders)."""

    def __init__(self, device: int = 0):
        h = ctypes.c_void_p()
        _check(lib.ctf_create(device, ctypes.byref(h)))
        self.handle = h
        self.device = device

    def close(self):
        if self.handle:
            _check(lib.ctf_destroy(self.handle))
            self.handle = None

    # -- textures -----------------------------------------------------------
    def _texture(self, desc: TextureDesc, keep=()):
        h = ctypes.c_void_p()
        _check(lib.ctf_texture_create(self.handle, ctypes.byref(desc), ctypes.byref(h)))
        return Texture(self, h, desc.kind, desc.width, desc.height)

    def sinusoid_texture(self, width, pqj, amp):
        pqj = np.ascontiguousarray(pqj, dtype=np.int32)
        amp = np.ascontiguousarray(amp, dtype=np.float32)
        d = TextureDesc()
        d.kind, d.width, d.height, d.n_terms = TEX_SINUSOIDS, width, width, pqj.shape[1]
        d.pqj, d.amp = pqj.ctypes.data, amp.ctypes.data
        return self._texture(d, (pqj, amp))

    def affine_texture(self, width, height, coef):
        d = TextureDesc()
        d.kind, d.width, d.height = TEX_AFFINE, width, height
        coef = np.asarray(coef, dtype=np.float64).reshape(4, 3)
        for c in range(4):
            for j in range(3):
                d.affine[c][j] = float(coef[c, j])
        return self._texture(d)

    def constant_texture(self, width, height, rgba):
        d = TextureDesc()
        d.kind, d.width, d.height = TEX_CONSTANT, width, height
        for c in range(4):
            d.constant[c] = float(rgba[c])
        return self._texture(d)

    def table_texture(self, table):
        table = np.ascontiguousarray(table, dtype=np.float32)
        h, w, _ = table.shape
        d = TextureDesc()
        d.kind, d.width, d.height = TEX_TABLE, w, h
        d.table = table.ctypes.data
        return self._texture(d, (table,))

    def decoder_texture(self, decoder: "Decoder", precision=FP16):
        d = TextureDesc()
        d.kind, d.width, d.height = TEX_DECODER, decoder.tex_w, decoder.tex_w
        d.decoder, d.precision = decoder.handle.value, precision
        return self._texture(d)

    # -- filtering ----------------------------------------------------------
    def filter(self, uv, duv, tex: "Texture", meth: Method, seed=0, out=None, tile_stats=None,
               frame_stats=None, lists=None, stf=None, stream=None):
        """ctf_filter on torch tensors; optional outputs are tensors or None."""
        import torch
        if uv.dim() != 3 or uv.shape[-1] != 2:
            raise CtfError("uv must be [H][W][2]")
        sh, sw = uv.shape[:2]
        if tuple(duv.shape) != (sh, sw, 4):
            raise CtfError("uv must be [H][W][2] and duv [H][W][4]")
        if out is None:
            out = torch.empty((sh, sw, 4), dtype=torch.float32, device=uv.device)
        dev, npx, nt = self.device, sh * sw, n_tiles(sw, sh, meth)
        f32, i32 = torch.float32, torch.int32
        args = (_buf(uv, "uv", f32, npx * 2, dev), _buf(duv, "duv", f32, npx * 4, dev), sw, sh, tex.handle,
                ctypes.byref(meth), seed & (2**64 - 1), _buf(out, "out", f32, npx * 4, dev),
                _buf(tile_stats, "tile_stats", None, nt * TILE_STATS_DTYPE.itemsize, dev),
                _buf(frame_stats, "frame_stats", torch.int64, FRAME_STATS_WORDS, dev),
                _buf(lists, "lists", i32, nt * MAX_ITEMS * 2, dev), _buf(stf, "stf", i32, npx * 2, dev))
        _check(lib.ctf_filter(self.handle, *args, _stream(stream)))
        return out

    def filter_layers(self, uv, duv, texs, xforms, meth: Method, seed=0, out=None, tile_stats=None,
                      frame_stats=None, stf=None, stream=None):
        """ctf_filter_layers: one launch over len(texs) material layers.

        xforms: [L][2][2] (layer uv = M uv); out: [L][H][W][4]."""
        import torch
        if uv.dim() != 3 or uv.shape[-1] != 2:
            raise CtfError("uv must be [H][W][2]")
        sh, sw = uv.shape[:2]
        if tuple(duv.shape) != (sh, sw, 4):
            raise CtfError("uv must be [H][W][2] and duv [H][W][4]")
        n = len(texs)
        xf = np.ascontiguousarray(np.asarray(xforms, dtype=np.float32).reshape(n, 4))
        handles = (ctypes.c_void_p * n)(*[t.handle.value for t in texs])
        if out is None:
            out = torch.empty((n, sh, sw, 4), dtype=torch.float32, device=uv.device)
        dev, npx, nt = self.device, sh * sw, n_tiles(sw, sh, meth)
        f32, i32 = torch.float32, torch.int32
        args = (_buf(uv, "uv", f32, npx * 2, dev), _buf(duv, "duv", f32, npx * 4, dev), sw, sh, n, handles,
                xf.ctypes.data, ctypes.byref(meth), seed & (2**64 - 1), _buf(out, "out", f32, n * npx * 4, dev),
                _buf(tile_stats, "tile_stats", None, n * nt * TILE_STATS_DTYPE.itemsize, dev),
                _buf(frame_stats, "frame_stats", torch.int64, FRAME_STATS_WORDS, dev),
                _buf(stf, "stf", i32, n * npx * 2, dev))
        _check(lib.ctf_filter_layers(self.handle, *args, _stream(stream)))
        return out

    def decoder(self, l0, l1, hidden, tex_w, init, channels=8) -> "Decoder":
        return Decoder(self, l0, l1, hidden, tex_w, init, channels)


class Texture:
    def __init__(self, ctx: Context, handle, kind, width, height):
        self.ctx, self.handle, self.kind, self.width, self.height = ctx, handle, kind, width, height

    def eval(self, xy, out=None, stream=None):
        """Texel values rgba[i] = f(xy[i]); xy int32 [n][2] on the GPU."""
        import torch
        if xy.dim() != 2 or xy.shape[1] != 2:
            raise CtfError("xy must be [n][2]")
        n = xy.shape[0]
        if out is None:
            out = torch.empty((n, 4), dtype=torch.float32, device=xy.device)
        dev = self.ctx.device
        _check(lib.ctf_texture_eval(self.handle, _buf(xy, "xy", torch.int32, n * 2, dev), n,
                                    _buf(out, "out", torch.float32, n * 4, dev), _stream(stream)))
        return out

    def close(self):
        if self.handle:
            _check(lib.ctf_texture_destroy(self.handle))
            self.handle = None


class Decoder:
    """Latent-grid + MLP texel decoder with float32 master parameters."""

    def __init__(self, ctx: Context, l0, l1, hidden, tex_w, init, channels=8):
        self.ctx = ctx
        self.desc = DecoderDesc(l0, l1, hidden, channels, tex_w)
        self.tex_w = tex_w
        self.count = lib.ctf_decoder_param_count(ctypes.byref(self.desc))
        init = np.ascontiguousarray(init, dtype=np.float32)
        if init.size != self.count:
            raise CtfError(f"init has {init.size} values, decoder needs {self.count}")
        h = ctypes.c_void_p()
        _check(lib.ctf_decoder_create(ctx.handle, ctypes.byref(self.desc), init.ctypes.data,
                                      ctypes.byref(h)))
        self.handle = h

    def params(self) -> np.ndarray:
        out = np.empty(self.count, np.float32)
        _check(lib.ctf_decoder_get_params(self.handle, out.ctypes.data, self.count))
        return out

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        _check(lib.ctf_decoder_set_params(self.handle, p.ctypes.data, p.size))

    def state(self) -> bytes:
        n = lib.ctf_decoder_state_bytes(self.handle)
        buf = ctypes.create_string_buffer(n)
        _check(lib.ctf_decoder_get_state(self.handle, buf, n))
        return buf.raw

    def set_state(self, blob: bytes):
        _check(lib.ctf_decoder_set_state(self.handle, blob, len(blob)))

    def loss_grad(self, xy, target, precision=BF16, stream=None):
        import torch
        if xy.dim() != 2 or xy.shape[1] != 2:
            raise CtfError("xy must be [n][2]")
        n, dev = xy.shape[0], self.ctx.device
        loss = torch.zeros(1, dtype=torch.float32, device=xy.device)
        grad = torch.zeros(self.count, dtype=torch.float32, device=xy.device)
        _check(lib.ctf_decoder_loss_grad(self.handle, _buf(xy, "xy", torch.int32, n * 2, dev),
                                         _buf(target, "target", torch.float32, n * 4, dev), n,
                                         precision, _dptr(loss), _dptr(grad), _stream(stream)))
        return loss, grad

    def loss_grad_noalloc(self, xy, target, loss, grad, precision=BF16, stream=None):
        """ctf_decoder_loss_grad_noalloc: the caller provides loss (float32 [1])
        and grad (float32 [param_count]); the library allocates nothing."""
        import torch
        if xy.dim() != 2 or xy.shape[1] != 2:
            raise CtfError("xy must be [n][2]")
        n, dev = xy.shape[0], self.ctx.device
        _check(lib.ctf_decoder_loss_grad_noalloc(
            self.handle, _buf(xy, "xy", torch.int32, n * 2, dev), _buf(target, "target", torch.float32, n * 4, dev),
            n, precision, _buf(loss, "loss", torch.float32, 1, dev), _buf(grad, "grad", torch.float32, self.count, dev),
            _stream(stream)))

    def train(self, target: Texture, steps, batch=65536, lr=1e-3, seed=0, precision=BF16,
              loss_trace=None, stream=None):
        import torch
        trace = _buf(loss_trace, "loss_trace", torch.float32, max(0, steps), self.ctx.device)
        _check(lib.ctf_decoder_train(self.handle, target.handle, steps, batch, lr,
                                     seed & (2**64 - 1), precision, trace, _stream(stream)))

    def close(self):
        if self.handle:
            _check(lib.ctf_decoder_destroy(self.handle))
            self.handle = None


def tile_stats_buffer(sw, sh, device="cuda", tile_h=None, meth: Optional[Method] = None, layers=1):
    """Zeroed tile records for a frame: the tile height follows the method's
    wave shape (8x4 waves write twice the tile rows of 8x8 waves)."""
    import torch
    th = tile_h if tile_h is not None else tile_height(meth)
    tiles = ((sw + 7) // 8) * ((sh + th - 1) // th)
    return torch.zeros((layers * tiles, TILE_STATS_DTYPE.itemsize), dtype=torch.uint8, device=device)


def frame_stats_buffer(device="cuda"):
    import torch
    return torch.zeros(FRAME_STATS_WORDS, dtype=torch.int64, device=device)


def tile_stats_numpy(buf) -> np.ndarray:
    return buf.cpu().numpy().view(TILE_STATS_DTYPE).reshape(-1)


def frame_stats_dict(buf) -> dict:
    v = buf.cpu().numpy().astype(np.int64)
    return {k: int(v[i]) for i, k in enumerate(FRAME_STATS_FIELDS)}


def lists_buffer(sw, sh, device="cuda", tile_h=None, meth: Optional[Method] = None):
    import torch
    th = tile_h if tile_h is not None else tile_height(meth)
    tiles = ((sw + 7) // 8) * ((sh + th - 1) // th)
    return torch.full((tiles, MAX_ITEMS, 2), -2**31, dtype=torch.int32, device=device)


def stf_buffer(sw, sh, device="cuda"):
    import torch
    return torch.full((sh, sw, 2), -2**31, dtype=torch.int32, device=device)
