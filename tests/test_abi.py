"""The C-ABI library loads and exports every entry point include/ctf.h declares.

No compute call is made: this runs without a GPU.
"""
import ctypes
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "ctf.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?\w+\s*\*?\s*(ctf_\w+)\s*\(", src, flags=re.M)))


def test_header_declares_the_filter_and_setup_calls():
    names = declared_functions()
    for must in ("ctf_filter", "ctf_texture_create", "ctf_texture_eval", "ctf_decoder_create",
                 "ctf_decoder_train", "ctf_decoder_loss_grad", "ctf_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_2506_17770_amd as ctf
    lib = ctypes.CDLL(ctf.LIB_PATH)
    names = declared_functions()
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    # the binding declares a signature for every entry point
    assert set(names) == set(ctf.SIGNATURES), set(names) ^ set(ctf.SIGNATURES)


def test_no_device_gives_a_clean_error_or_a_context():
    import paper_2506_17770_amd as ctf
    try:
        import torch
        has_gpu = torch.cuda.is_available()
    except Exception:
        has_gpu = False
    if has_gpu:
        return
    h = ctypes.c_void_p()
    rc = ctf.lib.ctf_create(0, ctypes.byref(h))
    assert rc != 0
    assert ctf.lib.ctf_last_error()


def test_decoder_create_validates_sizes_before_the_device():
    """Argument checks of ctf_decoder_create return before any device work
    (a dummy context handle is never dereferenced on these paths)."""
    import numpy as np
    import paper_2506_17770_amd as ctf
    dummy_ctx = ctypes.c_void_p(1)
    init = np.zeros(4, np.float32)
    h = ctypes.c_void_p()
    cases = [((16384, 4, 64, 8, 16384), 2),   # latent sides above 8192 (32-bit offsets)
             ((512, 128, 64, 4, 2048), 2),    # channels must be 8
             ((512, 128, 62, 8, 2048), 2),    # hidden must be a multiple of 4
             ((500, 128, 64, 8, 2048), 1),    # sides must be powers of two
             ((4096, 128, 64, 8, 2048), 1)]   # l0 above tex_w
    for fields, want in cases:
        d = ctf.DecoderDesc(*fields)
        st = ctf.lib.ctf_decoder_create(dummy_ctx, ctypes.byref(d), init.ctypes.data, ctypes.byref(h))
        assert st == want, (fields, st, ctf.lib.ctf_last_error())
        assert ctf.lib.ctf_last_error()


def test_filter_validates_screen_sides_before_the_device():
    """Screen sides outside 1..2^24 are rejected before the context, the
    texture or any buffer is touched (dummy handles and pointers)."""
    import paper_2506_17770_amd as ctf
    dummy = ctypes.c_void_p(1)
    m = ctf.method(ctf.LIST)
    xf = (ctypes.c_float * 4)(1, 0, 0, 1)
    texs = (ctypes.c_void_p * 1)(1)
    for sw, sh in [((1 << 24) + 1, 8), (8, (1 << 24) + 1), (0, 8), (8, -1)]:
        st = ctf.lib.ctf_filter(dummy, dummy, dummy, sw, sh, dummy, ctypes.byref(m), 0, dummy, None, None,
                                None, None, None)
        assert st == 1, (sw, sh, st)
        assert b"screen" in ctf.lib.ctf_last_error()
        st = ctf.lib.ctf_filter_layers(dummy, dummy, dummy, sw, sh, 1, texs, xf, ctypes.byref(m), 0, dummy,
                                       None, None, None, None)
        assert st == 1, (sw, sh, st)


def test_binding_fails_loudly_without_the_library(tmp_path):
    """A copy of the binding with no built library beside it refuses to
    import: nothing on the product path falls back to the CPU."""
    import shutil
    import subprocess
    import sys
    pkg = tmp_path / "paper_2506_17770_amd"
    pkg.mkdir()
    shutil.copy(os.path.join(ROOT, "paper_2506_17770_amd", "__init__.py"), pkg / "__init__.py")
    code = ("import sys; sys.path.insert(0, sys.argv[1])\n"
            "try:\n    import paper_2506_17770_amd\nexcept ImportError as e:\n    print('refused:', e); sys.exit(7)\n"
            "sys.exit(0)\n")
    r = subprocess.run([sys.executable, "-c", code, str(tmp_path)], capture_output=True, text=True, timeout=120)
    assert r.returncode == 7, r.stdout + r.stderr
    assert "no CPU fallback" in r.stdout


class _FakeDev:
    def __init__(self, index):
        self.index = index


class _FakeTensor:
    """Stands in for a device tensor: the binding's buffer checks read only
    these attributes (no GPU here)."""

    def __init__(self, numel, dtype, device=0, contiguous=True, cuda=True, itemsize=4):
        self._n, self.dtype, self.device = numel, dtype, _FakeDev(device)
        self._c, self.is_cuda, self._s = contiguous, cuda, itemsize

    def numel(self):
        return self._n

    def element_size(self):
        return self._s

    def is_contiguous(self):
        return self._c

    def data_ptr(self):
        return 4096


def test_binding_checks_caller_buffers():
    """A buffer the library would write past, or read with the wrong type or
    on another device, is refused before the call."""
    import pytest
    import torch
    import paper_2506_17770_amd as ctf
    f32 = torch.float32
    assert ctf._buf(None, "x", f32, 10, 0) is None
    assert ctf._buf(_FakeTensor(10, f32), "x", f32, 10, 0) == 4096
    bad = [_FakeTensor(9, f32),                     # too short
           _FakeTensor(10, torch.int32),            # wrong dtype
           _FakeTensor(10, f32, device=1),          # another device
           _FakeTensor(10, f32, contiguous=False),
           _FakeTensor(10, f32, cuda=False)]
    for t in bad:
        with pytest.raises(ctf.CtfError):
            ctf._buf(t, "x", f32, 10, 0)
    # byte-counted buffers (tile records)
    assert ctf._buf(_FakeTensor(128, torch.uint8, itemsize=1), "ts", None, 128, 0) == 4096
    with pytest.raises(ctf.CtfError):
        ctf._buf(_FakeTensor(127, torch.uint8, itemsize=1), "ts", None, 128, 0)


def test_tile_buffers_follow_the_wave_shape():
    """8x4 waves write a record per 8x4 tile: twice the rows of 8x8 tiles."""
    import paper_2506_17770_amd as ctf
    m8, m4 = ctf.method(ctf.LIST), ctf.method(ctf.LIST, wave_shape=ctf.WAVE_8X4)
    assert ctf.n_tiles(203, 77, m8) == 26 * 10 and ctf.n_tiles(203, 77, m4) == 26 * 20
    assert ctf.tile_stats_buffer(203, 77, device="cpu", meth=m4).shape == (26 * 20, 128)
    assert ctf.tile_stats_buffer(203, 77, device="cpu", meth=m8).shape == (26 * 10, 128)
    assert ctf.lists_buffer(203, 77, device="cpu", meth=m4).shape == (26 * 20, ctf.MAX_ITEMS, 2)
    assert ctf.tile_stats_buffer(203, 77, device="cpu", meth=m8, layers=6).shape == (6 * 26 * 10, 128)
