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
