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
