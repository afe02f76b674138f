"""The C-ABI library loads and exports every entry point include/gsbc.h
declares; host-only calls behave as documented (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "gsbc.h")).read()
    return re.findall(r"^GSBC_API [^(]*?\b(gsbc_\w+)\s*\(", src, flags=re.M)


def test_header_declares_the_calls():
    names = set(_declared())
    assert {"gsbc_reorder", "gsbc_encode", "gsbc_decode", "gsbc_decode_eval", "gsbc_create",
            "gsbc_destroy", "gsbc_sync", "gsbc_last_error", "gsbc_query_sizes",
            "gsbc_default_params"} <= names


def test_library_exports_every_declared_symbol():
    from paper_2607_14513_amd import gsbc
    lib = gsbc.load()
    for name in _declared():
        assert hasattr(lib, name), name
    # and the binding names exactly the declared set
    assert set(gsbc.EXPORTED) == set(_declared())


def test_host_only_calls():
    from paper_2607_14513_amd import gsbc
    p = gsbc.default_params()
    assert (p.grid_bits, p.refine_steps, p.bc7_mode_mask) == (3, 2, 0xFF)
    tex, blk, out = gsbc.query_sizes(17, 5)
    assert tex == 16 * 32 * 4 and blk == 16 * 2 * 16 and out == 5 * 17 * 12
    with pytest.raises(gsbc.GsbcError):
        gsbc.query_sizes(0)
    lib = gsbc.load()
    assert lib.gsbc_destroy(None) == gsbc.E_ARG
    assert lib.gsbc_sync(None) == gsbc.E_ARG
    assert lib.gsbc_create(None, 0, None) == gsbc.E_ARG


def test_create_without_a_device_fails_cleanly():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a device is present")
    from paper_2607_14513_amd import gsbc
    h = ctypes.c_void_p()
    assert gsbc.load().gsbc_create(ctypes.byref(h), 0, None) == gsbc.E_DEVICE
    assert not h.value
    with pytest.raises(RuntimeError):
        gsbc.Context(0)
