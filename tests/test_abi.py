"""The C ABI without a GPU: the built library loads, exports every function include/vapr.h declares,
and rejects bad arguments on the host before touching the device."""
import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vapr.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vapr_[a-z_0-9]+)\s*\(", text)))


def lib():
    from paper_2310_07854_amd import _lib as L

    if not os.path.exists(L.LIB_PATH):
        pytest.skip("libvapr.so not built (run __graft_entry__.build())")
    return L, L.load()


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("vapr_create", "vapr_set_robot", "vapr_set_worlds", "vapr_set_precision", "vapr_cost_fwd",
                     "vapr_cost_bwd", "vapr_optimizer_step", "vapr_quantize", "vapr_dequantize"):
        assert required in names


def test_every_declared_symbol_is_exported():
    L, _ = lib()
    out = subprocess.run(["nm", "-D", "--defined-only", L.LIB_PATH], capture_output=True, text=True, check=True).stdout
    exported = set(re.findall(r" T (vapr_[a-z_0-9]+)", out))
    missing = [n for n in declared_functions() if n not in exported]
    assert not missing, missing
    # and the Python binding declares a signature for each
    assert set(declared_functions()) == set(L.SIGNATURES)


def test_host_side_validation():
    L, so = lib()
    assert so.vapr_abi_version() == 4
    assert so.vapr_status_string(L.E_STATE) == b"invalid state"
    assert so.vapr_packed_bytes(L.E3M2, 5) == 4
    assert so.vapr_packed_bytes(L.E2M1, 3) == 2
    assert so.vapr_packed_bytes(99, 3) == 0
    buf = (ctypes.c_float * 16)()
    # unknown format, bad scale, f32 with a scale, negative count, misaligned buffer
    assert so.vapr_quantize(9, 0, buf, buf, 16, None) == L.E_INVALID
    assert so.vapr_quantize(L.E4M3, 17, buf, buf, 16, None) == L.E_INVALID
    assert so.vapr_quantize(L.F32, 1, buf, buf, 16, None) == L.E_INVALID
    assert so.vapr_quantize(L.E4M3, 0, buf, buf, -1, None) == L.E_INVALID
    assert so.vapr_quantize(L.E4M3, 0, ctypes.addressof(buf) + 1, buf, 4, None) == L.E_INVALID
    assert b"4-byte aligned" in so.vapr_last_error(None)  # the thread's last error, with no context
    assert so.vapr_quantize(L.E4M3, 0, buf, buf, 0, None) == L.OK  # nothing to do
    # context-taking calls reject a null context
    assert so.vapr_set_precision(None, None) == L.E_INVALID
    assert so.vapr_cost_bwd(None, None, None, 0, None, None) == L.E_INVALID
    assert so.vapr_ws_reset(None, None, 0) == L.E_INVALID
    assert so.vapr_sync(None) == L.E_INVALID
    assert so.vapr_destroy(None) == L.OK
