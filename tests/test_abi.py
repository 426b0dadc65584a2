"""CPU checks of the C-ABI library: it loads, exports every declared symbol, and rejects bad
arguments on the host before touching a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            src = open(os.path.join(ROOT, "include", fn)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(sl_[a-z_]+)\s*\(", src))
    return names


def test_library_exports_every_declared_symbol():
    import paper_2310_13908_amd as P
    lib = P.load()
    decl = declared_symbols()
    assert decl == set(P.EXPORTED)
    for name in decl:
        assert getattr(lib, name) is not None


def test_library_is_built_for_gfx950():
    import paper_2310_13908_amd as P
    blob = open(P._binding.LIB_PATH, "rb").read()
    assert b"gfx950" in blob


def test_host_side_validation_without_a_gpu():
    import paper_2310_13908_amd as P
    lib = P.load()
    # NULL context, bad sizes and bad scalars are rejected before any HIP call
    st = lib.sl_eval(None, 0, 10, 1, 1, 1, 1, 1, 1, 1, 10, None, None, None, 0.1, None, 1.0, 2, 3, 4, None)
    assert st == P.SL_EINVAL
    out = ctypes.c_void_p()
    assert lib.sl_create(0, 0, None) == P.SL_EINVAL
    assert "NULL" in P.sl_last_error()
    d = ctypes.c_double()
    assert lib.sl_get_param(None, P.SL_PARAM_RHO64, ctypes.byref(d)) == P.SL_EINVAL
    assert lib.sl_set_param(None, P.SL_PARAM_RHO64, 6.0) == P.SL_EINVAL
    assert lib.sl_patch_delta(None, 6, 4, 1, 2, 3, 1.0, 4, None) == P.SL_EINVAL
    assert "ctx is NULL" in P.sl_last_error()
    st = lib.sl_eval_noalloc(None, 0, 10, 1, 1, 1, 1, 1, 1, 1, 10, None, None, None, 0.1, None, 1.0,
                             2, 3, 4, None)
    assert st == P.SL_EINVAL
    assert "sl_eval_noalloc" in P.sl_last_error()


def test_pair_kernel_hash_ignores_comments_only():
    """The hash that keys the stored PMC traffic changes with the pair kernel's code and not with
    its comments or layout."""
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import bench
    src = "int f(int a) { // add one\n  return a + 1; /* done */ }\n"
    assert bench.code_text(src) == bench.code_text("int f(int a) {\n\n  return a + 1;   }")
    assert bench.code_text(src) != bench.code_text(src.replace("a + 1", "a + 2"))
    assert "//" not in bench.code_text(src) and "done" not in bench.code_text(src)
    for p in bench.PAIR_SOURCES:
        assert os.path.exists(os.path.join(bench.ROOT, p)), p
    assert re.fullmatch(r"[0-9a-f]{16}", bench.pair_kernel_sha())
