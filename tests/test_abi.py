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


def test_write_pmc_scales_by_the_calibration_copy(tmp_path, monkeypatch):
    """bench.py --write-pmc: per-dispatch means of each kernel, scaled to bytes by what the same
    counter read for the 1 GiB copy (the largest copy dispatch; the runtime's small copies are
    ignored), keyed by the pair kernel's hash."""
    import csv
    import json
    import sys
    sys.path.insert(0, ROOT)
    import bench
    hdr = ["Kernel_Name", "Counter_Name", "Counter_Value"]
    fetch = {"__amd_rocclr_copyBuffer": [2.0, 524288.0, 1.5],
             "void sl::(anonymous namespace)::k_pair<1, false, true, false, 4, false>(sl::PairArgs)": [100.0, 300.0],
             "void sl::(anonymous namespace)::k_pair<2, false, false, false, 1, false>(sl::PairArgs)": [1000.0],
             "void sl::(anonymous namespace)::k_reduce(double const*, int)": [64.0],
             "void at::native::elementwise_kernel(int)": [9e9]}
    write = {"__amd_rocclr_copyBuffer": [1.0, 1048576.0],
             "void sl::(anonymous namespace)::k_pair<1, false, true, false, 4, false>(sl::PairArgs)": [40.0, 40.0],
             "void sl::(anonymous namespace)::k_pair<2, false, false, false, 1, false>(sl::PairArgs)": [80.0],
             "void sl::(anonymous namespace)::k_reduce(double const*, int)": [8.0]}
    for tag in ("c3", "c2"):
        for counter, rows in (("FETCH_SIZE", fetch), ("WRITE_SIZE", write)):
            d = tmp_path / f"p_{tag}_{counter}"
            d.mkdir()
            with open(d / "run_counter_collection.csv", "w", newline="") as fh:
                w = csv.writer(fh)
                w.writerow(hdr)
                for k, vals in rows.items():
                    for v in vals:
                        w.writerow([k, counter, v])
    out = tmp_path / "pmc.json"
    monkeypatch.setattr(bench, "PMC_FILE", str(out))
    bench.write_pmc(str(tmp_path / "p"))
    rec = json.load(open(out))
    assert rec["pair_kernel_sha"] == bench.pair_kernel_sha()
    wl = rec["workloads"]["rbc_6x256x256_sh8"]
    assert wl["fetch_scale"] == 2.0 and wl["write_scale"] == 1.0
    assert wl["mixed"]["kernel"] == "k_pair<1, false, true, false, 4, false>"
    assert wl["mixed"]["dispatches"] == 2
    assert wl["mixed"]["fetch_bytes"] == 200 * 1024 * 2 and wl["mixed"]["write_bytes"] == 40 * 1024
    assert wl["mixed"]["hbm_bytes_per_launch"] == 200 * 2048 + 40 * 1024
    assert wl["fp64"]["hbm_bytes_per_launch"] == 1000 * 2048 + 80 * 1024
    assert wl["k_reduce"] == {"fetch_bytes": 64 * 2048, "write_bytes": 8 * 1024}
    assert set(rec["workloads"]) == {"rbc_6x256x256_sh8", "rbc_6x64x64_sh8"}
