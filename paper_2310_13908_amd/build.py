"""Build libstokeslet.so (all HIP sources under csrc/) for gfx950, in-tree.

`python -m paper_2310_13908_amd.build --host-ubsan` also builds libstokeslet_ubsan.so: the same
library with its host code under UndefinedBehaviorSanitizer (device code unchanged), which the
binding loads instead when SL_LIB names it."""
from __future__ import annotations

import glob
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
LIB = os.path.join(PKG, "libstokeslet.so")
LIB_UBSAN = os.path.join(PKG, "libstokeslet_ubsan.so")
ARCH = "gfx950"
# host code only (each sanitizer flag behind -Xarch_host), runtime linked as a dependency
# (reports are printed and the run goes on, so that one run lists them all)
UBSAN_FLAGS = ["-Xarch_host", "-fsanitize=undefined", "-Xarch_host", "-fno-omit-frame-pointer",
               "-shared-libsan"]

HIPCC_FLAGS = [
    f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC", "-shared",
    # packed FP32 instructions stay off: plain single-precision code only
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def sources():
    return sorted(glob.glob(os.path.join(PKG, "csrc", "*.hip")))


def _ubsan_rpath(hipcc: str) -> list:
    """-Wl,-rpath to the directory of clang's UBSan runtime, so the library finds it."""
    res = subprocess.run([hipcc, "-print-file-name=libclang_rt.ubsan_standalone-x86_64.so"],
                         capture_output=True, text=True)
    f = res.stdout.strip()
    if res.returncode != 0 or not os.path.isabs(f) or not os.path.exists(f):
        res = subprocess.run([hipcc, "-print-resource-dir"], capture_output=True, text=True)
        f = os.path.join(res.stdout.strip(), "lib", "linux", "libclang_rt.ubsan_standalone-x86_64.so")
    return [f"-Wl,-rpath,{os.path.dirname(f)}"] if os.path.exists(f) else []


def build(verbose: bool = False, host_ubsan: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    out = LIB_UBSAN if host_ubsan else LIB
    tmp = out + f".tmp{os.getpid()}"
    extra = UBSAN_FLAGS + _ubsan_rpath(hipcc) if host_ubsan else []
    cmd = [hipcc, *HIPCC_FLAGS, *extra, "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(PKG, "csrc"), "-o", tmp, *sources()]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError(f"hipcc failed building {os.path.basename(out)}")
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
    if "--host-ubsan" in sys.argv[1:]:
        print(build(verbose=True, host_ubsan=True))
