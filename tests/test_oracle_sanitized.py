"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer (host only).

slref.c is built with -fsanitize=address,undefined into a temporary directory and exercised in
a child Python process that preloads the sanitizer runtimes: every entry point, on small inputs
and on the edge cases (one point, coincident points, distinct targets, per-target delta, more
threads than points).  Any sanitizer report fails the test."""
import os
import subprocess
import sys
import textwrap

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

SCRIPT = textwrap.dedent("""
    import numpy as np
    import oracle
    from oracle import fmm
    rng = np.random.default_rng(7)
    for n in (1, 2, 37, 300):
        X = rng.normal(size=(n, 3)); w = rng.uniform(0.5, 1.5, n); f = rng.normal(size=(n, 3))
        if n > 2:
            X[1] = X[0]                      # coincident points: the r = 0 limit
        d = 0.3
        oracle.single_layer(X, w, f, d)
        oracle.single_layer(X, w, f, d, nthreads=1)
        oracle.single_layer(X, w, f, d, targets=X[: max(1, n // 2)] + 0.01)
        oracle.single_layer(X, w, f, d, delta_tgt=rng.uniform(0.1, 0.5, n))
        oracle.stokeslet(X, f, X + 5.0)
    for p in (0.0, 1e-3, 0.5, 3.0, 40.0):
        oracle.smoothing(p)
        oracle.kernel(p, 0.25)
    for n in (4, 6):
        g = np.linspace(0.1, 3.0, n)
        P = np.stack(np.meshgrid(g, g, indexing="ij"), -1).reshape(-1, 2)
        Xp = np.concatenate([np.c_[P, np.full(len(P), float(k))] for k in range(6)])
        oracle.patch_delta(Xp, n)
    X = rng.normal(size=(400, 3)); w = np.ones(400); f = rng.normal(size=(400, 3))
    fmm.single_layer_fmm(X, w, f, 0.05, k=5, p=4, max_iter=10)
    print("sanitized oracle: ok")
""")


def _runtime(name):
    try:
        p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True,
                           check=True).stdout.strip()
    except (OSError, subprocess.CalledProcessError):
        return None
    return p if os.path.isabs(p) and os.path.exists(p) else None


def test_oracle_under_asan_and_ubsan(tmp_path):
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("gcc's sanitizer runtimes are not installed")
    lib = str(tmp_path / "libslref_san.so")
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-fPIC", "-shared",
                    "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", "-o", lib,
                    os.path.join(ROOT, "oracle", "slref.c"), "-lm"], check=True)
    env = dict(os.environ, SLREF_LIB=lib, LD_PRELOAD=f"{asan} {ubsan}",
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
               OMP_NUM_THREADS="4", PYTHONPATH=ROOT)
    r = subprocess.run([sys.executable, "-c", SCRIPT], cwd=ROOT, env=env, capture_output=True,
                       text=True, timeout=600)
    report = r.stdout + r.stderr
    assert r.returncode == 0, report[-4000:]
    assert "AddressSanitizer" not in report and "runtime error" not in report, report[-4000:]
    assert "sanitized oracle: ok" in r.stdout
