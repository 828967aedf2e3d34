"""The oracle and the library's host-side planning built with AddressSanitizer
and UndefinedBehaviorSanitizer (host code only; no GPU): the oracle's pins
and its two parts against each other run clean, and the exported host-only
entry points (exact eps^2, grid geometry, context creation without a device)
run clean over many inputs."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"]


def runtime(name: str) -> str:
    out = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout.strip()
    return out if out and os.path.isabs(out) and os.path.exists(out) else ""


def test_oracle_pins_under_sanitizers(tmp_path):
    asan, ubsan = runtime("libasan.so"), runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("gcc sanitizer runtimes not found")
    so = tmp_path / "liboracle_san.so"
    subprocess.run(["gcc", "-O1", "-fopenmp", "-shared", "-fPIC", "-std=gnu11", *SAN,
                    str(ROOT / "oracle" / "dbscan_def.c"), str(ROOT / "oracle" / "hca_grid.c"),
                    "-o", str(so), "-lm"], check=True)
    script = f"""
import sys
sys.path.insert(0, {str(ROOT)!r}); sys.path.insert(0, {str(ROOT / 'tests')!r})
import numpy as np
import oracle, test_oracle as T
lib = oracle.load_variant({str(so)!r})
for pin in T.PINS:
    pin(lib)
rng = np.random.default_rng(3)
for trial in range(40):
    d = int(rng.integers(1, 9)); n = int(rng.integers(0, 300))
    pts = T.rand_points(rng, n, d, int(rng.integers(2, 60)), 0.1)
    eps = float(rng.uniform(0.5, 25.0)); mp = int(rng.integers(1, 9))
    want = oracle.dbscan(pts, eps, mp, lib=lib)
    for mode in (0, 1, 2):
        got = oracle.hca_grid(pts, eps, mp, rep_mode=mode, lib=lib)
        if mode != 1:
            assert (got == want).all(), (trial, mode)
print("clean")
"""
    env = dict(os.environ, LD_PRELOAD=f"{asan}:{ubsan}", ASAN_OPTIONS="detect_leaks=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, "-c", script], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0 and "clean" in r.stdout, r.stderr[-4000:]
    assert "runtime error" not in r.stderr, r.stderr[-4000:]


DRIVER = r'''
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include "hca.h"
int main()
{
    unsigned long long x = 12345;
    int bad = 0;
    for (int i = 0; i < 20000; i++) {
        x = x * 6364136223846793005ull + 1442695040888963407ull;
        const double eps = std::ldexp((double)(x >> 11) / 9007199254740992.0 + 0.5, (int)(x % 80) - 20);
        int64_t e2 = 0;
        if (hca_exact_eps2(eps, &e2) != HCA_OK) bad++;
        /* geometry enumerates the cube stencil: many small d, a few large */
        const int d = i < 19000 ? 1 + (int)((x >> 7) % 4) : 1 + (int)((x >> 7) % 64);
        if (i % 10 && d > 4) continue;
        hca_geometry g;
        const hca_status st = hca_get_geometry(eps, d, &g);
        if (st != HCA_OK && st != HCA_E_RANGE) bad++;
    }
    int64_t e2;
    if (hca_exact_eps2(0.0, &e2) != HCA_E_INVAL || hca_exact_eps2(NAN, &e2) != HCA_E_INVAL) bad++;
    hca_ctx *ctx = nullptr;
    const hca_status st = hca_create(&ctx, 0);      /* no device here: an error, not a crash */
    if (st == HCA_OK) hca_destroy(ctx);
    hca_destroy(nullptr);
    std::printf("%s\n", bad ? "bad" : "clean");
    return bad;
}
'''


def test_host_planner_under_sanitizers(tmp_path):
    """hca_api.cpp and hca_tune.cpp built with host-side sanitizers, linked
    with the device objects of the normal build."""
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    bdir = ROOT / "paper_1912_00323_amd" / "csrc" / "_build"
    objs = [bdir / f"{s}.o" for s in ("hca_sort.hip", "hca_grid.hip", "hca_highd.hip", "hca_batch.hip",
                                       "hca_static.hip", "hca_server.cpp")]
    if not os.path.exists(hipcc) or not all(o.exists() for o in objs):
        pytest.skip("hipcc or the library's objects (built by build()) are missing")
    csrc = ROOT / "paper_1912_00323_amd" / "csrc"
    (tmp_path / "driver.cpp").write_text(DRIVER)
    host_san = [f for s in SAN for f in (["-Xarch_host", s] if s.startswith("-fsanitize") or s.startswith("-fno-san")
                                          else [s])]
    exe = tmp_path / "planner_check"
    cmd = [hipcc, "-O1", "-std=c++17", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
           "-packed-fp32-ops", f"-I{ROOT / 'include'}", f"-I{csrc}", *host_san,
           str(csrc / "hca_api.cpp"), str(csrc / "hca_tune.cpp"), str(tmp_path / "driver.cpp"),
           "-x", "none", *map(str, objs), "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               HIP_VISIBLE_DEVICES="")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0 and "clean" in r.stdout, (r.stdout[-2000:], r.stderr[-4000:])
    assert "runtime error" not in r.stderr, r.stderr[-4000:]
