"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The oracle's C source, built with gcc's sanitizers, runs O1 and O2 on small
  dense, rectangular and banded inputs (and checks them against numpy).
* The library, built with clang's sanitizers on its host code only (the GPU
  code is built as usual), runs every host path that needs no device: grid
  construction, traversal plans, argument validation, and ps_create up to
  the point where it finds no GPU (so its clean-up after a device error runs
  too).

Each case runs in a child Python with the sanitizer runtime preloaded, leak
detection off (the HIP runtime and CPython keep allocations to the end), and
undefined behaviour fatal; a report ends the child with a non-zero status.
"""
import glob
import os
import subprocess
import sys
import textwrap
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2606_26785_amd", "csrc")
HIPCC = "/opt/rocm/bin/hipcc"

# host-only sanitizer flags: each one applies to the host pass of hipcc
HOST_SAN = "-Xarch_host -fsanitize=address -Xarch_host -fsanitize=undefined -Xarch_host -fno-omit-frame-pointer".split()
GCC_SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]


def _run_child(script, preload, tmp_path):
    path = tmp_path / "child.py"
    path.write_text(textwrap.dedent(script))
    env = dict(os.environ)
    env["LD_PRELOAD"] = preload
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:exitcode=23"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:exitcode=24:print_stacktrace=1"
    r = subprocess.run([sys.executable, str(path)], capture_output=True, text=True, timeout=600, env=env,
                       cwd=str(tmp_path))
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert r.returncode == 0 and "child ok" in r.stdout, out[-4000:]


def test_oracle_under_asan_and_ubsan(tmp_path):
    lib = tmp_path / "libpsoracle_san.so"
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c99", "-fopenmp", "-fPIC", "-shared"] + GCC_SAN +
                          [os.path.join(ROOT, "oracle", "ps_oracle.c"), "-o", str(lib), "-lm"])
    preload = subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    script = """
        import sys
        sys.path.insert(0, %r)
        import numpy as np
        import oracle
        oracle._LIB = %r
        rng = np.random.default_rng(3)
        for m, n in ((7, 7), (9, 6), (1, 1)):
            C = rng.standard_normal((m, n)) + 1j * rng.standard_normal((m, n))
            zs = np.array([0.3 - 0.2j, -1.0 + 0.5j])
            sig, sweeps = oracle.sigma_min_dense(C, zs)
            for z, s in zip(zs, sig):
                A = C - z * np.eye(m, n)
                assert abs(s - np.linalg.svd(A, compute_uv=False)[-1]) < 1e-12 * max(1.0, np.abs(A).max())
            sv = oracle.singular_values_dense(C)
            assert np.allclose(np.sort(sv), np.sort(np.linalg.svd(C, compute_uv=False)), atol=1e-12)
        n = 30
        T = (np.diag(np.full(n, 1.0 + 0.5j)) + np.diag(np.full(n - 1, 0.7), 1) + np.diag(np.full(n - 1, -0.4j), -1)
             + np.diag(np.full(n - 3, 0.2), 3))
        for C in (T, np.vstack([T, T[:4]])):
            band, kl, ku = oracle.band_from_dense(C)
            zs = np.array([0.9 + 0.4j, 2.0 - 1.0j])
            sig = oracle.sigma_min_banded(band, C.shape[0], n, kl, ku, zs)
            for z, s in zip(zs, sig):
                ref = np.linalg.svd(C - z * np.eye(C.shape[0], n), compute_uv=False)[-1]
                assert abs(s - ref) < 1e-10
            small = oracle.banded_smallest(band, C.shape[0], n, kl, ku, zs[0], k=3)
            ref = np.sort(np.linalg.svd(C - zs[0] * np.eye(C.shape[0], n), compute_uv=False))[:3]
            assert np.allclose(small, ref, atol=1e-10)
        print("child ok")
    """ % (ROOT, str(lib))
    _run_child(script, preload, tmp_path)


def _clang_asan_runtime():
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def test_library_host_code_under_asan_and_ubsan(tmp_path):
    rt = _clang_asan_runtime()
    if rt is None or not os.path.exists(HIPCC):
        pytest.skip("clang sanitizer runtime or hipcc not installed")
    srcs = sorted(glob.glob(os.path.join(CSRC, "*.hip")))
    flags = ["-O1", "-g", "--offload-arch=gfx950", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", os.path.join(ROOT, "include"), "-I", CSRC] + HOST_SAN

    def compile_one(src):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        r = subprocess.run([HIPCC] + flags + ["-c", src, "-o", obj], capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        return obj

    with ThreadPoolExecutor(max_workers=4) as ex:
        objs = list(ex.map(compile_one, srcs))
    lib = str(tmp_path / "libps_san.so")
    r = subprocess.run([HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-shared-libasan"] + HOST_SAN[:4] + objs +
                       ["-L/opt/rocm/lib", "-Wl,-rpath,/opt/rocm/lib", "-lrocblas", "-o", lib],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    script = """
        import sys
        sys.path.insert(0, %r)
        import numpy as np
        import paper_2606_26785_amd as P
        P.LIB_PATH = %r
        P.load()
        P.ps_grid(-1, 1, -2, 2, 7, 5).close()
        for bad in ((0, 1, 0, 1, 0, 3), (0, float("nan"), 0, 1, 3, 3)):
            try:
                P.ps_grid(*bad)
                raise SystemExit("bad grid accepted")
            except P.PSError:
                pass
        for nx, ny, tx, ty, b in ((1, 1, 1, 1, 1), (7, 5, 2, 3, 2), (33, 17, 4, 3, 5), (64, 64, 8, 8, 16)):
            for trav in (0, 1, 2):
                tiles = P.debug_order(nx, ny, tx, ty, b, trav)
                assert sorted(np.concatenate(tiles).tolist()) == list(range(nx * ny))
        rng = np.random.default_rng(0)
        C = rng.standard_normal((6, 4)) + 1j * rng.standard_normal((6, 4))
        rowptr = np.array([0, 1, 2, 3, 4, 4, 4], dtype=np.int64)
        colind = np.array([0, 1, 2, 3], dtype=np.int32)
        cases = [dict(dense=C[:3]), dict(dense=C, params=P.default_params(r=3)),
                 dict(dense=C, params=P.default_params(precond=2, rbar=4)), dict(dense=C),
                 dict(csr=(rowptr, colind, np.ones(4, dtype=np.complex128)), m=6, n=4)]
        for kw in cases:
            try:
                P.ps_create(**kw).close()
            except P.PSError:
                pass
        print("child ok")
    """ % (ROOT, lib)
    _run_child(script, rt, tmp_path)
