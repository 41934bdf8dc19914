"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

* The oracle (oracle.c) built by gcc with -fsanitize=address,undefined runs the
  oracle's pin suite (tests/test_oracle.py) in a child process.
* The HIP library's host side, built with the sanitizers on the host pass only
  (``python -m paper_1904_12759_amd.build --sanitize`` -> libmcexpmv_san.so, built
  here when missing or older than the sources), runs the C-ABI checks that need
  no GPU (tests/test_abi.py: exports, status strings, argument validation).
* A canary: the same gcc flags stop a planted heap overflow, so a silent pass
  above is not a harness that checks nothing.
"""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_1904_12759_amd")
GCC_SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def _gcc_runtime():
    libs = [subprocess.check_output(["gcc", f"-print-file-name={n}"], text=True).strip()
            for n in ("libasan.so", "libubsan.so")]
    if not all(os.path.isabs(p) and os.path.exists(p) for p in libs):
        pytest.skip("gcc sanitizer runtimes not installed")
    return " ".join(libs)


def _run_pytest(args, env_extra):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", **env_extra)
    return subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                           *args], cwd=ROOT, env=env, capture_output=True, text=True,
                          timeout=900)


def test_sanitizer_canary_catches_heap_overflow(tmp_path):
    src = tmp_path / "bad.c"
    src.write_text("#include <stdlib.h>\nint main(void){int *p=malloc(4*sizeof(int));"
                   "p[4]=1;int r=p[4];free(p);return r-1;}\n")
    exe = tmp_path / "bad"
    subprocess.check_call(["gcc", *GCC_SAN, str(src), "-o", str(exe)])
    r = subprocess.run([str(exe)], capture_output=True, text=True)
    assert r.returncode != 0 and "heap-buffer-overflow" in r.stderr


def test_oracle_pins_under_asan_ubsan(tmp_path):
    pre = _gcc_runtime()
    lib = tmp_path / "liboracle_san.so"
    subprocess.check_call(["gcc", "-std=c11", "-O1", "-g", "-ffp-contract=off", "-fno-fast-math",
                           "-fPIC", "-shared", "-pthread", *GCC_SAN,
                           os.path.join(ROOT, "oracle", "oracle.c"), "-o", str(lib), "-lm"])
    r = _run_pytest(["tests/test_oracle.py"], {"LD_PRELOAD": pre, "ORACLE_LIB": str(lib)})
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "passed" in r.stdout


def _san_lib_current(lib):
    if not os.path.exists(lib):
        return False
    t = os.path.getmtime(lib)
    srcs = glob.glob(os.path.join(PKG, "csrc", "*")) + glob.glob(os.path.join(ROOT, "include", "*.h"))
    return all(os.path.getmtime(s) <= t for s in srcs)


def test_library_host_code_under_asan_ubsan():
    clang = "/opt/rocm/llvm/bin/clang"
    if not os.path.exists(clang):
        pytest.skip("ROCm clang not installed")
    rt = subprocess.check_output([clang, "-print-file-name=libclang_rt.asan-x86_64.so"],
                                 text=True).strip()
    if not os.path.exists(rt):
        pytest.skip("clang AddressSanitizer runtime not installed")
    sys.path.insert(0, ROOT)
    from paper_1904_12759_amd import build as b
    if not _san_lib_current(b.SAN_LIB):
        b.build(sanitize=True)
    r = _run_pytest(["tests/test_abi.py"], {"LD_PRELOAD": rt, "MC_EXPMV_LIB": b.SAN_LIB})
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "passed" in r.stdout
