"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer:
every source is rebuilt with the sanitizers on the host side only (the GPU
code is unchanged), linked into a C driver that walks the C ABI paths needing
no GPU, and run."""
import os
import shutil
import subprocess

import pytest

from paper_2405_12497_amd import build as B

HERE = os.path.dirname(os.path.abspath(__file__))


def test_host_code_under_asan_and_ubsan(tmp_path):
    hipcc = B._hipcc()
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
    objs = []
    for src in B.sources():
        obj = str(tmp_path / (src + ".o"))
        flags = B.COMMON + (B.DEVICE if src.endswith(".hip") else []) + ["-O1", "-g"] + san
        r = subprocess.run([hipcc, *flags, "-c", os.path.join(B.CSRC, src), "-o", obj], capture_output=True,
                           text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        objs.append(obj)
    exe = str(tmp_path / "capi_sanitize")
    r = subprocess.run([hipcc, f"--offload-arch={B.ARCH}", *san, "-g", "-I", os.path.join(os.path.dirname(HERE), "include"),
                        "-x", "c", os.path.join(HERE, "capi_sanitize_main.c"), "-x", "none", *objs, "-o", exe],
                       capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe, str(tmp_path)], capture_output=True, text=True, env=env, timeout=300)
    print(r.stdout[-2000:], r.stderr[-4000:])
    assert r.returncode == 0, r.stderr[-4000:]
    assert "sanitized host checks passed" in r.stdout
