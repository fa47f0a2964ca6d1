"""The library's host code under AddressSanitizer (no GPU): a build of every
HIP source with the sanitizer on the host side only (device code as usual),
then the argument-validation tests of the C ABI run against it with the
sanitizer runtime preloaded (the host planning checks carry their own
sanitizer build).  Any invalid
read or write in the host-side validation, planning or error paths aborts
the run and fails this test."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_2102_02440_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _hipcc_ok():
    return os.path.exists(HIPCC)


@pytest.mark.skipif(not _hipcc_ok(), reason="hipcc not installed")
def test_host_code_under_asan(tmp_path):
    out = str(tmp_path / "libcompass_asan.so")
    srcs = sorted(os.path.join(CSRC, f) for f in os.listdir(CSRC) if f.endswith(".hip"))
    cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-shared",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Xarch_host", "-fsanitize=address",
           "-Xarch_host", "-fno-omit-frame-pointer", "-shared-libsan",
           "-I", os.path.join(ROOT, "include"), "-I", CSRC, *srcs, "-o", out]
    subprocess.check_call(cmd, stderr=subprocess.DEVNULL)
    rt = subprocess.check_output(
        [HIPCC, "-print-file-name=libclang_rt.asan-x86_64.so"], text=True).strip()
    assert os.path.exists(rt), rt
    env = dict(os.environ, LD_PRELOAD=rt, COMPASS_LIB=out,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1")
    run = subprocess.run(
        [sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-p", "no:cacheprovider",
         os.path.join(HERE, "test_abi.py")],
        env=env, cwd=ROOT, capture_output=True, text=True, timeout=600)
    tail = (run.stdout + run.stderr)[-4000:]
    assert run.returncode == 0, tail
    assert "AddressSanitizer" not in run.stderr, tail
    assert " passed" in run.stdout, tail
