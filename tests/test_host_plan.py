"""Host-side planning arithmetic of the builds, compiled with g++ (no GPU):
fused-scan chunks stay below INT32_MAX rows (int32 partials), the batch
plan's LDS guard with a forced budget, and the two-phase build's survivor
buffer, batches and hashing chunks.  Built with AddressSanitizer and
UndefinedBehaviorSanitizer (an overflow in the planning arithmetic aborts)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2102_02440_amd", "csrc")


def test_plan_arithmetic(tmp_path):
    exe = str(tmp_path / "plan_check")
    subprocess.check_call(["g++", "-std=c++17", "-O1", "-g", "-Wall",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-I", CSRC,
                           os.path.join(HERE, "host", "plan_check.cpp"), "-o", exe])
    out = subprocess.run([exe], capture_output=True, text=True)
    print(out.stdout)
    assert out.returncode == 0, out.stdout + out.stderr
    assert "ALL OK" in out.stdout
