"""Host code under sanitizers (no GPU): the planner (time recipe, modified
frequencies, quadrature, B and its inverse, the least-squares optimiser, the
largest |mu_d|) and the host step of a deflated GMRES restart, built with g++
and AddressSanitizer + UndefinedBehaviorSanitizer into a driver that runs
them on explicit and implicit plans, plain and truncated least squares, two
to eight frequencies and restart lengths 12 to 60.  The GPU kernels are not
covered here (GPU sanitizer builds are not available)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not found")
def test_host_code_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    src = os.path.join(ROOT, "paper_2507_23613_amd", "csrc")
    exe = str(tmp_path / "host_sanitize_driver")
    subprocess.run(["g++", "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-I", src,
                    os.path.join(ROOT, "tests", "host_sanitize_driver.cpp"),
                    os.path.join(src, "plan.cpp"), os.path.join(src, "krylov.cpp"),
                    "-o", exe], check=True, timeout=900)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stdout + r.stderr
    lines = r.stdout.splitlines()
    assert lines[-1] == "done bad=0"
    assert sum(x.startswith("plan ") and x.endswith("finite=1") for x in lines) == 12
    assert sum(x.startswith("deflation ") and x.endswith("orth=1") for x in lines) == 3
