"""Build the MFWH HIP library (libmfwh.so) in-tree for gfx950.

    python -m paper_2507_23613_amd.build        # or build() from Python

Every HIP source is compiled with hipcc for gfx950 with packed-FP32 code
generation disabled; the host-only planner is compiled with g++.  Objects go
to paper_2507_23613_amd/_build/, the library to paper_2507_23613_amd/libmfwh.so.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libmfwh.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

HIP_FLAGS = ["-O3", "-std=c++17", f"--offload-arch={ARCH}", "-fPIC", "-Wall",
             "-Wno-unused-result", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-munsafe-fp-atomics", f"-I{ROOT}/include"]
CXX_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall", f"-I{ROOT}/include"]


def _sources():
    hip = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))
    cpp = sorted(f for f in os.listdir(CSRC) if f.endswith(".cpp"))
    return hip, cpp


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    return r


def _torch_lib():
    """Directory of the HIP runtime bundled with PyTorch.  The library links
    against it so that a process using PyTorch for device memory has exactly
    one HIP runtime (two runtimes in one process do not share devices)."""
    import importlib.util
    spec = importlib.util.find_spec("torch")
    if spec is None or not spec.submodule_search_locations:
        raise RuntimeError("PyTorch (ROCm build) is required to link libmfwh.so")
    d = os.path.join(list(spec.submodule_search_locations)[0], "lib")
    if not os.path.exists(os.path.join(d, "libamdhip64.so")):
        raise RuntimeError(f"no libamdhip64.so under {d}")
    return d


def build(verbose=False):
    os.makedirs(OUT, exist_ok=True)
    hip, cpp = _sources()
    jobs = []
    for f in hip:
        jobs.append([HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, f),
                     "-o", os.path.join(OUT, f + ".o")])
    for f in cpp:
        jobs.append(["g++", *CXX_FLAGS, "-c", os.path.join(CSRC, f),
                     "-o", os.path.join(OUT, f + ".o")])
    workers = min(len(jobs), int(os.environ.get("MAX_JOBS", "8")))
    with ThreadPoolExecutor(max_workers=max(1, workers)) as ex:
        for r in ex.map(_run, jobs):
            if verbose and (r.stdout or r.stderr):
                print(r.stdout + r.stderr, file=sys.stderr)
    objs = [os.path.join(OUT, f + ".o") for f in hip + cpp]
    tmp = LIB + ".tmp"
    tl = _torch_lib()
    clang = os.path.join(os.path.dirname(os.path.realpath(HIPCC)), "..", "lib", "llvm", "bin",
                         "clang++")
    if not os.path.exists(clang):
        clang = "/opt/rocm/lib/llvm/bin/clang++"
    _run([clang, "-shared", "-fPIC", "-o", tmp, *objs, f"-L{tl}", "-l:libamdhip64.so",
          f"-Wl,-rpath,{tl}", "-Wl,--disable-new-dtags", "-Wl,--no-undefined", "-lstdc++",
          "-lm"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
