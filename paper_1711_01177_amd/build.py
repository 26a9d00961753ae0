"""Build libgrim.so (HIP kernels + C ABI + serving runtime) for gfx950 in-tree.

    python -m paper_1711_01177_amd.build

Every HIP translation unit is compiled with hipcc for gfx950 with the
packed-FP32 target feature disabled; the objects are linked into one shared
library next to this file.
"""
import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libgrim.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

SOURCES = ["grim_kernels.hip", "grim_checker.hip", "grim_seed.hip", "grim_window.hip",
           "grim_build.hip", "grim_probe.hip", "grim_copy.hip", "grim_api.hip", "grim_host.cpp",
           "grim_serve.cpp", "grim_serve_hip.cpp"]

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-result",
          f"-I{INCLUDE}", f"-I{CSRC}"]
DEVICE = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines()
                    if "packed-fp32-ops" not in l and "not a recognized feature" not in l)
    if r.returncode != 0:
        raise RuntimeError(f"command failed ({r.returncode}): {' '.join(cmd)}\n{out}")
    return out


def build(verbose=False):
    """Compile every source and link libgrim.so (always rebuilds)."""
    with tempfile.TemporaryDirectory(prefix="grim_build_") as tmp:
        objs = []
        for src in SOURCES:
            path = os.path.join(CSRC, src)
            obj = os.path.join(tmp, src + ".o")
            if src.endswith(".hip"):
                cmd = [HIPCC, "-x", "hip", *DEVICE, *COMMON, "-c", path, "-o", obj]
            else:
                cmd = [HIPCC, *COMMON, "-c", path, "-o", obj]
            out = _run(cmd)
            if verbose and out.strip():
                print(out)
            objs.append(obj)
        tmp_lib = LIB + ".tmp"
        _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", tmp_lib,
              "-lpthread"])
        os.replace(tmp_lib, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
