"""Build libdmrg.so (HIP, gfx950) in-tree with hipcc.

    python paper_2001_04890_amd/build.py

(Run by path: importing the package would load the library that is being rebuilt.)
"""
import concurrent.futures
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdmrg.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Packed-FP32 instructions are disabled for every HIP translation unit.
COMMON = ["--offload-arch=gfx950", "-O3", "-std=c++17", "-fPIC",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
SOURCES = ["kernels.hip", "hpsi_lds.hip", "hpsi_big.hip", "hpsi_big64.hip", "hpsi_lds64.hip", "mlp.hip", "host.cpp", "plan.cpp", "mlp_host.cpp",
           "renorm_host.cpp", "davidson.cpp", "eigen.cpp", "noalloc.cpp", "grow.hip", "grow.cpp",
           "sweep.cpp", "davidson_batch.hip", "davidson_batch.cpp"]


def _run(cmd):
    r = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    out = "\n".join(l for l in r.stdout.splitlines() if "packed-fp32-ops" not in l)
    if r.returncode != 0:
        raise RuntimeError("build failed: " + " ".join(cmd) + "\n" + out)
    return out


def build(verbose=False):
    build_dir = os.path.join(HERE, "_build")
    os.makedirs(build_dir, exist_ok=True)
    def compile_one(src):
        obj = os.path.join(build_dir, src.replace(".", "_") + ".o")
        lang = ["-x", "hip"] if src.endswith(".cpp") else []
        return obj, _run([HIPCC] + COMMON + lang + ["-c", os.path.join(CSRC, src), "-o", obj])

    # translation units compile in parallel (at most 8 hipcc processes)
    with concurrent.futures.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        results = list(ex.map(compile_one, SOURCES))
    objs = []
    for obj, out in results:
        if verbose and out.strip():
            print(out)
        objs.append(obj)
    tmp = LIB + ".tmp"
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
