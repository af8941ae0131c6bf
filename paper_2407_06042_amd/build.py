"""Build libdmala.so (gfx950 only) in-tree with hipcc.

Each source compiles to an object in _build/ in parallel; objects are relinked
into paper_2407_06042_amd/libdmala.so.  Run as `python -m paper_2407_06042_amd.build`.
"""
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(PKG, "libdmala.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

FLAGS = [
    "--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17",
    # packed fp32 VALU ops are avoided in every kernel
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-variable", "-Wno-unknown-pragmas",
    "-I", os.path.join(ROOT, "include"),
]

SOURCES = [
    "api.cpp", "plan.cpp", "setup.hip", "estimate.hip", "sampler.hip",
    "sampler_f64_naive.hip", "sampler_f64_pre.hip", "sampler_naive.hip",
    "sampler_f16x2.hip", "sampler_f16x1.hip", "sampler_bf16x1.hip",
    "sampler_lrn_f16x2.hip", "sampler_lrn_f16x1.hip", "sampler_lrn_bf16x1.hip", "mlp.hip", "static_ws.hip",
    "sampler_mhgd_f64.hip", "sampler_mhgd_f16x2.hip", "sampler_mhgd_bf16x1.hip", "gx_loop.hip",
]


def _compile(src, verbose):
    obj = os.path.join(BUILD, src + ".o")
    cmd = [HIPCC] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    msgs = [l for l in (r.stdout + r.stderr).splitlines() if "packed-fp32-ops" not in l]
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, "\n".join(msgs)))
    if verbose and msgs:
        print("\n".join(msgs), file=sys.stderr)
    return obj


def build(verbose=False, jobs=None):
    os.makedirs(BUILD, exist_ok=True)
    jobs = jobs or min(len(SOURCES), max(1, os.cpu_count() or 1))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    tmp = LIB + ".tmp"
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + objs,
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
