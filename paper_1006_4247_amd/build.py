"""Build libhsgpt.so (HIP, gfx950) in-tree with hipcc.

Every translation unit is compiled in parallel, then linked into one shared
library next to this file.  Packed FP32 instructions are disabled
(-packed-fp32-ops) on purpose: all HIP code is built with that flag.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "libhsgpt.so")
BUILD_DIR = os.path.join(HERE, "_build")
SOURCES = ["abi.hip", "sweep_resident.hip", "sweep_stream.hip", "sweep_wave.hip", "exchange.hip",
           "decimate.hip", "coolheat.hip", "mlp.hip", "plan.hip", "sweep_batch.hip", "probe.hip"]
ARCH = os.environ.get("HSG_OFFLOAD_ARCH", "gfx950")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-I" + INCLUDE,
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    # no implicit contraction: every fused multiply-add is written out, so each
    # kernel instance evaluates exactly the stated operations (bitwise-equal results
    # across tile shapes and variants)
    "-ffp-contract=off",
    "-munsafe-fp-atomics", "-Wall", "-Wno-unused-function",
]


def _compile(src):
    obj = os.path.join(BUILD_DIR, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + FLAGS + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s\n%s" % (src, " ".join(cmd), r.stderr))
    return obj, r.stderr


def build(verbose=False):
    """Compile every HIP source for gfx950 and link libhsgpt.so (always rebuilds)."""
    os.makedirs(BUILD_DIR, exist_ok=True)
    with cf.ThreadPoolExecutor(max_workers=min(len(SOURCES), os.cpu_count() or 4)) as ex:
        results = list(ex.map(_compile, SOURCES))
    objs = [o for o, _ in results]
    if verbose:
        for _, err in results:
            if err.strip():
                sys.stderr.write(err)
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n%s\n%s" % (" ".join(cmd), r.stderr))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
