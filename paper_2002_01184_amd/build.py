"""Compile libhmc.so (HIP for gfx950) in-tree.

    python -m paper_2002_01184_amd.build

Every .hip source under csrc/ is compiled with hipcc for gfx950 only, with
packed-FP32 instructions disabled, and linked into
paper_2002_01184_amd/libhmc.so.
"""
from __future__ import annotations

import glob
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libhmc.so")
BUILD_DIR = os.path.join(ROOT, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = ["-std=c++17", "-O3", "-fPIC", "--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang",
         "-packed-fp32-ops", "-munsafe-fp-atomics", "-Wall", "-Wno-unused-function",
         "-I" + os.path.join(ROOT, "include")]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


# Host-runtime sanitizer build: AddressSanitizer and UndefinedBehaviorSanitizer on
# the host side of every source only (the kernels are built as usual); the
# resulting library needs the compiler's ASan runtime preloaded.
HOST_SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                 "-Xarch_host", "-fno-omit-frame-pointer", "-g"]


def build(verbose: bool = False, jobs: int = 8, sanitize: bool = False, out: str = LIB,
          build_dir: str = BUILD_DIR) -> str:
    os.makedirs(build_dir, exist_ok=True)
    srcs = sources()
    objs = [os.path.join(build_dir, os.path.basename(s) + ".o") for s in srcs]
    san = HOST_SANITIZE if sanitize else []

    def compile_one(pair):
        src, obj = pair
        cmd = [HIPCC, *FLAGS, *san, "-c", src, "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{r.stdout}\n{r.stderr}")
        if verbose and r.stderr.strip():
            print(r.stderr, file=sys.stderr)
        return obj

    with ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(compile_one, zip(srcs, objs)))
    tmp = out + ".tmp"
    link_san = [*HOST_SANITIZE[:4], "-shared-libsan"] if sanitize else []
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", *link_san, "-o", tmp, *objs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
