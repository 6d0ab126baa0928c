"""Build the FP64 CPU oracle (test infrastructure) into oracle/liboracle.so.

Plain gcc, OpenMP over chains, IEEE arithmetic (no fast-math, no FMA
contraction) so results do not depend on the compiler's instruction choice.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "liboracle.so")


def build(verbose: bool = False, sanitize: bool = False, out: str = LIB) -> str:
    """sanitize: AddressSanitizer + UndefinedBehaviorSanitizer build (load it with
    gcc's libasan preloaded and ORACLE_LIB_PATH pointing at `out`)."""
    src = os.path.join(HERE, "oracle.c")
    tmp = out + ".tmp"
    san = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"] \
        if sanitize else []
    cmd = ["gcc", "-std=c11", "-O2", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
           "-fno-fast-math", "-D_GNU_SOURCE", "-Wall", "-Wextra", *san, "-o", tmp, src, "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
