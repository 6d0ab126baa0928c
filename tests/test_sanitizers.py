"""AddressSanitizer + UndefinedBehaviorSanitizer builds of the host code, run on
the CPU:

  * the FP64 oracle (plain C, gcc), driven by the oracle's own pin tests in a
    child process with gcc's ASan runtime preloaded;
  * the host runtime of libhmc.so (argument validation, workspace carving,
    error reporting), built with the sanitizers on the host side of every
    source only, driven by the C-ABI tests with clang's ASan runtime preloaded.

A sanitizer report makes the child process fail (UBSan does not recover), so
the test checks the exit status and that no report was printed.
"""
import glob
import os
import shutil
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path.insert(0, ROOT)

REPORTS = ("ERROR: AddressSanitizer", "runtime error:", "ERROR: LeakSanitizer")


def _run_child(env_extra, tests, timeout):
    env = dict(os.environ)
    env.update(env_extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=0:exitcode=23"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", *tests],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=timeout)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    for rep in REPORTS:
        assert rep not in out, out[-4000:]
    return out


def test_oracle_under_asan_ubsan(tmp_path):
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if shutil.which("gcc") is None or not os.path.isabs(asan):
        pytest.skip("gcc's ASan runtime unavailable")
    from oracle import build as ob
    lib = ob.build(sanitize=True, out=str(tmp_path / "liboracle_san.so"))
    tests = [os.path.join("tests", f) for f in ("test_oracle_hmc.py", "test_oracle_adapt.py",
                                                "test_oracle_remc.py", "test_oracle_transform.py",
                                                "test_oracle_nuts.py", "test_oracle_rng.py")]
    _run_child({"LD_PRELOAD": asan, "ORACLE_LIB_PATH": lib, "OMP_NUM_THREADS": "4"}, tests, timeout=900)


def test_host_runtime_under_asan_ubsan(tmp_path):
    rt = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not rt or not os.path.exists("/opt/rocm/bin/hipcc"):
        pytest.skip("hipcc or clang's ASan runtime unavailable")
    from paper_2002_01184_amd import build as hb
    lib = hb.build(sanitize=True, out=str(tmp_path / "libhmc_san.so"), build_dir=str(tmp_path / "obj"))
    _run_child({"LD_PRELOAD": rt[-1], "HMC_LIB_PATH": lib}, [os.path.join("tests", "test_abi.py")], timeout=300)
