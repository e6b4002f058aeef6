"""The oracle and the host runtime under AddressSanitizer and
UndefinedBehaviorSanitizer, on the CPU.

- The oracle pins (tests/test_oracle_pins.py) run against the oracle built
  with gcc's sanitizers (oracle/build.py --sanitize), with libasan preloaded.
- The boundary checks (tests/test_abi.py: symbol exports, parameter
  validation, argument errors of every entry point) run against the library
  whose host runtime is built with clang's sanitizers
  (paper_1110_5004_amd/build.py --sanitize), with clang's ASan runtime
  preloaded.

Each runs in a subprocess of its own (the two ASan runtimes cannot share a
process).  Undefined behaviour aborts, ASan stops at its first report, and
either shows up as a failing exit status or a report in the output.  The
Laplace-law pin (70 s under the sanitizers, the same kernels as the flat
interface pin on a larger grid) is left out to keep the suite short."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
REPORTS = ("ERROR: AddressSanitizer", "runtime error:", "ERROR: LeakSanitizer")


def _run(args, env_extra, timeout):
    env = dict(os.environ)
    env.update(env_extra)
    env.update(ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1",
               OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, "-m", "pytest", *args, "-q", "-x", "-p", "no:cacheprovider"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=timeout)
    out = r.stdout + r.stderr
    assert r.returncode == 0 and not any(s in out for s in REPORTS), out[-4000:]
    return out


def test_oracle_pins_under_sanitizers():
    sys.path.insert(0, ROOT)
    from oracle import build as ob
    libasan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True,
                             text=True).stdout.strip()
    if not os.path.isabs(libasan) or not os.path.exists(libasan):
        pytest.skip("gcc's libasan is not installed")
    lib = ob.build_sanitized()
    out = _run(["tests/test_oracle_pins.py", "-k", "not laplace"],
               dict(LD_PRELOAD=libasan, LBM_ORACLE_LIB=lib), timeout=600)
    assert " passed" in out


def test_host_runtime_under_sanitizers():
    sys.path.insert(0, ROOT)
    from paper_1110_5004_amd import build as pb
    rts = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not rts:
        pytest.skip("clang's ASan runtime is not installed")
    lib = pb.build_host_sanitized()
    out = _run(["tests/test_abi.py"], dict(LD_PRELOAD=rts[-1], LBM_HIP_LIB=lib), timeout=300)
    assert " passed" in out
