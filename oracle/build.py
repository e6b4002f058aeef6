"""Build the FP64 CPU oracle (test infrastructure) as a shared library.

Plain C, gcc, no fast-math and no FMA contraction, OpenMP over independent
per-node loops.  The output lands in oracle/_build/liblbm_oracle.so.
"""
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUT_DIR, "liblbm_oracle.so")
SOURCES = [os.path.join(HERE, "lbm_oracle.c")]


def build(extra_flags=(), out=LIB, verbose=False):
    """Compile the oracle; returns the library path.  extra_flags lets the
    mutation tests build deliberately broken copies under another name."""
    os.makedirs(os.path.dirname(out), exist_ok=True)
    cmd = ["gcc", "-std=c99", "-O2", "-fPIC", "-shared", "-fopenmp",
           "-ffp-contract=off", "-fno-fast-math", "-Wall", "-Wextra",
           *extra_flags, *SOURCES, "-o", out + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


SAN_LIB = os.path.join(OUT_DIR, "liblbm_oracle_san.so")


def build_sanitized(verbose=False):
    """The oracle with AddressSanitizer and UndefinedBehaviorSanitizer (gcc's
    runtimes; a process loading it must preload libasan).  Any undefined
    behaviour aborts."""
    return build(("-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                  "-fno-sanitize-recover=undefined"), out=SAN_LIB, verbose=verbose)


def ensure_built():
    """Build when the library is missing or older than a source or header."""
    deps = SOURCES + [os.path.join(HERE, "lbm_oracle.h")]
    if (not os.path.exists(LIB) or
            os.path.getmtime(LIB) < max(os.path.getmtime(d) for d in deps)):
        build()
    return LIB


if __name__ == "__main__":
    if "--sanitize" in sys.argv:
        build_sanitized(verbose=True)
    else:
        build(verbose=True)
    sys.exit(0)
