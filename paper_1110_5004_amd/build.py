"""Build the gfx950 library liblbm_hip.so from csrc/ with hipcc.

Every HIP source is compiled for gfx950 only, without fast-math and with the
packed-FP32 instructions disabled, then linked into one shared library that
exports the C ABI of include/lbm.h.
"""
import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_build")
LIB = os.path.join(OUT_DIR, "liblbm_hip.so")
SOURCES = ["lbm_runtime.cpp", "lbm_common.hip", "lbm_d2q9.hip", "lbm_d3q19.hip",
           "lbm_d3q19_march.hip"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

# -ffp-contract=on: a*b+c inside one expression becomes an FMA, decided by
# the front end per source expression, so every tile shape and the batched
# launch still compute each node to the same bits (no fast-math).
FLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-Wall", "-ffp-contract=on",
         "-Wno-unused-function", "-Xclang", "-target-feature", "-Xclang",
         "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), "-I", CSRC]


def _compile(src, verbose):
    obj = os.path.join(OUT_DIR, os.path.basename(src) + ".o")
    lang = ["-x", "hip"] if src.endswith((".hip", ".cpp")) else []
    cmd = [HIPCC, *FLAGS, *lang, "-c", os.path.join(CSRC, src), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {src}:\n{r.stdout}\n{r.stderr}")
    warn = "\n".join(l for l in r.stderr.splitlines()
                     if "packed-fp32-ops" not in l and l.strip())
    return obj, warn


def build(verbose=False, jobs=None):
    """Compile every source and link; returns the library path."""
    os.makedirs(OUT_DIR, exist_ok=True)
    jobs = jobs or min(len(SOURCES), os.cpu_count() or 4, 16)
    with cf.ThreadPoolExecutor(jobs) as ex:
        results = list(ex.map(lambda s: _compile(s, verbose), SOURCES))
    for _, warn in results:
        if warn and verbose:
            print(warn, file=sys.stderr)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC",
           *[o for o, _ in results], "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


SAN_LIB = os.path.join(OUT_DIR, "liblbm_hip_hostsan.so")
# host code only: -Xarch_host keeps the sanitizers off the gfx950 code
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host",
            "-fno-omit-frame-pointer"]


def build_host_sanitized(verbose=False):
    """The library with AddressSanitizer and UndefinedBehaviorSanitizer on the
    host runtime (parameter validation, layout, argument checks of every
    entry point; lbm_runtime.cpp), linked with the kernels of the normal
    build.  A process loading it must preload clang's ASan runtime
    (libclang_rt.asan-x86_64.so of /opt/rocm/llvm)."""
    if not all(os.path.exists(os.path.join(OUT_DIR, s + ".o")) for s in SOURCES):
        build(verbose=verbose)
    obj = os.path.join(OUT_DIR, "lbm_runtime_hostsan.o")
    cmd = [HIPCC, *FLAGS, *HOST_SAN, "-g", "-x", "hip", "-c",
           os.path.join(CSRC, "lbm_runtime.cpp"), "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on lbm_runtime.cpp:\n{r.stdout}\n{r.stderr}")
    objs = [obj] + [os.path.join(OUT_DIR, s + ".o") for s in SOURCES if s != "lbm_runtime.cpp"]
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", *HOST_SAN, *objs,
           "-o", SAN_LIB + ".tmp"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(SAN_LIB + ".tmp", SAN_LIB)
    return SAN_LIB


if __name__ == "__main__":
    if "--sanitize" in sys.argv:
        print(build_host_sanitized(verbose="-v" in sys.argv))
    else:
        build(verbose="-v" in sys.argv)
        print(LIB)
