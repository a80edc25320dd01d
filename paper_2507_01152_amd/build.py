"""Build the gfx950 HIP library libsonosim.so in-tree with hipcc."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
OBJ = os.path.join(HERE, "_build")
LIB = os.path.join(HERE, "lib", "libsonosim.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

SOURCES = ["physics.hip", "conv_mfma.hip", "recon.hip", "probe.hip", "noalloc.hip", "sonosim_api.cpp",
           "sonosim_batch.cpp", "surrogate.cpp"]

COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-I", INCLUDE, "-I", CSRC,
          # no packed FP32 instructions in generated code
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
# host-side files: plane geometry and tap tables without FMA contraction
HOST_EXTRA = ["-ffp-contract=off"]
# instrumented host code for the sanitizer test (device code is built as usual; the runtime comes from
# clang's shared ASan library, preloaded by the process that loads this build)
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]


def _compile(src: str, obj_dir: str, sanitize: bool) -> str:
    obj = os.path.join(obj_dir, os.path.splitext(src)[0] + ".o")
    flags = COMMON + (HOST_EXTRA if src.endswith(".cpp") or src == "noalloc.hip" else [])
    if sanitize:
        flags = flags + SANITIZE
    cmd = [HIPCC] + flags + ["-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError(f"hipcc failed on {src}")
    return obj


def build(verbose: bool = False, sanitize: bool = False, lib: str = LIB, obj_dir: str = OBJ) -> str:
    """Compile every source for gfx950 and link the shared library (sanitize: host code under
    AddressSanitizer and UndefinedBehaviorSanitizer, into `lib`, for the CPU-side sanitizer test)."""
    os.makedirs(obj_dir, exist_ok=True)
    os.makedirs(os.path.dirname(lib), exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(8, len(SOURCES))) as ex:
        objs = list(ex.map(lambda s: _compile(s, obj_dir, sanitize), SOURCES))
    tmp = lib + ".tmp%d" % os.getpid()
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-o", tmp] + objs
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("link failed")
    os.replace(tmp, lib)
    if verbose:
        print("built", lib)
    return lib


if __name__ == "__main__":
    build(verbose=True)
