"""Build libhc.so (the C-ABI library) for gfx950 with hipcc.

Usage: python -m paper_2602_18741_amd.build [-v] [--sanitize]
Every call compiles (the sources are few and hipcc is fast); objects go to
_build/ under the package, the library next to this file.
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "libhc.so")
BUILD_DIR = os.path.join(PKG, "_build")
SOURCES = ["hc_api.hip", "k_latent.hip", "k_spectral.hip", "k_records.hip", "k_encode.hip",
           "k_codec.hip", "k_gen.hip", "k_upsample.hip",
           "k_upsample_train.hip", "k_probe.hip"]
ARCH = "gfx950"

# Packed FP32 instructions are disabled for all device code: hipcc then emits
# scalar FP32 ops only.
DEVICE_FLAGS = ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
COMMON = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", "-Wall", "-Wno-unused-function",
          "-Wno-unused-command-line-argument", "-Wno-unknown-cuda-version"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found (ROCm is required to build the library)")


def _run(cmd, verbose):
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"command failed ({r.returncode}): {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    if verbose and r.stderr.strip():
        print(r.stderr, file=sys.stderr)
    return r


# Host-only sanitizers for the checking build: device code is compiled as
# usual, the host code (argument validation, launch set-up) with AddressSanitizer
# and UndefinedBehaviorSanitizer.
SANITIZE = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=all"]
SANITIZED_OUT = os.path.join(BUILD_DIR, "sanitized", "libhc.so")


def asan_runtime() -> str:
    """Path of the AddressSanitizer runtime of hipcc's clang (to preload into
    a process that loads the sanitized library)."""
    r = subprocess.run([hipcc(), "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True,
                       text=True)
    path = r.stdout.strip()
    if r.returncode != 0 or not os.path.isfile(path):
        raise RuntimeError("AddressSanitizer runtime of hipcc's clang not found")
    return path


def build(verbose: bool = False, jobs: int | None = None, sanitize: bool = False) -> str:
    """Compile every source and link the library: libhc.so next to this file,
    or with sanitize the host-sanitized copy under _build/sanitized/ (for
    checking runs on the CPU; the product loads only libhc.so)."""
    cc = hipcc()
    odir = os.path.dirname(SANITIZED_OUT) if sanitize else BUILD_DIR
    out = SANITIZED_OUT if sanitize else OUT
    extra = SANITIZE if sanitize else []
    os.makedirs(odir, exist_ok=True)
    objs = []
    cmds = []
    for src in SOURCES:
        obj = os.path.join(odir, src.replace(".hip", ".o"))
        objs.append(obj)
        cmds.append([cc, *COMMON, *DEVICE_FLAGS, *extra, "-c", os.path.join(CSRC, src), "-o", obj])
    jobs = jobs or min(len(cmds), max(1, (os.cpu_count() or 2)))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        list(ex.map(lambda c: _run(c, verbose), cmds))
    tmp = out + ".tmp"
    _run([cc, "-shared", f"--offload-arch={ARCH}", *extra, "-o", tmp, *objs], verbose)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, sanitize="--sanitize" in sys.argv))
