"""Build libsem.so in-tree with hipcc for gfx950.

Every source is compiled to an object in parallel, then linked into
``paper_2312_09888_amd/libsem.so``.  ``python -m paper_2312_09888_amd.build``
runs it from the command line.
"""

import concurrent.futures
import hashlib
import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OBJ = os.path.join(PKG, "_build")
LIB = os.path.join(PKG, "libsem.so")

SOURCES = ["sem_api.cpp", "sem_basis.cpp", "sem_mctable.cpp", "sem_kernels.hip", "sem_c0.hip",
           "sem_ae.hip", "sem_bw.hip",
           "sem_noalloc.hip"]

ARCH = "gfx950"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # packed FP32 instructions are disabled for all device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
    "-Wall", "-Wno-unused-result",
]


def source_sha256():
    """SHA-256 of the library's sources as they are now: every file of csrc/
    (.hip, .cpp, .h) in name order, each as its name then its bytes, then
    include/sem.h the same way.  The build stores it in the library
    (sem_build_info), so a loaded library can be matched to the tree."""
    h = hashlib.sha256()
    files = sorted(f for f in os.listdir(CSRC) if f.endswith((".hip", ".cpp", ".h")))
    paths = [os.path.join(CSRC, f) for f in files] + [os.path.join(ROOT, "include", "sem.h")]
    for path in paths:
        h.update(os.path.basename(path).encode())
        with open(path, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _hip_version():
    res = subprocess.run([HIPCC, "--version"], capture_output=True, text=True)
    for line in res.stdout.splitlines():
        if line.startswith("HIP version:"):
            return line.split(":", 1)[1].strip()
    return "unknown"


def _compile(src, defines=()):
    obj = os.path.join(OBJ, os.path.splitext(src)[0] + ".o")
    cmd = [HIPCC] + COMMON + list(defines) + ["-c", os.path.join(CSRC, src), "-o", obj]
    if src.endswith(".cpp"):
        cmd.insert(1, "-xhip")
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{res.stdout}\n{res.stderr}")
    return obj, res.stderr


def build(verbose=False):
    """Compile every source and link libsem.so (always rebuilds)."""
    if not os.path.exists(HIPCC):
        raise RuntimeError(f"hipcc not found at {HIPCC}")
    os.makedirs(OBJ, exist_ok=True)
    # the build record compiled into sem_api.cpp (sem_build_info)
    record = [f'-DSEM_SOURCES_SHA256="{source_sha256()}"',
              f'-DSEM_HIP_VERSION="{_hip_version()}"']
    with concurrent.futures.ThreadPoolExecutor(max_workers=len(SOURCES)) as ex:
        results = list(ex.map(lambda src: _compile(src, record if src == "sem_api.cpp" else ()),
                              SOURCES))
    if verbose:
        for (obj, err) in results:
            if err.strip():
                print(err, file=sys.stderr)
    tmp = LIB + ".tmp"
    cmd = [HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", tmp] + \
        [o for o, _ in results]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stdout}\n{res.stderr}")
    os.replace(tmp, LIB)
    return LIB


def clean():
    shutil.rmtree(OBJ, ignore_errors=True)
    if os.path.exists(LIB):
        os.remove(LIB)


if __name__ == "__main__":
    print(build(verbose=True))
