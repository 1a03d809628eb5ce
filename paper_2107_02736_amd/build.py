"""Build step of the HIP library libdeann.so (gfx950), in-tree.

    python -m paper_2107_02736_amd.build      # or build() from Python
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libdeann.so")
# measurement support (bench.py --ceilings), outside the DEANN library
CEILING_LIB = os.path.join(HERE, "libdeann_ceiling.so")
OBJDIR = os.path.join(HERE, "_build")
SOURCES = ["prep.hip", "kde_fwd.hip", "cert.hip", "knn.hip", "sample.hip", "backward.hip", "ivf.hip",
           "hybrid.hip", "api.cpp"]
ARCH = "gfx950"
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    # no packed FP32 instructions anywhere in the device code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function",
]


def _hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def _compile(src: str) -> str:
    obj = os.path.join(OBJDIR, src + ".o")
    lang = ["-x", "hip"] if src.endswith(".cpp") else []
    cmd = [_hipcc(), *FLAGS, *lang, "-c", os.path.join(CSRC, src), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for {src}:\n{res.stderr}")
    return obj


def _link(objs, out: str) -> None:
    tmp = out + ".tmp"
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"link failed:\n{res.stderr}")
    os.replace(tmp, out)


def build(verbose: bool = False) -> str:
    """Compile every source and link libdeann.so (and the measurement library
    libdeann_ceiling.so); returns the path of libdeann.so."""
    os.makedirs(OBJDIR, exist_ok=True)
    with ThreadPoolExecutor(max_workers=min(6, os.cpu_count() or 1)) as ex:
        objs = list(ex.map(_compile, SOURCES + ["ceiling.hip"]))
    _link(objs[:-1], LIB)
    _link(objs[-1:], CEILING_LIB)
    if verbose:
        print(f"built {LIB} and {CEILING_LIB}")
    return LIB


ASAN_LIB = os.path.join(OBJDIR, "libdeann_asan.so")


def asan_runtime() -> str | None:
    """Path of the host AddressSanitizer runtime of hipcc's clang, or None."""
    res = subprocess.run([_hipcc(), "-print-file-name=libclang_rt.asan-x86_64.so"],
                         capture_output=True, text=True)
    path = res.stdout.strip()
    return path if res.returncode == 0 and os.path.isabs(path) and os.path.exists(path) else None


def build_asan(verbose: bool = False) -> str:
    """The C ABI layer (api.cpp) with host AddressSanitizer, linked with the
    kernels' objects of the last build() into _build/libdeann_asan.so.  Only the
    host code is instrumented (the device code is built as usual).  Load it
    with the runtime preloaded (LD_PRELOAD=asan_runtime()) and DEANN_LIB set."""
    os.makedirs(OBJDIR, exist_ok=True)
    obj = os.path.join(OBJDIR, "api_asan.o")
    cmd = [_hipcc(), "-O1", "-g", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer",
           "-x", "hip", "-c", os.path.join(CSRC, "api.cpp"), "-o", obj]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"hipcc failed for api.cpp (asan):\n{res.stderr}")
    others = [os.path.join(OBJDIR, src + ".o") for src in SOURCES if src != "api.cpp"]
    missing = [o for o in others if not os.path.exists(o)]
    if missing:
        raise RuntimeError(f"run build() first: missing {missing}")
    # the sanitizer's symbols stay undefined in the library: the runtime is
    # preloaded into the process that loads it
    cmd = [_hipcc(), f"--offload-arch={ARCH}", "-shared", "-fPIC", obj, *others, "-o", ASAN_LIB]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError(f"asan link failed:\n{res.stderr}")
    if verbose:
        print(f"built {ASAN_LIB}")
    return ASAN_LIB


if __name__ == "__main__":
    build(verbose=True)
    if len(sys.argv) > 1 and sys.argv[1] == "asan":
        build_asan(verbose=True)
    sys.exit(0)
