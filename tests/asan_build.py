"""Builds of the host code under AddressSanitizer, for the CPU sanitizer tests (never loaded by
a GPU run): libqh_asan.so (the library with its host pass instrumented; device code as usual)
and the oracle's liborc_asan.so. Run them with the matching runtime preloaded (see runtime()).

    python -m tests.asan_build
"""
from __future__ import annotations

import concurrent.futures as cf
import glob
import os
import subprocess

from paper_2103_06737_amd.build import CSRC, FLAGS, HIPCC, SOURCES

HERE = os.path.dirname(os.path.abspath(__file__))
OUT_DIR = os.path.join(HERE, "_build_asan")
LIB = os.path.join(OUT_DIR, "libqh_asan.so")
# host pass only: each sanitizer flag goes to the host compilation
HOST_ASAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]


def _stale(target: str, sources) -> bool:
    if not os.path.exists(target):
        return True
    t = os.path.getmtime(target)
    return any(os.path.getmtime(s) > t for s in sources)


def build_library() -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES] + glob.glob(os.path.join(CSRC, "*.h"))
    if not _stale(LIB, srcs):
        return LIB
    os.makedirs(OUT_DIR, exist_ok=True)

    def comp(src):
        obj = os.path.join(OUT_DIR, os.path.splitext(src)[0] + ".o")
        subprocess.check_call([HIPCC, *FLAGS, *HOST_ASAN, "-c", os.path.join(CSRC, src), "-o", obj])
        return obj

    with cf.ThreadPoolExecutor(max_workers=5) as ex:
        objs = list(ex.map(comp, SOURCES))
    tmp = LIB + ".tmp"
    subprocess.check_call([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-shared-libsan", *HOST_ASAN, "-o",
                           tmp, *objs])
    os.replace(tmp, LIB)
    return LIB


def build_oracle() -> str:
    root = os.path.dirname(HERE)
    src = os.path.join(root, "oracle", "pic.c")
    out = os.path.join(root, "oracle", "_build", "liborc_asan.so")
    if _stale(out, [src]):
        os.makedirs(os.path.dirname(out), exist_ok=True)
        subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                               "-fsanitize=address", "-fno-omit-frame-pointer", "-o", out, src, "-lm"])
    return out


def runtime(kind: str) -> str:
    """The sanitizer runtime to preload: 'clang' for the library (hipcc's host pass), 'gcc' for
    the oracle."""
    if kind == "gcc":
        return subprocess.check_output(["gcc", "-print-file-name=libasan.so"], text=True).strip()
    found = glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so")
    if not found:
        raise FileNotFoundError("no clang AddressSanitizer runtime under /opt/rocm/llvm")
    return found[0]


if __name__ == "__main__":
    print(build_library())
    print(build_oracle())
