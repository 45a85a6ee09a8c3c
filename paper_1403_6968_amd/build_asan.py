"""Host-side AddressSanitizer build of liblinview (CPU diagnostics).

The host code of every translation unit (argument validation, workspace
layouts, the C ABI, the serving and batching bookkeeping) is instrumented
with AddressSanitizer; device code is compiled as in build_lib.  The library
goes to _build/asan/liblinview.so.  Loading it needs the sanitizer runtime
preloaded into the host process (asan_runtime() finds it).
"""

from __future__ import annotations

import glob
import os
import shutil
from concurrent.futures import ThreadPoolExecutor

from paper_1403_6968_amd import build_lib

OUT_DIR = os.path.join(build_lib.BUILD, "asan")
LIB = os.path.join(OUT_DIR, "liblinview.so")
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer"]


def asan_runtime() -> str | None:
    """The clang AddressSanitizer runtime that matches hipcc, if present."""
    hits = sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/*/libclang_rt.asan-x86_64.so")) + \
        sorted(glob.glob("/opt/rocm/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    return hits[-1] if hits else None


def build() -> str:
    """Compile every source with the host sanitizer and link the library."""
    os.makedirs(OUT_DIR, exist_ok=True)
    objs, cmds = [], []
    for src in build_lib.SOURCES:
        obj = os.path.join(OUT_DIR, src.replace(".hip", ".o"))
        objs.append(obj)
        cmds.append([build_lib.HIPCC, *build_lib.FLAGS, *HOST_SAN, "-c", os.path.join(build_lib.CSRC, src), "-o", obj])
    with ThreadPoolExecutor(max_workers=min(len(cmds), 4)) as ex:
        list(ex.map(build_lib._run, cmds))
    tmp = LIB + ".tmp"
    build_lib._run([build_lib.HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *HOST_SAN, *objs, "-o", tmp])
    shutil.move(tmp, LIB)
    for o in objs:
        os.remove(o)
    return LIB


if __name__ == "__main__":
    print(build())
