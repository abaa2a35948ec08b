"""Host-sanitized build of libgwd for the CPU tests of the C ABI: every source compiled as for the
product library, with AddressSanitizer and UndefinedBehaviorSanitizer on the host code only (the
gfx950 device code is built as usual). Load it in a process started with the sanitizer runtime
preloaded (runtime_path()); nothing on the product path uses this library."""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

from paper_2201_11133_amd import build as b

OUT_DIR = os.path.join(os.path.dirname(b.HERE), "_build", "asan")
OUT = os.path.join(OUT_DIR, "libgwd_asan.so")
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-g"]


def runtime_path() -> str:
    clang = os.path.join(os.path.dirname(b.HIPCC), "..", "llvm", "bin", "clang++")
    if not os.path.exists(clang):
        clang = "/opt/rocm/llvm/bin/clang++"
    r = subprocess.run([clang, "-print-file-name=libclang_rt.asan-x86_64.so"], capture_output=True, text=True)
    return r.stdout.strip()


def build() -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    srcs = b.sources()

    def comp(src):
        obj = os.path.join(OUT_DIR, os.path.basename(src) + ".o")
        r = subprocess.run([b.HIPCC, "-x", "hip", "-c", src, "-o", obj] + b.FLAGS + HOST_SAN,
                           capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr[-4000:]}")
        return obj

    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(comp, srcs))
    r = subprocess.run([b.HIPCC, "-shared", "-o", OUT] + objs + [f"--offload-arch={b.ARCH}", "-fPIC"] + HOST_SAN,
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stdout + r.stderr)
    return OUT


if __name__ == "__main__":
    print(build())
    sys.stdout.flush()
