"""Build step of the HIP library: hipcc for gfx950 -> paper_2011_05749_amd/_lib/libsfft.so.

    python paper_2011_05749_amd/build.py

Every translation unit is compiled to an object of its own (in parallel),
then the objects are linked into one shared library.  Objects are kept under
``_lib/obj`` keyed by a hash of their source, the headers and the flags, and
reused when nothing changed, unless ``force`` is set.  Packed-FP32
instructions are disabled for all device code
(``-Xclang -target-feature -Xclang -packed-fp32-ops``); hipcc's host pass
warns that it does not know the feature, which is harmless.
"""
from __future__ import annotations

import hashlib
import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT = os.path.join(HERE, "_lib", "libsfft.so")
OBJ = os.path.join(HERE, "_lib", "obj")
SOURCES = ["sfft_level0.hip", "sfft_ffast.hip", "sfft_tree.hip", "sfft_jump.hip", "sfft_col.hip",
           "sfft_colres.hip", "sfft_finalize.hip", "sfft_noalloc.hip", "sfft_host.cpp",
           "sfft_server.cpp", "sfft_pack.hip"]
HEADERS = [os.path.join(CSRC, "sfft_internal.h"), os.path.join(CSRC, "sfft_device.h"),
           os.path.join(CSRC, "sfft_host.h"),
           os.path.join(ROOT, "include", "sfft.h")]
ARCH = "gfx950"
FLAGS = [f"--offload-arch={ARCH}", "-O3", "-std=c++17", "-fPIC",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-Wno-unused-command-line-argument", "-Wno-unused-function"]


def _key(src: str) -> str:
    h = hashlib.sha256(" ".join(FLAGS).encode())
    for f in [os.path.join(CSRC, src), *HEADERS]:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def build(verbose: bool = False, jobs: int | None = None, force: bool = False) -> str:
    hipcc = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
    os.makedirs(OBJ, exist_ok=True)
    tag = os.getpid()
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]

    def compile_one(src):
        stem = os.path.splitext(src)[0]
        obj = os.path.join(OBJ, f"{stem}.{_key(src)}.o")
        if os.path.exists(obj) and not force:
            return src, obj, None
        tmp = f"{obj}.{tag}.tmp"
        cmd = [hipcc, *FLAGS, "-I", os.path.join(ROOT, "include"), "-c",
               os.path.join(CSRC, src), "-o", tmp]
        if verbose:
            print(" ".join(cmd), flush=True)
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode == 0:
            for old in os.listdir(OBJ):
                if old.startswith(stem + ".") and old.endswith(".o"):
                    os.remove(os.path.join(OBJ, old))
            os.replace(tmp, obj)
        return src, obj, r

    jobs = jobs or min(len(srcs), max(1, os.cpu_count() or 1), 16)
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        results = list(ex.map(compile_one, srcs))
    objs = []
    failed = False
    for src, obj, r in results:
        if r is not None and r.returncode != 0:
            sys.stderr.write(f"--- {src}\n{r.stdout}{r.stderr}")
            failed = True
        objs.append(obj)
    if failed:
        raise RuntimeError("hipcc build of libsfft.so failed")
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    tmp = f"{OUT}.{tag}.tmp"
    cmd = [hipcc, f"--offload-arch={ARCH}", "-shared", "-fPIC", *objs, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc link of libsfft.so failed")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True, force="--force" in sys.argv))
