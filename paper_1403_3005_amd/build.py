"""Builds libnkbc.so (the HIP library behind include/nk_bc.h) in-tree for gfx950.

Each source is compiled to an object of its own (in parallel; every kernel is
launched from the file that defines it, so no relocatable device code is
needed) and the objects are linked into one shared library.
"""
from __future__ import annotations

import os
import subprocess
import tempfile
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libnkbc.so")
SOURCES = ["nk_kernels.hip", "nk_lds.hip", "nk_bfs.hip", "nk_relabel.hip", "nk_directed.hip", "nk_api.hip",
           "nk_server.hip", "nk_tune.hip", "nk_multi.hip", "nk_group.hip", "nk_noalloc.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-munsafe-fp-atomics",
    # packed FP32 instructions stay off
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]


def _clean(text: str) -> str:
    return "\n".join(l for l in text.splitlines() if "packed-fp32-ops" not in l)


def build(verbose: bool = False) -> str:
    inc = ["-I", os.path.join(os.path.dirname(HERE), "include")]
    with tempfile.TemporaryDirectory(prefix="nkbuild") as tmpdir:
        def compile_one(src):
            obj = os.path.join(tmpdir, os.path.basename(src) + ".o")
            res = subprocess.run([HIPCC] + FLAGS + inc + ["-c", "-o", obj, src], stdout=subprocess.PIPE,
                                 stderr=subprocess.STDOUT, text=True)
            return src, obj, res.returncode, _clean(res.stdout)

        srcs = sources()
        workers = max(1, min(len(srcs), int(os.environ.get("MAX_JOBS", os.cpu_count() or 1))))
        with ThreadPoolExecutor(max_workers=workers) as ex:
            results = list(ex.map(compile_one, srcs))
        failed = [r for r in results if r[2] != 0]
        if failed:
            raise RuntimeError("hipcc failed:\n" + "\n".join(f"{r[0]}:\n{r[3]}" for r in failed))
        if verbose:
            for r in results:
                if r[3].strip():
                    print(r[3])
        tmp = LIB + ".tmp%d" % os.getpid()
        res = subprocess.run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + [r[1] for r in results]
                             + ["-lpthread"], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
        if res.returncode != 0:
            raise RuntimeError("link failed:\n" + _clean(res.stdout))
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
