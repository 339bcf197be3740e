"""Build librkr.so (all HIP kernels + the C ABI) for gfx950 with hipcc.

Compiles each source to an object in ``_build/`` (skipped when up to date unless
``force``), then links the shared library next to this file's package.
"""
from __future__ import annotations

import os
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.dirname(HERE)
ROOT = os.path.dirname(PKG)
OUT = os.path.join(PKG, "librkr.so")
BUILD = os.path.join(ROOT, "_build")
SOURCES = ["count.hip", "exact.hip", "prep.hip", "select.hip", "query.hip", "mlp.hip", "paper_table.hip", "api.cpp"]
HEADERS = ["rkr_internal.h", "tile_common.h", "kernels.h", "query.h", "mlp.h", "paper_table.h"]
FLAGS = ["--offload-arch=gfx950", "-O3", "-fPIC", "-std=c++17", "-ffp-contract=off",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include"), "-I" + HERE, "-Wno-unused-result"]


def _obj(src: str) -> str:
    return os.path.join(BUILD, src + ".o")


def _stale(src: str) -> bool:
    o = _obj(src)
    if not os.path.exists(o):
        return True
    t = os.path.getmtime(o)
    deps = [os.path.join(HERE, src)] + [os.path.join(HERE, h) for h in HEADERS] + \
        [os.path.join(ROOT, "include", "rkr.h"), __file__]
    return any(os.path.getmtime(p) > t for p in deps)


def _compile(src: str) -> None:
    lang = ["-x", "hip"] if src.endswith(".cpp") else []
    cmd = ["hipcc", *FLAGS, *lang, "-c", os.path.join(HERE, src), "-o", _obj(src)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("hipcc failed for " + src)


def build(force: bool = False, jobs: int = 6) -> str:
    os.makedirs(BUILD, exist_ok=True)
    todo = [s for s in SOURCES if force or _stale(s)]
    with ThreadPoolExecutor(max_workers=max(1, jobs)) as ex:
        list(ex.map(_compile, todo))
    if force or todo or not os.path.exists(OUT):
        tmp = OUT + ".tmp%d" % os.getpid()
        cmd = ["hipcc", "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp,
               *[_obj(s) for s in SOURCES]]
        subprocess.check_call(cmd)
        os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(force="--force" in sys.argv))
