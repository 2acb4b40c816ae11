"""Builds libgw.so (the HIP path, gfx950) and gwinputs/libgwgen.so.

Every source is compiled with hipcc for gfx950 with packed FP32 ops disabled;
objects go to _build/ and the shared libraries sit next to their Python
bindings.  ``python -m paper_2104_09857_amd.build`` or ``build()``.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2104_09857_amd")
SRC = os.path.join(PKG, "csrc")
BUILD = os.path.join(ROOT, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
         "-I" + os.path.join(ROOT, "include")]
SOURCES = ["common.hip", "gt.hip", "chi.hip", "screen.hip", "sigma.hip", "screener.hip", "qp.cpp",
           "integrals.hip"]
LIBS = ["-lrocsolver", "-lrocblas"]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + r.stdout + r.stderr)
    return r


def _compile(src, out, extra=()):
    _run([HIPCC, *FLAGS, *extra, "-c", src, "-o", out])
    return out


def build(verbose: bool = False) -> None:
    os.makedirs(BUILD, exist_ok=True)
    jobs = []
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        for s in SOURCES:
            src = os.path.join(SRC, s)
            obj = os.path.join(BUILD, os.path.splitext(s)[0] + ".o")
            extra = ("-x", "hip") if s.endswith(".hip") else ()
            jobs.append(ex.submit(_compile, src, obj, extra))
        gen_obj = os.path.join(BUILD, "gwgen.o")
        jobs.append(ex.submit(_compile, os.path.join(ROOT, "gwinputs", "csrc", "gwgen.hip"), gen_obj,
                              ("-x", "hip")))
        objs = [j.result() for j in jobs]
    lib_objs = objs[:-1]
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o", os.path.join(PKG, "libgw.so"),
          *lib_objs, "-L/opt/rocm/lib", *LIBS, "-Wl,-rpath,/opt/rocm/lib"])
    _run([HIPCC, f"--offload-arch={ARCH}", "-shared", "-fPIC", "-o",
          os.path.join(ROOT, "gwinputs", "libgwgen.so"), objs[-1]])
    if verbose:
        print("built", os.path.join(PKG, "libgw.so"))


if __name__ == "__main__":
    build(verbose=True)
    sys.exit(0)
