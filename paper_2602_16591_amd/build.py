"""Builds the HIP library libpswfe.so for gfx950 in-tree (paper_2602_16591_amd/_lib/).

Usage: python -m paper_2602_16591_amd.build   (or call build()).
"""
from __future__ import annotations

import os
import re
import shutil
import subprocess
import sys
import tempfile
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
OUT_DIR = os.path.join(HERE, "_lib")
LIB = os.path.join(OUT_DIR, "libpswfe.so")
ARCH = os.environ.get("PSWFE_ARCH", "gfx950")

SOURCES = ["host.cpp", "kernels.hip", "capi.hip"]
# particles.hip is compiled once per (precision, P range) listed in kernels.hpp
PARTICLE_SOURCE = "particles.hip"


def particle_instances() -> list[tuple[int, int, int]]:
    """(prec, lo, hi) of every particle-kernel instance, from PSWFE_PARTICLE_INSTANCES."""
    with open(os.path.join(CSRC, "kernels.hpp")) as f:
        text = f.read()
    body = text.split("#define PSWFE_PARTICLE_INSTANCES(X)", 1)[1].split("\n\n", 1)[0]
    inst = [tuple(int(v) for v in t) for t in re.findall(r"X\((\d+), (\d+), (\d+)\)", body)]
    if not inst:
        raise RuntimeError("no particle-kernel instances found in kernels.hpp")
    return inst


HIP_FLAGS = [
    "-O3", "-std=c++20", "-fPIC", f"--offload-arch={ARCH}",
    # packed FP32 instructions are kept out of the generated code
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics", "-Wall", "-Wno-unused-function",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = True, jobs: int | None = None) -> str:
    os.makedirs(OUT_DIR, exist_ok=True)
    cc = hipcc()
    jobs = jobs or max(1, min(16, os.cpu_count() or 1))
    units = [(src, os.path.splitext(src)[0] + ".o", []) for src in SOURCES]
    for prec, lo, hi in particle_instances():
        units.append((PARTICLE_SOURCE, f"particles_{prec}_{lo}.o",
                      [f"-DPSWFE_PREC={prec}", f"-DPSWFE_PLO={lo}", f"-DPSWFE_PHI={hi}"]))
    # longest compiles first
    units.sort(key=lambda u: 0 if u[0] == PARTICLE_SOURCE else 1)
    objs, running, failed = [], [], []
    t0 = time.time()

    def reap(block: bool) -> None:
        for item in list(running):
            name, proc, log = item
            if block or proc.poll() is not None:
                proc.wait()
                running.remove(item)
                log.seek(0)
                msg = log.read().decode(errors="replace").strip()
                log.close()
                if proc.returncode != 0:
                    failed.append((name, msg))
                elif verbose and msg:
                    print(msg)
                if block:
                    return

    for src, obj_name, defs in units:
        obj = os.path.join(OUT_DIR, obj_name)
        lang = ["-x", "hip"] if src.endswith(".hip") else ["-x", "c++"]
        cmd = [cc, *HIP_FLAGS, *defs, *lang, "-c", os.path.join(CSRC, src), "-o", obj,
               f"-I{os.path.join(ROOT, 'include')}"]
        if src.endswith(".cpp"):
            cmd = [c for c in cmd if not c.startswith("--offload-arch")]
        while len(running) >= jobs:
            reap(block=False)
            if len(running) >= jobs:
                time.sleep(0.2)
        log = tempfile.TemporaryFile()   # compiler output, read when the job ends
        running.append((obj_name, subprocess.Popen(cmd, stdout=log, stderr=subprocess.STDOUT), log))
        objs.append(obj)
    while running:
        reap(block=True)
    if failed:
        for name, msg in failed:
            sys.stderr.write(f"--- {name}\n{msg}\n")
        raise RuntimeError("compiling " + ", ".join(n for n, _ in failed) + " failed")
    tmp = LIB + ".tmp"
    cmd = [cc, "-shared", "-fPIC", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    if verbose:
        print(f"built {LIB} in {time.time() - t0:.1f}s")
    return LIB


if __name__ == "__main__":
    build()
