"""Compiles the package's native libraries in-tree.

* ``lib/libgvelpa.so``: the HIP library behind the C ABI in ``include/gvelpa.h``
  (gfx950 device code + host runtime), built with ``hipcc``.
* ``lib/libgvelpa_gen.so``: the host-only seeded graph generators (g++/OpenMP).
* ``lib/libgvelpa_gen_gpu.so``: the same R-MAT generator assembled into CSR on
  the GPU (``include/gvelpa_gen.h``), built with ``hipcc``.
* ``lib/libgvelpa_cpu.so``: the multicore CPU comparator in the paper's design
  (``include/gvelpa_cpu.h``, g++/OpenMP; never called by the GPU path).

``build_all()`` always recompiles; ``ensure_built()`` compiles only what is
missing.  Nothing here runs any GPU code.
"""
from __future__ import annotations

import os
import subprocess
from pathlib import Path

PKG = Path(__file__).resolve().parent
ROOT = PKG.parent
LIBDIR = PKG / "lib"
CSRC = PKG / "csrc"
INCLUDE = ROOT / "include"

LPA_LIB = LIBDIR / "libgvelpa.so"
GEN_LIB = LIBDIR / "libgvelpa_gen.so"
GEN_GPU_LIB = LIBDIR / "libgvelpa_gen_gpu.so"
CPU_LIB = LIBDIR / "libgvelpa_cpu.so"

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# Device code is compiled for gfx950 only.  Packed-FP32 instruction selection
# is switched off for every HIP translation unit.
HIP_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-munsafe-fp-atomics",
    "-Wno-unused-result",
]


def _run(cmd: list[str]) -> None:
    proc = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)
    if proc.returncode != 0:
        raise RuntimeError("build failed:\n" + " ".join(cmd) + "\n" + proc.stdout)


def lpa_sources() -> list[Path]:
    return sorted((CSRC / "lpa").glob("*.hip")) + sorted((CSRC / "lpa").glob("*.cpp"))


def build_gen() -> Path:
    LIBDIR.mkdir(exist_ok=True)
    tmp = GEN_LIB.with_suffix(".so.tmp")
    _run(["g++", "-O3", "-std=c++17", "-fPIC", "-shared", "-fopenmp",
          str(CSRC / "gen" / "graphgen.cpp"), "-o", str(tmp)])
    os.replace(tmp, GEN_LIB)
    return GEN_LIB


def build_cpu() -> Path:
    LIBDIR.mkdir(exist_ok=True)
    tmp = CPU_LIB.with_suffix(".so.tmp")
    _run(["g++", "-O3", "-std=c++17", "-fPIC", "-shared", "-fopenmp", "-I", str(INCLUDE),
          str(CSRC / "cpu" / "lpa_omp.cpp"), "-o", str(tmp)])
    os.replace(tmp, CPU_LIB)
    return CPU_LIB


def build_gen_gpu() -> Path:
    LIBDIR.mkdir(exist_ok=True)
    tmp = GEN_GPU_LIB.with_suffix(".so.tmp")
    _run([HIPCC, *HIP_FLAGS, "-shared", "-I", str(INCLUDE), str(CSRC / "gen" / "rmat_gpu.hip"), "-o", str(tmp)])
    os.replace(tmp, GEN_GPU_LIB)
    return GEN_GPU_LIB


def build_lpa() -> Path:
    LIBDIR.mkdir(exist_ok=True)
    objdir = PKG / "_build"
    objdir.mkdir(exist_ok=True)
    cmds, objs = [], []
    for src in lpa_sources():
        obj = objdir / (src.name + ".o")
        flags = HIP_FLAGS if src.suffix == ".hip" else ["-O3", "-std=c++17", "-fPIC"]
        cmd = [HIPCC, *flags, "-I", str(INCLUDE), "-I", str(CSRC / "lpa"), "-c", str(src), "-o", str(obj)]
        if src.suffix == ".cpp":
            cmd = [HIPCC, "-x", "c++", "-D__HIP_PLATFORM_AMD__", "-O3", "-std=c++17", "-fPIC",
                   "-I", str(INCLUDE), "-I", str(CSRC / "lpa"), "-c", str(src), "-o", str(obj)]
        cmds.append(cmd)
        objs.append(str(obj))
    # one compiler process per source file, a few at a time
    from concurrent.futures import ThreadPoolExecutor
    workers = max(1, min(len(cmds), os.cpu_count() or 1, 8))
    with ThreadPoolExecutor(workers) as ex:
        list(ex.map(_run, cmds))
    tmp = LPA_LIB.with_suffix(".so.tmp")
    _run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", *objs, "-o", str(tmp)])
    os.replace(tmp, LPA_LIB)
    return LPA_LIB


def build_all() -> None:
    build_gen()
    build_cpu()
    build_gen_gpu()
    build_lpa()


def ensure_built() -> None:
    if not GEN_LIB.exists():
        build_gen()
    if not GEN_GPU_LIB.exists():
        build_gen_gpu()
    if not CPU_LIB.exists():
        build_cpu()
    if not LPA_LIB.exists():
        build_lpa()
