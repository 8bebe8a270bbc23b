"""Builds the HIP library ``libcgh.so`` for gfx950 in-tree with hipcc.

Every source under ``csrc/`` is compiled to an object in ``_build/`` (in
parallel), then linked into ``paper_1002_0916_amd/libcgh.so``.
"""
from __future__ import annotations

import glob
import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libcgh.so")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

# -ffp-contract=off: every fused multiply-add in the kernels is written out
# explicitly, and the compensated two-product must not be re-associated.
# Packed FP32 instructions are disabled for all device code.
HIPFLAGS = [
    "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-ffp-contract=off",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"), "-Wall",
]


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def _compile(src: str) -> str:
    obj = os.path.join(BUILD, os.path.basename(src) + ".o")
    cmd = [HIPCC, *HIPFLAGS, "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (src, r.stderr))
    return obj


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    srcs = sources()
    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(_compile, srcs))
    tmp = LIB + ".tmp%d" % os.getpid()
    cmd = [HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc link failed:\n%s" % r.stderr)
    os.replace(tmp, LIB)
    if verbose:
        print("built", LIB)
    return LIB


def build_variant(lib_path: str, defines, verbose: bool = False) -> str:
    """Builds the library with extra preprocessor definitions into
    ``lib_path`` (objects in their own build folder): diagnostic builds such
    as the adjoint's wave trace (``CGH_WAVE_TRACE``).  Not used by the
    package, which loads ``libcgh.so``."""
    tag = os.path.splitext(os.path.basename(lib_path))[0]
    bdir = os.path.join(BUILD, tag)
    os.makedirs(bdir, exist_ok=True)
    flags = [*HIPFLAGS, *("-D" + d for d in defines)]

    def comp(src):
        obj = os.path.join(bdir, os.path.basename(src) + ".o")
        r = subprocess.run([HIPCC, *flags, "-c", src, "-o", obj], capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("hipcc failed for %s:\n%s" % (src, r.stderr))
        return obj

    srcs = sources()
    with ThreadPoolExecutor(max_workers=min(8, len(srcs))) as ex:
        objs = list(ex.map(comp, srcs))
    r = subprocess.run([HIPCC, "--offload-arch=" + ARCH, "-shared", "-fPIC", *objs, "-o", lib_path],
                       capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc link failed:\n%s" % r.stderr)
    if verbose:
        print("built", lib_path)
    return lib_path


PROBE_SRC = os.path.join(HERE, "probe", "issue_rates.hip")
PROBE_BIN = os.path.join(HERE, "probe", "issue_rates")


def build_probe(verbose: bool = False) -> str:
    """Builds the machine-constant probe (a standalone program, not part of
    the library): FP32 issue rates of FMA and the transcendentals, and their
    accuracy."""
    cmd = [HIPCC, *HIPFLAGS, PROBE_SRC, "-o", PROBE_BIN]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s:\n%s" % (PROBE_SRC, r.stderr))
    if verbose:
        print("built", PROBE_BIN)
    return PROBE_BIN


def dump_isa(out_dir: str) -> None:
    """Writes the gfx950 assembly of every source to ``out_dir`` (inspection)."""
    os.makedirs(out_dir, exist_ok=True)
    for src in sources():
        out = os.path.join(out_dir, os.path.basename(src) + ".s")
        subprocess.run([HIPCC, *HIPFLAGS, "-S", "--cuda-device-only", src, "-o", out], check=True)


if __name__ == "__main__":
    build(verbose=True)
