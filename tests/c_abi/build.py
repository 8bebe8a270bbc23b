"""Builds tests/c_abi/check (a plain-C consumer of include/cgh.h) with gcc,
linked against the in-tree libcgh.so and the HIP runtime."""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def command(out: str) -> list[str]:
    return ["gcc", "-std=gnu99", "-O1", "-Wall", "-Werror", "-D__HIP_PLATFORM_AMD__",
            "-I" + os.path.join(ROCM, "include"), "-I" + os.path.join(ROOT, "include"),
            os.path.join(HERE, "check.c"), "-o", out,
            "-L" + os.path.join(ROOT, "paper_1002_0916_amd"), "-lcgh",
            "-L" + os.path.join(ROCM, "lib"), "-lamdhip64", "-lm",
            "-Wl,-rpath,$ORIGIN/../../paper_1002_0916_amd",
            "-Wl,-rpath," + os.path.join(ROCM, "lib")]


def build(out: str | None = None) -> str:
    out = out or os.path.join(HERE, "check")
    subprocess.run(command(out), check=True)
    return out


if __name__ == "__main__":
    print(build(sys.argv[1] if len(sys.argv) > 1 else None))
