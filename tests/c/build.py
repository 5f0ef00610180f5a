"""Compile tests/c/zmc_abi_check.c against include/zmc.h and libzmc.so, with
the oracle linked in (test infrastructure) and HIP's C runtime API for the
device buffers."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SRC = os.path.join(HERE, "zmc_abi_check.c")
OUT = os.path.join(HERE, "zmc_abi_check")
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")


def build(out=OUT, cc="gcc"):
    lib_dir = os.path.join(ROOT, "paper_1910_01965_amd")
    cmd = [cc, "-std=c99", "-O2", "-Wall", "-Wextra", "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "oracle"), SRC, os.path.join(ROOT, "oracle", "zmc_oracle.c"),
           "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROCM, "include"),
           "-L", lib_dir, "-l:libzmc.so", "-Wl,-rpath,$ORIGIN/../../paper_1910_01965_amd",
           "-L", os.path.join(ROCM, "lib"), "-lamdhip64", "-Wl,-rpath," + os.path.join(ROCM, "lib"),
           "-lm", "-o", out + ".tmp"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build())
