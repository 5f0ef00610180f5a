"""Compile tests/c/zmc_abi_check.c against include/zmc.h and libzmc.so, with
the oracle linked in (test infrastructure)."""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
SRC = os.path.join(HERE, "zmc_abi_check.c")
OUT = os.path.join(HERE, "zmc_abi_check")


def build(out=OUT, cc="gcc"):
    lib_dir = os.path.join(ROOT, "paper_1910_01965_amd")
    cmd = [cc, "-std=c99", "-O2", "-Wall", "-Wextra", "-I", os.path.join(ROOT, "include"),
           "-I", os.path.join(ROOT, "oracle"), SRC, os.path.join(ROOT, "oracle", "zmc_oracle.c"),
           "-L", lib_dir, "-l:libzmc.so", "-Wl,-rpath,$ORIGIN/../../paper_1910_01965_amd", "-lm",
           "-o", out + ".tmp"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build())
