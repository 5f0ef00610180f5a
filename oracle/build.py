"""Compile the plain-C oracle into oracle/libzmc_oracle.so.

TEST INFRASTRUCTURE ONLY.  ISO C99 mode keeps the compiler from contracting
multiply-adds, so the only fused operation is the explicit fma() of the
uniform map.
"""
import os
import subprocess

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "zmc_oracle.c")
LIB = os.path.join(HERE, "libzmc_oracle.so")


def build(out=LIB, src=SRC, cc="gcc", extra=()):
    """Compile `src` into the shared library `out`; returns `out`."""
    cmd = [cc, "-std=c99", "-O2", "-Wall", "-Wextra", "-fPIC", "-shared",
           "-I", HERE, *extra, src, "-o", out + ".tmp", "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


CLI_SRC = os.path.join(HERE, "zmc_oracle_cli.c")
CLI = os.path.join(HERE, "zmc_oracle_cli")


def build_cli(out=CLI, cc="gcc"):
    """Compile the command-line front end (oracle + CLI) into `out`."""
    cmd = [cc, "-std=c99", "-O2", "-Wall", "-Wextra", "-I", HERE, CLI_SRC, SRC, "-o", out + ".tmp",
           "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(out + ".tmp", out)
    return out


if __name__ == "__main__":
    print(build())
    print(build_cli())
