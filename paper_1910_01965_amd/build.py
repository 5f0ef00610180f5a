"""Build libzmc.so (HIP, gfx950) in-tree with hipcc.

Every HIP translation unit is compiled with the packed-FP32 target feature
switched off; the objects are linked into one shared library next to this
file.  Run `python -m paper_1910_01965_amd.build` or call build().
"""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(ROOT, "include")
LIB = os.path.join(HERE, "libzmc.so")
FAMILIES = ("SinSum", "Gauss", "CosExp", "Const", "Linear")
REALS = ("float", "double")
# (source, extra defines, object name): the family kernels build one
# translation unit per (family, precision, N = 1..8 or 9..16) so that they
# compile in parallel
SOURCES = ([("zmc_api.hip", (), "zmc_api"), ("zmc_batch.hip", (), "zmc_batch"),
            ("zmc_tune.hip", (), "zmc_tune"), ("zmc_kernels.hip", (), "zmc_kernels"),
            ("zmc_server.hip", (), "zmc_server"), ("zmc_rtc.hip", (), "zmc_rtc")]
           + [("zmc_family.hip", (f"-DZMC_FAMILY={f}", f"-DZMC_REAL={r}", f"-DZMC_NLO={lo}"),
               f"zmc_{f}_{r}_N{lo}")
              for f in FAMILIES for r in REALS for lo in (1, 9)]
           + [("zmc_any.hip", (f"-DZMC_REAL={r}",), f"zmc_any_{r}") for r in REALS])
ARCH = "gfx950"
ROCM = os.environ.get("ROCM_PATH", "/opt/rocm")
# device headers that the run-time compiler of user integrands needs, embedded
# into the library as text
RTC_HEADERS = ("zmc_device.hpp", "zmc_scan.hpp", "zmc_user.hpp")


def hipcc():
    path = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(path):
        raise RuntimeError("hipcc not found; the ROCm toolchain is required to build libzmc")
    return path


def flags():
    return ["-std=c++17", "-O3", f"--offload-arch={ARCH}", "-fPIC",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
            "-I", INCLUDE, "-I", CSRC, "-Wall", "-Wno-unused-function"]


def write_rtc_headers(path):
    """The device headers as C string literals: kRtcHeaderCount,
    kRtcHeaderNames[], kRtcHeaderTexts[] (included by zmc_rtc.hip)."""
    delim = "zmchdr"
    parts = [f"constexpr int kRtcHeaderCount = {len(RTC_HEADERS)};",
             "const char* const kRtcHeaderNames[] = {" + ", ".join(f'"{h}"' for h in RTC_HEADERS) + "};",
             "const char* const kRtcHeaderTexts[] = {"]
    for h in RTC_HEADERS:
        text = open(os.path.join(CSRC, h)).read()
        if f"){delim}\"" in text:
            raise RuntimeError(f"{h} contains the raw-string delimiter")
        parts.append(f'R"{delim}({text}){delim}",')
    parts.append("};")
    with open(path + ".tmp", "w") as fh:
        fh.write("\n".join(parts) + "\n")
    os.replace(path + ".tmp", path)


def build(out=LIB, jobs=None, verbose=False):
    """Compile every source and link `out`; returns its path."""
    objdir = os.path.join(HERE, "_build")
    os.makedirs(objdir, exist_ok=True)
    cc = hipcc()
    write_rtc_headers(os.path.join(objdir, "zmc_rtc_headers.inc"))

    def compile_one(entry):
        src, defines, name = entry
        obj = os.path.join(objdir, name + ".o")
        cmd = [cc, *flags(), "-I", objdir, *defines, "-c", os.path.join(CSRC, src), "-o", obj]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError(f"hipcc failed for {src}:\n{r.stderr}")
        if verbose and r.stderr:
            print(r.stderr)
        return obj

    if jobs is None:
        jobs = max(1, min(16, os.cpu_count() or 1))
    with ThreadPoolExecutor(max_workers=jobs) as ex:
        objs = list(ex.map(compile_one, SOURCES))
    tmp = out + ".tmp"
    subprocess.run([cc, "-shared", f"--offload-arch={ARCH}", "-fPIC", *objs, f"-L{ROCM}/lib",
                    "-lhiprtc", "-lrocprofiler-sdk-roctx", f"-Wl,-rpath,{ROCM}/lib", "-o", tmp],
                   check=True)
    os.replace(tmp, out)
    return out


if __name__ == "__main__":
    print(build(verbose=True))
