"""Compiles libsde.so (every HIP source under csrc/) for gfx950 with hipcc.

The objects are built in parallel into csrc/_build/ and linked into
paper_0903_3852_amd/libsde.so, next to the Python binding that loads it.
"""
import concurrent.futures as cf
import glob
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
OBJDIR = os.path.join(CSRC, "_build")
LIB = os.path.join(HERE, "libsde.so")
ARCH = "gfx950"
ROCM_LIB = "/opt/rocm/lib"  # roctx (ranges around the C-ABI calls)

# Packed FP32 VALU forms are switched off for all device code.
HIPFLAGS = ["--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-Wall",
            "-Wno-unused-command-line-argument",
            "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc():
    exe = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(exe):
        raise RuntimeError("hipcc not found: the ROCm toolchain is required to build libsde")
    return exe


def sources():
    return sorted(glob.glob(os.path.join(CSRC, "*.hip")))


def _compile(src, verbose):
    obj = os.path.join(OBJDIR, os.path.basename(src) + ".o")
    cmd = [hipcc()] + HIPFLAGS + ["-I", os.path.join(HERE, "..", "include"), "-c", src, "-o", obj]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    out = "\n".join(line for line in (r.stdout + r.stderr).splitlines()
                    if "packed-fp32-ops" not in line)
    if r.returncode != 0:
        raise RuntimeError(f"hipcc failed on {os.path.basename(src)}:\n{out}")
    if out.strip() and verbose:
        print(out, flush=True)
    return obj


PROBE_SRC = os.path.join(HERE, "probe", "valu_issue.hip")
PROBE_LIB = os.path.join(HERE, "libvaluprobe.so")


def build_probe(verbose=False):
    """Compile the VALU issue-cost probe (bench.py --workload valu_costs)
    into its own small library; libsde does not contain it."""
    tmp = PROBE_LIB + ".tmp"
    cmd = [hipcc()] + HIPFLAGS + ["-shared", PROBE_SRC, "-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed on valu_issue.hip:\n" + r.stdout + r.stderr)
    os.replace(tmp, PROBE_LIB)
    return PROBE_LIB


def build(verbose=False, jobs=None):
    """Compile every csrc/*.hip and link libsde.so (always rebuilds), then
    the issue-cost probe."""
    os.makedirs(OBJDIR, exist_ok=True)
    srcs = sources()
    jobs = jobs or min(len(srcs), os.cpu_count() or 4, 8)
    with cf.ThreadPoolExecutor(jobs) as ex:
        objs = list(ex.map(lambda s: _compile(s, verbose), srcs))
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-shared", "-fPIC", "-o", tmp] + objs + [
        "-L" + ROCM_LIB, "-Wl,-rpath," + ROCM_LIB, "-lrocprofiler-sdk-roctx"]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    build_probe(verbose)
    return LIB


if __name__ == "__main__":
    build(verbose="-v" in sys.argv)
