"""Builds the HIP library (gfx950) in-tree: paper_1907_11771_amd/lib/libgbs.so.

    python -m paper_1907_11771_amd.build
"""
import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB_DIR = os.path.join(HERE, "lib")
LIB = os.path.join(LIB_DIR, "libgbs.so")
SOURCES = ["plan.hip", "weights.cpp"]
ARCH = "gfx950"


def hipcc():
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose=False):
    os.makedirs(LIB_DIR, exist_ok=True)
    tmp = LIB + ".tmp"
    cmd = [hipcc(), "--offload-arch=" + ARCH, "-O3", "-std=c++17", "-fPIC", "-shared",
           # no packed FP32 instructions in generated code
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
           "-Wno-unused-command-line-argument",
           "-I", os.path.join(ROOT, "include"), "-o", tmp]
    cmd += [os.path.join(CSRC, s) for s in SOURCES]
    if verbose:
        print(" ".join(cmd), flush=True)
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        sys.stderr.write(res.stdout + res.stderr)
        raise RuntimeError("hipcc failed (%d)" % res.returncode)
    check_kernels(tmp)
    os.replace(tmp, LIB)
    return LIB


def check_kernels(lib):
    """Every kernel the host code of ``lib`` launches must be in its gfx950
    code object (a source edited while hipcc's host and device passes ran
    apart would leave a launch stub without its kernel).  Skipped when the
    ROCm binary tools are not at hand."""
    import re
    import tempfile
    llvm = "/opt/rocm/llvm/bin"
    tools = [shutil.which("objcopy"), shutil.which("nm"), os.path.join(llvm, "clang-offload-bundler"),
             os.path.join(llvm, "llvm-readelf")]
    if not all(t and os.path.exists(t) for t in tools):
        return
    objcopy, nm, bundler, readelf = tools
    with tempfile.TemporaryDirectory() as d:
        fat, co = os.path.join(d, "fatbin"), os.path.join(d, "co.o")
        run = lambda cmd: subprocess.run(cmd, capture_output=True, text=True, check=True).stdout
        run([objcopy, "-O", "binary", "--only-section=.hip_fatbin", lib, fat])
        run([bundler, "--unbundle", "--type=o", "--input=" + fat, "--output=" + co,
             "--targets=hipv4-amdgcn-amd-amdhsa--" + ARCH])
        dev = set(re.findall(r"\b(_Z\w+)\b", run([readelf, "--syms", co])))
        missing = []
        for sym in run([nm, "-D", lib]).split():
            m = re.search(r"(\d+)__device_stub__", sym)
            if not m:
                continue
            n = int(m.group(1))
            comp = sym[m.end(1):m.end(1) + n]              # "__device_stub__" + name
            kernel = sym[:m.start(1)] + str(n - 15) + comp[15:] + sym[m.end(1) + n:]
            if kernel not in dev:
                missing.append(kernel)
    if missing:
        raise RuntimeError("%d kernels launched by the host code are missing from the code "
                           "object (rebuild from an unchanged tree), e.g. %s"
                           % (len(missing), missing[0]))


if __name__ == "__main__":
    print(build(verbose=True))
