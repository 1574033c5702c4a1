"""Build the HIP library libmpa.so for gfx950 in-tree.

Every source under csrc/ is compiled with hipcc (kernels as HIP, the C ABI as
host C++ against the HIP runtime) and linked into
paper_1101_0086_amd/libmpa.so.  Objects go to _build/ at the repository root.
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
OUT = os.path.join(PKG, "libmpa.so")
BUILD = os.path.join(ROOT, "_build")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

COMMON = ["-O3", "-fPIC", "-std=c++17", "-Wall", "-Wno-unused-function",
          "-I", os.path.join(ROOT, "include"), "-I", CSRC]
DEVICE = ["-x", "hip", "--offload-arch=gfx950",
          # no packed-FP32 instructions anywhere in device code
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]
HOST = ["-x", "c++", "-D__HIP_PLATFORM_AMD__", "-I", "/opt/rocm/include"]


# Block sizes compiled into the long-step kernels (the C++ dispatchers list
# the same sizes).  The launchers of each (precision, block size) pair of the
# files below are compiled as separate objects (-DMPA_SPLIT plus
# -DMPA_PART_T / -DMPA_PART_B), so that the template instantiations build in
# parallel; the object without a part holds the dispatching code.
BLOCKS = (512, 1024, 2048, 4096)
SPLIT = ("mpa_kernels.hip", "adjoint_kernels.hip")


def _sources():
    out = []
    for f in sorted(os.listdir(CSRC)):
        src = os.path.join(CSRC, f)
        if f.endswith(".hip"):
            if f in SPLIT:
                out.append((src, DEVICE + ["-DMPA_SPLIT"], f + ".o"))
                for t in ("float", "double"):
                    for b in BLOCKS:
                        out.append((src, DEVICE + ["-DMPA_SPLIT", f"-DMPA_PART_T={t}", f"-DMPA_PART_B={b}"],
                                    f"{f}.{t}{b}.o"))
            else:
                out.append((src, DEVICE, f + ".o"))
        elif f.endswith(".cpp"):
            out.append((src, HOST, f + ".o"))
    # longest compiles first
    out.sort(key=lambda x: 0 if "MPA_PART_T" in " ".join(x[1]) and "adjoint" in x[0] else 1)
    return out


def _compile(src, flags, objname):
    obj = os.path.join(BUILD, objname)
    cmd = [HIPCC] + COMMON + flags + ["-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"compile failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    return obj, r.stderr


def build(verbose: bool = False, jobs: int = 0) -> str:
    jobs = jobs or min(16, os.cpu_count() or 8)
    os.makedirs(BUILD, exist_ok=True)
    srcs = _sources()
    with cf.ThreadPoolExecutor(max_workers=min(jobs, len(srcs))) as ex:
        results = list(ex.map(lambda a: _compile(*a), srcs))
    objs = [o for o, _ in results]
    if verbose:
        for _, err in results:
            if err.strip():
                print(err, file=sys.stderr)
    tmp = OUT + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs + ["-lamdhip64"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError(f"link failed: {' '.join(cmd)}\n{r.stdout}\n{r.stderr}")
    os.replace(tmp, OUT)
    return OUT


if __name__ == "__main__":
    print(build(verbose=True))
