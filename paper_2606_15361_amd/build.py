"""Build libsnd.so (HIP for gfx950 + host C++) in-tree with hipcc.

    python -m paper_2606_15361_amd.build
"""

from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
LIB = os.path.join(HERE, "libsnd.so")
BUILD = os.path.join(HERE, "_build")

HIP_SOURCES = ["kernels.hip", "kernels_lds.hip", "kernels_fast_binary.hip", "kernels_fast_graded.hip",
               "kernels_fast_float.hip", "kernels_bits.hip", "detect.hip", "label.hip",
               "detect_noalloc.hip", "group_lin.hip", "group_pack.hip"]
CXX_SOURCES = ["plan.cpp", "capi.cpp", "detect_host.cpp", "stream_host.cpp", "batch_host.cpp", "tune_host.cpp",
               "multirate_host.cpp", "validate_host.cpp", "fdmt_host.cpp", "subband_host.cpp"]

COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function", "-ffp-contract=off",
          "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]
# Packed FP32 instructions are disabled for all device code.
DEVICE = ["--offload-arch=gfx950", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    if os.path.exists(LIB):  # a failed build must not leave an older library behind
        os.remove(LIB)
    cc = hipcc()
    objs = []
    jobs = []
    for src in HIP_SOURCES + CXX_SOURCES:
        path = os.path.join(CSRC, src)
        if not os.path.exists(path):
            raise FileNotFoundError(f"libsnd source missing: {path}")
        obj = os.path.join(BUILD, src + ".o")
        if src.endswith(".hip"):
            cmd = [cc, "-x", "hip"] + COMMON + DEVICE + ["-c", path, "-o", obj]
        else:
            cmd = [cc] + COMMON + ["--offload-arch=gfx950", "-c", path, "-o", obj]
        jobs.append((cmd, src))
        objs.append(obj)
    procs = [(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT), src) for cmd, src in jobs]
    failed = []
    for p, src in procs:
        out, _ = p.communicate()
        text = out.decode(errors="replace")
        # hipcc's host pass does not know the device-only target feature; that warning is noise
        lines = [ln for ln in text.splitlines() if "packed-fp32-ops" not in ln and ln.strip()]
        if p.returncode != 0:
            failed.append((src, text))
        elif verbose and lines:
            print("\n".join(lines))
    if failed:
        for src, text in failed:
            sys.stderr.write(f"--- {src} ---\n{text}\n")
        raise RuntimeError("libsnd build failed: " + ", ".join(s for s, _ in failed))
    tmp = LIB + ".tmp"
    cmd = [cc, "-shared", "-fPIC", "--offload-arch=gfx950", "-o", tmp] + objs + ["-lrocprofiler-sdk-roctx"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose=True))
