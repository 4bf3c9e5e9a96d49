"""libsnd's host C++ under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

The host translation units (plan builder, detection's host part, streaming, batching, tuning,
multi-rate, validation, FDMT tables and the C-ABI layer) are compiled with g++ and the
sanitizers, linked with the library's device objects (built by build(); their kernels are
never launched), and driven by tests/sanitize_host.cpp: plan creation on the 1024-channel x
4096-DM shape in every mode and storage type and on ragged and degenerate trees, candidate
extraction from staged cells, the cross-band merge, stream admission and checkpoint checks,
batch record sizing, FDMT tables and the validation helpers.
"""

import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


def test_library_host_code_under_sanitizers(tmp_path):
    from paper_2606_15361_amd import build as B
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host g++")
    hip_objs = [os.path.join(B.BUILD, s + ".o") for s in B.HIP_SOURCES]
    if not all(os.path.exists(o) for o in hip_objs):
        B.build()
    flags = ["-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all",
             "-D__HIP_PLATFORM_AMD__", "-I/opt/rocm/include", "-I" + os.path.join(ROOT, "include"), "-I" + B.CSRC]
    san = ["-fsanitize=address", "-fsanitize=undefined"]
    procs, objs = [], []
    for src in B.CXX_SOURCES + ["sanitize_host.cpp"]:
        path = os.path.join(HERE if src == "sanitize_host.cpp" else B.CSRC, src)
        obj = str(tmp_path / (src + ".o"))
        objs.append(obj)
        procs.append(subprocess.Popen([gxx] + flags + san + ["-c", path, "-o", obj], stdout=subprocess.PIPE,
                                      stderr=subprocess.STDOUT))
    for p in procs:
        out, _ = p.communicate(timeout=300)
        assert p.returncode == 0, out.decode(errors="replace")[-3000:]
    exe = str(tmp_path / "sanitize_host")
    subprocess.run([gxx] + san + ["-o", exe] + objs + hip_objs +
                   ["-L/opt/rocm/lib", "-lamdhip64", "-lrocprofiler-sdk-roctx", "-Wl,-rpath,/opt/rocm/lib"],
                   check=True, capture_output=True, timeout=300)
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr[-5000:]
    assert "sanitized host run ok" in r.stdout
