"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):
the library's sources are compiled with the sanitizers on their host part
(device code is built as usual and never launched), linked with the test program
tests/sanitize/abi_host_check.cpp, and run with leak detection on.  The program
creates grids of many sizes and tile sizes, fills every layout query into
buffers of exactly the reported sizes, builds the two-hop pattern and
two-grid pairs, and walks the argument-error and injected allocation-failure
paths (SYMPIX_FAIL_ALLOC)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1504_04653_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# sanitizers on the host compilation only (each flag behind -Xarch_host)
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-omit-frame-pointer", "-Xarch_host", "-fno-sanitize-recover=undefined"]
FLAGS = ["-std=c++17", "-O1", "-g", "-fPIC", "--offload-arch=gfx950",
         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]


@pytest.mark.slow
def test_host_abi_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    if not (os.path.exists(HIPCC) or shutil.which("hipcc")):
        pytest.skip("hipcc not available")
    srcs = [os.path.join(CSRC, "geometry.cpp"), os.path.join(CSRC, "api.cpp"), os.path.join(CSRC, "kernels.hip"), os.path.join(CSRC, "sht.hip"), os.path.join(CSRC, "precond.hip"),
            os.path.join(ROOT, "tests", "sanitize", "abi_host_check.cpp")]
    objs, procs = [], []
    for src in srcs:                     # the compilations run side by side
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        procs.append(subprocess.Popen([HIPCC, *FLAGS, *SAN, "-c", src, "-o", obj], stdout=subprocess.PIPE,
                                      stderr=subprocess.PIPE, text=True))
        objs.append(obj)
    for pr in procs:
        _, err = pr.communicate()
        assert pr.returncode == 0, err[-3000:]
    exe = str(tmp_path / "abi_host_check")
    res = subprocess.run([HIPCC, "--offload-arch=gfx950", *SAN, *objs, "-o", exe], capture_output=True, text=True)
    assert res.returncode == 0, res.stderr[-3000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    env.pop("SYMPIX_FAIL_ALLOC", None)
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert res.returncode == 0, (res.stdout + res.stderr)[-5000:]
    assert "abi_host_check OK" in res.stdout
    assert "runtime error" not in res.stderr and "AddressSanitizer" not in res.stderr
