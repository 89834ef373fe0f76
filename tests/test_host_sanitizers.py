"""Host code of the C ABI under AddressSanitizer and UndefinedBehaviorSanitizer
(no GPU needed): the library is rebuilt with host-side sanitizers (device code
unchanged) and linked with tests/host_sanitize/abi_host_checks.cpp, which runs
every argument-validation path, the footprint arithmetic over 2880 grid and
option combinations, and plan and server creation without a usable GPU."""
import os
import shutil
import subprocess
import tempfile

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1509_00680_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/lib/llvm/bin/clang++"
SOURCES = ["gps_api", "gps_ops", "gps_cavity", "gps_fft", "gps_fft_fast", "gps_server"]
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=undefined"]


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)),
                    reason="needs the ROCm compilers")
def test_abi_host_paths_clean_under_asan_ubsan():
    d = tempfile.mkdtemp(prefix="gps_san_")
    try:
        procs = []
        for f in SOURCES:
            cmd = [HIPCC, "-O1", "-g", "-fPIC", "-std=c++17", "--offload-arch=gfx950",
                   "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"] + HOST_SAN + [
                   "-fno-omit-frame-pointer", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
                   "-c", os.path.join(CSRC, f + ".hip"), "-o", os.path.join(d, f + ".o")]
            procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.PIPE))
        for pr in procs:
            out, err = pr.communicate()
            assert pr.returncode == 0, err.decode()[-2000:]
        drv = os.path.join(d, "drv.o")
        r = subprocess.run([CLANG, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
                            "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer",
                            "-I", os.path.join(ROOT, "include"), "-c",
                            os.path.join(HERE, "host_sanitize", "abi_host_checks.cpp"), "-o", drv],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        exe = os.path.join(d, "abi_host_checks")
        r = subprocess.run([HIPCC, "-g", "--offload-arch=gfx950"] + HOST_SAN[:4] + [drv] +
                           [os.path.join(d, f + ".o") for f in SOURCES] + ["-o", exe],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-2000:]
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
                   UBSAN_OPTIONS="print_stacktrace=1")
        r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
        assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
        assert "0 failures" in r.stdout
    finally:
        shutil.rmtree(d, ignore_errors=True)
