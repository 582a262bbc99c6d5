"""The two FP64 oracles and the host side of the C ABI under AddressSanitizer
and UndefinedBehaviorSanitizer (CPU only).

tests/sanitize/oracle_check.cpp drives every oracle entry point on small and
ragged lattices (2x2 up to 7x4, 3D down to 2x2x2, every closure, the 3D
moment-space collision as well as single relaxation); the build
links the oracle sources with g++ -fsanitize=address,undefined.
tests/sanitize/capi_check.cpp drives the host paths of the library
(validation, sizes, calls refused before bind, error strings); the HIP
sources are built with the sanitizers on their host pass only.
"""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang++"
HOST_SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
            "-Xarch_host", "-fno-sanitize-recover=all"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1", OMP_NUM_THREADS="2")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, (cmd, r.stdout[-3000:], r.stderr[-3000:])
    return r


def test_oracles_clean_under_asan_and_ubsan(tmp_path):
    if not shutil.which("g++"):
        pytest.skip("g++ missing")
    exe = str(tmp_path / "oracle_check")
    _run(["g++", "-std=c++17", "-O1", "-g", "-fopenmp", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
          os.path.join(ROOT, "oracle", "lbmhd_oracle.cpp"),
          os.path.join(ROOT, "oracle", "lbmhd3_oracle.cpp"),
          os.path.join(HERE, "sanitize", "oracle_check.cpp"), "-o", exe])
    r = _run([exe], env=ENV, timeout=600)
    assert r.stdout.strip().endswith("ok") and "runtime error" not in r.stderr


def test_capi_host_paths_clean_under_asan_and_ubsan(tmp_path):
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("ROCm toolchain missing")
    csrc = os.path.join(ROOT, "paper_1607_08675_amd", "csrc")
    inc = ["-I", os.path.join(ROOT, "include"), "-I", csrc]
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"] + HOST_SAN + inc
    srcs = ["lbmhd_kernels", "lbmhd_adjoint", "lbmhd_capi", "lbmhd3"]
    objs = [str(tmp_path / (s + ".o")) for s in srcs]
    with ThreadPoolExecutor(4) as ex:
        list(ex.map(lambda so: _run([HIPCC] + flags + ["-c", os.path.join(csrc, so[0] + ".hip"),
                                                       "-o", so[1]]), zip(srcs, objs)))
    drv = str(tmp_path / "capi_check.o")
    _run([CLANG, "-std=c++17", "-O1", "-g", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"] + inc + ["-c", os.path.join(HERE, "sanitize", "capi_check.cpp"),
                                              "-o", drv])
    exe = str(tmp_path / "capi_check")
    _run([CLANG, "-fsanitize=address,undefined", drv] + objs +
         ["-L/opt/rocm/lib", "-lamdhip64", "-Wl,-rpath,/opt/rocm/lib", "-o", exe])
    r = _run([exe], env=ENV, timeout=300)
    assert r.stdout.strip().endswith("ok") and "runtime error" not in r.stderr
