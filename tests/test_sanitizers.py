"""AddressSanitizer + UndefinedBehaviorSanitizer runs of the CPU oracle and of the library's host
runtime (CPU only).

The oracle is compiled with gcc for each stencil together with tests/sanitize/oracle_driver.c,
which walks every oracle entry point over small grids in every boundary configuration and the
documented error paths.  The host runtime (the C ABI's validation, setters, geometry and tile
classification, launch settings and the overlapping-buffer check) is compiled with hipcc for
gfx950 with the sanitizers on its host side only, and driven by
tests/sanitize/host_runtime_driver.cpp without a device.  Any sanitizer report, including a leak,
fails the run (-fno-sanitize-recover, LeakSanitizer on at exit).
"""
import os
import shutil
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = os.path.join(HERE, "sanitize")
CSRC = os.path.join(ROOT, "paper_2504_20169_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang++"
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="2")


def _run(cmd, **kw):
    res = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert res.returncode == 0, "%s\n%s%s" % (" ".join(cmd), res.stdout, res.stderr[-4000:])
    return res


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
@pytest.mark.parametrize("q", [37, 17, 9])
def test_oracle_under_asan_and_ubsan(q, tmp_path):
    exe = str(tmp_path / ("oracle_san_%d" % q))
    _run(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", "-ffp-contract=off", "-fopenmp", "-DORC_Q=%d" % q, "-o", exe,
          os.path.join(SAN, "oracle_driver.c"), os.path.join(ROOT, "oracle", "lbm_oracle.c"), "-lm"])
    res = _run([exe], env=ENV, timeout=300)
    assert "0 failures" in res.stdout, res.stdout


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="ROCm toolchain not found")
def test_host_runtime_under_asan_and_ubsan(tmp_path):
    host_san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                "-Xarch_host", "-fno-sanitize-recover=all"]
    flags = ["-O1", "-g", "-fno-omit-frame-pointer", "--offload-arch=gfx950", "-std=c++17", "-fPIC",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", os.path.join(ROOT, "include"), "-I", CSRC] + host_san
    srcs = ["lbm_kernels.hip", "lbm_kernels_d2q17.hip", "lbm_kernels_d2q9.hip", "lbm_capi.hip"]
    objs = [str(tmp_path / (s + ".o")) for s in srcs]
    cmds = [[HIPCC] + flags + ["-c", os.path.join(CSRC, s), "-o", o] for s, o in zip(srcs, objs)]
    drv = str(tmp_path / "driver.o")
    cmds.append([CLANG, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
                 "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "include"), "-c",
                 os.path.join(SAN, "host_runtime_driver.cpp"), "-o", drv])
    with ThreadPoolExecutor(max_workers=len(cmds)) as ex:
        list(ex.map(_run, cmds))
    exe = str(tmp_path / "host_san")
    _run([CLANG, "-fsanitize=address,undefined"] + objs + [drv, "-L/opt/rocm/lib", "-lamdhip64",
                                                          "-lrocprofiler-sdk-roctx",
                                                          "-Wl,-rpath,/opt/rocm/lib", "-o", exe])
    res = _run([exe], env=ENV, timeout=300)
    assert " 0 failures" in res.stdout, res.stdout
