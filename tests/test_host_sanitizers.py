"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer
(CPU only): runtime.hip's host side and coeffs.cpp are rebuilt with the
sanitizers (device code unchanged, host flags only), linked with the
in-tree kernel objects into tests/host_driver.c, and the driver is run; any
sanitizer report fails the test."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2505_16932_amd")
CSRC = os.path.join(PKG, "csrc")
INC = os.path.join(ROOT, "include")
HIPCC = "/opt/rocm/bin/hipcc"
LLVM = "/opt/rocm/llvm/bin"


def _run(cmd, **kw):
    p = subprocess.run(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True, **kw)
    assert p.returncode == 0, " ".join(cmd) + "\n" + p.stdout[-4000:]
    return p.stdout


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(LLVM + "/clang")),
                    reason="needs the ROCm toolchain")
def test_host_code_under_sanitizers(tmp_path):
    objs = [os.path.join(PKG, "_build", f) for f in ("kernels.hip.o", "learned.hip.o")]
    if not all(os.path.exists(o) for o in objs):
        from paper_2505_16932_amd import build
        build.build()
    d = str(tmp_path)
    # host passes only: each sanitizer flag goes behind -Xarch_host
    _run([HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-c",
          os.path.join(CSRC, "runtime.hip"), "-o", d + "/runtime.o", "-I", INC, "-I", CSRC,
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
          "-Xarch_host", "-fno-omit-frame-pointer"])
    _run([LLVM + "/clang++", "-O1", "-g", "-std=c++17", "-fPIC", "-c", os.path.join(CSRC, "coeffs.cpp"),
          "-o", d + "/coeffs.o", "-I", INC, "-fsanitize=address,undefined", "-fno-omit-frame-pointer"])
    _run([LLVM + "/clang", "-O1", "-g", "-c", os.path.join(ROOT, "tests", "host_driver.c"),
          "-o", d + "/driver.o", "-I", INC, "-fsanitize=address,undefined"])
    _run([HIPCC, "--offload-arch=gfx950", "-o", d + "/driver", d + "/driver.o", d + "/runtime.o",
          d + "/coeffs.o"] + objs + ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"])
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", HIP_VISIBLE_DEVICES="")
    p = subprocess.run([d + "/driver", d], stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True,
                       env=env, timeout=300)
    print(p.stdout[-2000:])
    assert "Sanitizer" not in p.stdout and "runtime error" not in p.stdout
    assert p.returncode == 0 and "host checks: 0 failures" in p.stdout
