"""The C ABI's host code (abi.hip, noalloc.hip) built with AddressSanitizer
and UndefinedBehaviorSanitizer on the host side and driven through its
validation and error paths by tests/helpers/abi_sanitize_driver.cpp, linked
against host-only stand-ins of the kernel launchers
(tests/helpers/abi_host_stubs.cpp).  No GPU is used: device allocations fail
and the clean-up of partially built plans runs."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = "/opt/rocm/bin/hipcc"
CSRC = os.path.join(ROOT, "paper_1006_3340_amd", "csrc")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]
INC = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not available")
def test_abi_host_code_under_asan_and_ubsan(tmp_path):
    host = ["-x", "hip", "--cuda-host-only", "-O1", "-g", "-std=c++17", *SAN, *INC]
    objs = []
    for src, flags in ((os.path.join(CSRC, "abi.hip"), host),
                       (os.path.join(HERE, "helpers", "abi_host_stubs.cpp"), host),
                       (os.path.join(HERE, "helpers", "abi_sanitize_driver.cpp"), host),
                       # the static workspace is a device variable: build its device code too
                       (os.path.join(CSRC, "noalloc.hip"),
                        ["-x", "hip", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17",
                         "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *SAN, *INC])):
        obj = str(tmp_path / (os.path.basename(src) + ".o"))
        subprocess.run([HIPCC, *flags, "-c", src, "-o", obj], check=True, capture_output=True)
        objs.append(obj)
    exe = str(tmp_path / "abi_sanitize")
    subprocess.run([HIPCC, "--offload-arch=gfx950", *SAN, *objs, "-o", exe], check=True,
                   capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", HIP_VISIBLE_DEVICES="")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
