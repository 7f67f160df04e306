"""AddressSanitizer + UndefinedBehaviorSanitizer builds of host code, run on
the CPU: the C oracle driven through every entry point on small workloads
(tests/sanitize/oracle_driver.c), and the host side of libdig (workspace
planning, configuration and argument checks of every entry point;
tests/sanitize/libdig_host_driver.cpp).  The device code of libdig is built
as usual; only its host pass is instrumented, and nothing touches a GPU."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2501_10965_amd", "csrc")
SOURCES = ["dig_api", "dig_kernels", "dig_synth", "dig_mlp"]
# leaks of the HIP runtime at exit are not this code's
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1:verify_asan_link_order=0",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, (cmd[0], r.returncode, r.stdout[-2000:], r.stderr[-4000:])
    return r


def test_oracle_under_asan_and_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    _run(["gcc", "-O1", "-g", "-std=gnu11", "-ffp-contract=off", "-fno-omit-frame-pointer",
          "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
          "-I", os.path.join(ROOT, "oracle"), os.path.join(SAN, "oracle_driver.c"),
          os.path.join(ROOT, "oracle", "dsmc_oracle.c"), "-lm", "-o", exe])
    r = _run([exe], env=ENV, timeout=120)
    for case in ("cavity", "vss slab", "annulus"):
        assert f"{case}:" in r.stdout, r.stdout
    assert "runtime error" not in r.stderr, r.stderr


@pytest.mark.skipif(shutil.which("hipcc") is None, reason="needs hipcc")
def test_libdig_host_code_under_asan_and_ubsan(tmp_path):
    objs = []
    for s in SOURCES:
        o = str(tmp_path / f"{s}.o")
        # host pass instrumented, device pass as usual
        _run(["hipcc", "--offload-arch=gfx950", "-O1", "-std=c++17", "-fPIC", "-c",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-Xarch_host", "-fsanitize=address,undefined",
              "-Xarch_host", "-fno-sanitize-recover=all",
              "-Xarch_host", "-fno-omit-frame-pointer",
              os.path.join(CSRC, f"{s}.hip"), "-o", o])
        objs.append(o)
    clang = "/opt/rocm/llvm/bin/clang++"
    drv = str(tmp_path / "driver.o")
    _run([clang, "-O1", "-g", "-std=c++17", "-fsanitize=address,undefined",
          "-fno-sanitize-recover=all", "-I", os.path.join(ROOT, "include"), "-c",
          os.path.join(SAN, "libdig_host_driver.cpp"), "-o", drv])
    exe = str(tmp_path / "libdig_host_driver")
    _run([clang, "-fsanitize=address,undefined"] + objs + [drv, "-L/opt/rocm/lib", "-lamdhip64",
         "-Wl,-rpath,/opt/rocm/lib", "-o", exe])
    r = _run([exe], env=ENV, timeout=120)
    assert "libdig host checks passed" in r.stdout, (r.stdout, r.stderr)
    assert "runtime error" not in r.stderr, r.stderr
