"""AddressSanitizer and UndefinedBehaviorSanitizer (with LeakSanitizer) over
host code, on the CPU: the oracle (tests/sanitize/oracle_driver.c: every
search against the brute definition, spatial trees, WSPD) and the host side
of libpargeo_hip (tests/sanitize/host_driver.c: argument validation, handle
lifetimes, workspace planning).  Device code is not instrumented: the
library's sources are compiled for the host only (--cuda-host-only, each
-fsanitize behind -Xarch_host), and the device images the host objects
would register are replaced by empty stand-ins, since the driver launches
no kernel."""
import concurrent.futures
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2207_01834_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang"
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd[:3])} ... failed:\n{r.stdout[-3000:]}\n{r.stderr[-3000:]}"
    return r


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_asan_ubsan(tmp_path):
    exe = str(tmp_path / "oracle_driver")
    run(["gcc", "-O1", "-g", "-std=gnu11", "-ffp-contract=off",
         "-fsanitize=address,undefined,float-cast-overflow", "-fno-sanitize-recover=all",
         "-fno-omit-frame-pointer", os.path.join(ROOT, "tests", "sanitize", "oracle_driver.c"),
         os.path.join(ROOT, "oracle", "oracle.c"), "-lpthread", "-lm", "-o", exe])
    r = run([exe], env=ENV, timeout=300)
    assert "ok" in r.stdout


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="ROCm toolchain not available")
def test_host_runtime_under_asan_ubsan(tmp_path):
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-fno-omit-frame-pointer"]
    srcs = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))

    def compile_one(f):
        obj = str(tmp_path / (f[:-4] + ".o"))
        run([HIPCC, "--cuda-host-only", "-O1", "-g", "-fPIC", "-std=c++17", "-I", os.path.join(ROOT, "include"),
             "-I", CSRC, *san, "-c", os.path.join(CSRC, f), "-o", obj])
        return obj

    with concurrent.futures.ThreadPoolExecutor(8) as ex:
        objs = list(ex.map(compile_one, srcs))
    # the device images each host object registers at load time: empty
    # stand-ins (no kernel is launched)
    syms = set()
    for o in objs:
        syms.update(re.findall(r"__hip_fatbin_[0-9a-f]+", run(["nm", "-u", o]).stdout))
    stub = tmp_path / "images.c"
    stub.write_text("".join(f"const char {s}[64] __attribute__((aligned(4096))) = {{0}};\n" for s in sorted(syms)))
    run([CLANG, "-c", str(stub), "-o", str(tmp_path / "images.o")])
    drv = str(tmp_path / "host_driver.o")
    run([CLANG, "-O1", "-g", "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
         "-I", os.path.join(ROOT, "include"), "-c", os.path.join(ROOT, "tests", "sanitize", "host_driver.c"),
         "-o", drv])
    exe = str(tmp_path / "host_driver")
    run([HIPCC, *san, drv, str(tmp_path / "images.o"), *objs, "-o", exe])
    r = run([exe], env=ENV, timeout=300)
    assert "ok" in r.stdout
