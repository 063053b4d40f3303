"""The oracle and the C ABI's host code under AddressSanitizer and
UndefinedBehaviorSanitizer (host code only; the GPU kernels are not
instrumented).  Two drivers (tests/sanitize/) are built and run:

* oracle_driver.c compiles the C oracle in with gcc and calls every entry
  point on random and degenerate boxes, with brute-force and tree
  searches;
* capi_driver.cpp calls every entry point of include/crk.h with a null
  context and the context/tuning checks with bad values, against the
  library's host code (capi.hip) built with the sanitizers for the host
  pass only, linked with the rest of the library.

Each must exit 0 with no sanitizer report."""
import os
import shutil
import subprocess
from pathlib import Path

import pytest

ROOT = Path(__file__).resolve().parents[1]
SAN = ROOT / "tests" / "sanitize"
CSRC = ROOT / "paper_2510_03557_amd" / "csrc"
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang++"


def _run(exe, tmp_path):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env,
                       timeout=300)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    return out


def test_oracle_under_asan_ubsan(tmp_path):
    if not shutil.which("gcc"):
        pytest.skip("gcc not available")
    exe = tmp_path / "oracle_asan"
    subprocess.run(["gcc", "-O1", "-g", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                    "-o", str(exe), str(SAN / "oracle_driver.c"), "-lm"],
                   check=True, capture_output=True, text=True, timeout=300)
    assert "all calls returned 0" in _run(exe, tmp_path)


def test_capi_host_checks_under_asan_ubsan(tmp_path):
    if not (os.path.exists(HIPCC) and os.path.exists(CLANG)):
        pytest.skip("hipcc not available")
    objs = []
    # the library's host code with the sanitizers (host pass only), the
    # other sources as built for the product
    san = ["-Xarch_host", "-fsanitize=address,undefined",
           "-Xarch_host", "-fno-sanitize-recover=all"]
    flags = ["-O1", "-g", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wno-unused-command-line-argument"]
    for src in ("capi", "primitives", "tree", "lists", "passes", "integrate",
                "substep", "pm", "halo"):
        obj = tmp_path / f"{src}.o"
        extra = san if src == "capi" else []
        prebuilt = ROOT / "paper_2510_03557_amd" / "_build" / f"{src}.o"
        if src != "capi" and prebuilt.exists():
            objs.append(str(prebuilt))
            continue
        subprocess.run([HIPCC, *flags, *extra, "-c", str(CSRC / f"{src}.hip"),
                        "-o", str(obj)], check=True, capture_output=True,
                       text=True, timeout=600)
        objs.append(str(obj))
    drv = tmp_path / "driver.o"
    subprocess.run([CLANG, "-O1", "-g", "-std=c++17",
                    "-fsanitize=address,undefined", "-c",
                    str(SAN / "capi_driver.cpp"), "-o", str(drv)],
                   check=True, capture_output=True, text=True, timeout=300)
    exe = tmp_path / "capi_asan"
    r = subprocess.run([CLANG, "-fsanitize=address,undefined", "-o", str(exe),
                        str(drv), *objs, "-L/opt/rocm/lib", "-lamdhip64",
                        "-lhipfft", "-Wl,-rpath,/opt/rocm/lib"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "0 unexpected statuses" in _run(exe, tmp_path)
