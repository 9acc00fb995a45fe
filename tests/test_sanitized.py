"""The oracle and the library's host code under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only).

- The two oracles (D2Q9 and D3Q19) are compiled with gcc together with their
  drivers (`oracle/sanitize_check.c`, `oracle/sanitize_check3.c`), which walk
  every force mode, interface kind, boundary kind and diagnostic on small
  problems.
- The library's translation units are compiled with the sanitizers on their
  host side only (the GPU code is built as usual and never runs here) and
  linked to `tests/sanitize_host_check.cpp`, which drives problem validation,
  the workspace layout, the mesh checks and the argument guards of the C ABI.

Any out-of-bounds access, use after free, leak or undefined behaviour aborts
the executable, and the test fails with its report.
"""
import concurrent.futures as cf
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")
CSRC = os.path.join(ROOT, "paper_2003_12186_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANG = "/opt/rocm/llvm/bin/clang++"
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
           UBSAN_OPTIONS="print_stacktrace=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout}\n{r.stderr}"
    return r.stdout


@pytest.mark.parametrize("driver", ["sanitize_check.c", "sanitize_check3.c"])
def test_oracle_under_sanitizers(tmp_path, driver):
    exe = str(tmp_path / "check")
    _run(["gcc", "-std=c11", "-O1", "-g", *SAN, "-I", ORACLE, os.path.join(ORACLE, driver),
          "-o", exe, "-lm"])
    out = _run([exe], env=ENV, timeout=300)
    assert "ok" in out


@pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)), reason="no ROCm toolchain")
def test_library_host_code_under_sanitizers(tmp_path):
    units = {"sweep.hip": [], "interface.hip": ["-ffp-contract=off"], "runtime.hip": [],
             "learned.hip": [], "d3q19.hip": ["-ffp-contract=off"]}
    # sanitizers on the host side of each unit only (each -fsanitize flag
    # behind -Xarch_host); the device code is built as for the library
    host_san = []
    for f in SAN:
        host_san += ["-Xarch_host", f]

    def compile_unit(name, extra):
        obj = str(tmp_path / name.replace(".hip", ".o"))
        _run([HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *host_san, *extra,
              "-I", os.path.join(ROOT, "include"), "-c", os.path.join(CSRC, name), "-o", obj])
        return obj

    with cf.ThreadPoolExecutor(max_workers=len(units)) as ex:
        objs = list(ex.map(lambda kv: compile_unit(*kv), units.items()))
    drv = str(tmp_path / "drv.o")
    _run([CLANG, "-std=c++17", "-O1", "-g", *SAN, "-c",
          os.path.join(ROOT, "tests", "sanitize_host_check.cpp"), "-o", drv])
    exe = str(tmp_path / "hostcheck")
    _run([CLANG, *SAN[:1], drv, *objs, "-L/opt/rocm/lib", "-lamdhip64",
          "-Wl,-rpath,/opt/rocm/lib", "-o", exe])
    out = _run([exe], env=ENV, timeout=300)
    assert "sanitize-host-check ok" in out
    shutil.rmtree(tmp_path, ignore_errors=True)
