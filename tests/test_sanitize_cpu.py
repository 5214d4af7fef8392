"""Address and undefined-behaviour sanitizer builds (CPU only).

1. The oracle (oracle/cv_oracle.c) with a driver that feeds it adversarial
   records (ties, duplicate rows, the extreme int64 ids, non-finite
   coordinates, speeds outside every fast format, empty input) and checks the
   invariants that need no second implementation.
2. The library's host code (device code is compiled but never launched): every
   size query at the edges of its domain and every argument check, with the
   answers the header documents.

Either driver exits non-zero on the first sanitizer report."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_2305_07454_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
CLANGXX = "/opt/rocm/llvm/bin/clang++"
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-4000:]}\n{r.stderr[-4000:]}"
    return r.stdout


@pytest.fixture(scope="module")
def out(tmp_path_factory):
    return tmp_path_factory.mktemp("sanitize")


def test_oracle_under_sanitizers(out):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not found")
    exe = str(out / "oracle_driver")
    _run(["gcc", "-std=c11", "-O1", "-g", "-ffp-contract=off", *SAN, "-o", exe,
          os.path.join(HERE, "oracle_driver.c"), os.path.join(ROOT, "oracle", "cv_oracle.c"), "-lm"])
    for n, seed in [(0, 1), (1, 2), (2, 3), (4999, 4), (60000, 5)]:
        s = _run([exe, str(n), str(seed)], env=ENV, timeout=300)
        assert s.startswith("ok"), s


def _host_objects(out):
    # -fsanitize applies to the host pass only (the device code is compiled
    # as usual so that the objects link; no kernel runs)
    flags = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-ffp-contract=off",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", "-Wno-unused-result",
             "-I", os.path.join(ROOT, "include"), "-I", CSRC]
    for f in SAN:
        flags += ["-Xarch_host", f]
    srcs = sorted(x for x in os.listdir(CSRC) if x.endswith(".hip"))
    procs = []
    for s in srcs:
        o = str(out / (s + ".o"))
        procs.append((s, o, subprocess.Popen([HIPCC, *flags, "-c", os.path.join(CSRC, s), "-o", o],
                                             stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True)))
    objs = []
    for s, o, p in procs:
        so, se = p.communicate()
        assert p.returncode == 0, f"{s}:\n{se[-4000:]}"
        objs.append(o)
    return objs


def test_library_host_code_under_sanitizers(out):
    if not (os.path.exists(HIPCC) and os.path.exists(CLANGXX)):
        pytest.skip("hipcc not found")
    objs = _host_objects(out)
    drv = str(out / "host_driver.o")
    _run([CLANGXX, "-O1", "-g", "-std=c++17", *SAN, "-I", os.path.join(ROOT, "include"), "-c",
          os.path.join(HERE, "host_driver.cpp"), "-o", drv])
    exe = str(out / "host_driver")
    link = [HIPCC, "--offload-arch=gfx950", "-o", exe, drv, *objs]
    for f in SAN[:1]:
        link += ["-Xarch_host", f]
    _run(link)
    # leaks inside the HIP runtime's own start-up are not this library's
    s = _run([exe], env=dict(ENV, ASAN_OPTIONS="detect_leaks=0"), timeout=300)
    assert s.startswith("ok"), s
