"""Sanitizer builds of the host runtime (CPU only).

* The host thread pool (a lock-free ticket scheme) and the host block cache,
  stressed from several threads at once (tests/sanitize/pool_stress.cpp),
  built with ThreadSanitizer and with AddressSanitizer + UndefinedBehavior-
  Sanitizer by the host compiler.
* Concurrent task builds through the C ABI on host-only contexts
  (tests/sanitize/build_stress.cpp), with the library's host sources built by
  hipcc with the sanitizer on the host side only (the device code of the HIP
  sources is built as usual; nothing here touches a GPU).

Each program exits 0 only when every result check holds, and the sanitizer
makes it fail on any report."""
import concurrent.futures as cf
import glob
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2505_02692_amd", "csrc")
SAN = os.path.join(ROOT, "tests", "sanitize")
OUT = os.path.join(ROOT, "_build", "sanitize")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
SANITIZERS = {"thread": ["-fsanitize=thread"], "address": ["-fsanitize=address,undefined"]}
ENV = dict(os.environ, TSAN_OPTIONS="halt_on_error=1 exitcode=66",
           ASAN_OPTIONS="halt_on_error=1 detect_leaks=0", UBSAN_OPTIONS="halt_on_error=1 print_stacktrace=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd)}\n{r.stdout[-3000:]}\n{r.stderr[-3000:]}"
    return r


@pytest.mark.parametrize("san", sorted(SANITIZERS))
def test_pool_stress_under_sanitizer(san):
    os.makedirs(OUT, exist_ok=True)
    exe = os.path.join(OUT, f"pool_stress_{san}")
    _run(["g++", "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer"] + SANITIZERS[san] +
         ["-I", CSRC, os.path.join(SAN, "pool_stress.cpp"), "-o", exe, "-lpthread"])
    r = _run([exe], env=ENV, timeout=300)
    print(r.stdout.strip())


def _host_flags(san):
    # the sanitizer applies to the host side only (-Xarch_host before each flag)
    flags = []
    for f in SANITIZERS[san]:
        flags += ["-Xarch_host", f]
    return flags


@pytest.mark.parametrize("san", sorted(SANITIZERS))
def test_concurrent_task_builds_under_sanitizer(san):
    os.makedirs(OUT, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    common = ["-std=c++17", "-fPIC", "--offload-arch=gfx950"] + inc
    jobs = []
    for src in sorted(glob.glob(os.path.join(CSRC, "*.cpp"))):
        obj = os.path.join(OUT, f"{san}_{os.path.basename(src)}.o")
        jobs.append([HIPCC, "-O1", "-g"] + common + _host_flags(san) + ["-c", src, "-o", obj])
    for src in sorted(glob.glob(os.path.join(CSRC, "*.hip"))):
        obj = os.path.join(OUT, f"{san}_{os.path.basename(src)}.o")
        jobs.append([HIPCC, "-O2"] + common + ["-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                                                "-x", "hip", "-c", src, "-o", obj])
    main_obj = os.path.join(OUT, f"{san}_build_stress.o")
    jobs.append([HIPCC, "-O1", "-g", "-std=c++17"] + inc + _host_flags(san) +
                ["-c", os.path.join(SAN, "build_stress.cpp"), "-o", main_obj])
    with cf.ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        list(ex.map(_run, jobs))
    exe = os.path.join(OUT, f"build_stress_{san}")
    objs = sorted(glob.glob(os.path.join(OUT, f"{san}_*.o")))
    _run([HIPCC, "--offload-arch=gfx950"] + _host_flags(san) + objs + ["-o", exe, "-lpthread"])
    r = _run([exe], env=ENV, timeout=600)
    print(r.stdout.strip())
