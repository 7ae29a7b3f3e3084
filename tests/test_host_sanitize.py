"""The library's host logic under AddressSanitizer and UndefinedBehaviorSanitizer.

Every library source is compiled as for the library, with the sanitizers on
the host pass only (the device code is built but never launched), and linked with
``tests/host_sanitize/driver.cpp``, which checks the tile configuration
codes, emulates the work lists of every tile shape / split level / order on
random ragged sectors against H_l V + V H_r^T, round-trips blocks through
export and import (and has inconsistent descriptors refused), and reads a
malformed autotuner cache.  No GPU is needed.
"""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def build(out_dir):
    from paper_0707_0159_amd import build as B
    os.makedirs(out_dir, exist_ok=True)
    # host pass only, sanitizers on it; each -fsanitize after -Xarch_host
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
    flags = [f"--offload-arch={B.ARCH}", "-Xarch_host", "-O1", "-Xarch_host", "-g", "-fPIC", "-std=c++17", "-Wno-unused-result",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-I", os.path.join(ROOT, "include"), "-I", B.CSRC] + san
    objs = []
    procs = []
    for src in B.SOURCES + ["driver.cpp"]:
        path = os.path.join(ROOT, "tests", "host_sanitize", src) if src == "driver.cpp" else os.path.join(B.CSRC, src)
        obj = os.path.join(out_dir, src + ".o")
        objs.append(obj)
        procs.append((src, subprocess.Popen([HIPCC, *flags, "-x", "hip", "-c", path, "-o", obj],
                                            stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True)))
    for src, p in procs:
        out = p.communicate()[0]
        assert p.returncode == 0, f"{src}:\n{out[-4000:]}"
    exe = os.path.join(out_dir, "driver")
    r = subprocess.run([HIPCC, f"--offload-arch={B.ARCH}", *san, "-o", exe, *objs, "-L/opt/rocm/lib", "-lrocsolver",
                        "-lrocblas", "-Wl,-rpath,/opt/rocm/lib"], capture_output=True, text=True)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    return exe


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    return build(str(tmp_path_factory.mktemp("host_sanitize")))


def run(exe, *args):
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1",
               HIP_VISIBLE_DEVICES="")
    r = subprocess.run([exe, *args], capture_output=True, text=True, env=env, timeout=600)
    print(r.stdout[-3000:])
    print(r.stderr[-6000:])
    return r


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_host_logic_under_asan_ubsan(driver):
    r = run(driver)
    assert r.returncode == 0
    assert "host checks passed" in r.stdout


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_work_list_emulation_catches_a_dropped_k_step(driver):
    """A K step removed from one item of every work list: the emulation no
    longer matches H_l V + V H_r^T, so the driver must report failures."""
    r = run(driver, "--mutate")
    assert r.returncode == 1
    assert "FAIL" in r.stdout and "check(s) failed" in r.stdout
