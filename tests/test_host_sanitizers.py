"""The library's host code (plan geometry and window labels of eq:inverse1-3,
the dense Rayleigh-Ritz solvers, the status paths of the C ABI) built with
AddressSanitizer and UndefinedBehaviorSanitizer and driven by
tests/host_sanitizer_driver.cpp on host-only plans.  The device translation
units are linked uninstrumented from the regular build; the sanitizer flags
reach the host compilation only (-Xarch_host), and nothing here touches a GPU.
"""

import os
import subprocess
from concurrent.futures import ThreadPoolExecutor

import pytest

from paper_2404_04507_amd import build as B

HERE = os.path.dirname(os.path.abspath(__file__))
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]


def _device_objects():
    host = {os.path.join(B.BUILD, os.path.splitext(s)[0] + ".o") for s in B.HOST_SOURCES}
    return [obj for obj, _ in B._jobs() if obj not in host]


def _compile(args):
    src, obj, extra = args
    cmd = [B.HIPCC, "-O1", "-g", "-std=c++17", "-fPIC", "-pthread", f"--offload-arch={B.ARCH}",
           "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", *SAN,
           "-I", os.path.join(B.ROOT, "include"), "-I", B.CSRC, *extra, "-x", "hip", "-c", src, "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    return obj, r.returncode, r.stderr


def test_host_code_under_address_and_undefined_behavior_sanitizers(tmp_path):
    dev = _device_objects()
    missing = [o for o in dev if not os.path.exists(o)]
    if missing:
        pytest.skip(f"device objects not built ({len(missing)} missing): run __graft_entry__.build() first")
    jobs = [(os.path.join(B.CSRC, s), str(tmp_path / (os.path.splitext(s)[0] + ".o")), []) for s in B.HOST_SOURCES]
    jobs.append((os.path.join(HERE, "host_sanitizer_driver.cpp"), str(tmp_path / "driver.o"), []))
    with ThreadPoolExecutor(max_workers=min(len(jobs), os.cpu_count() or 4)) as ex:
        results = list(ex.map(_compile, jobs))
    for obj, rc, err in results:
        assert rc == 0, f"compiling {obj} failed:\n{err[-3000:]}"
    exe = str(tmp_path / "host_sanitizer_driver")
    link = [B.HIPCC, f"--offload-arch={B.ARCH}", "-pthread", "-Xarch_host", "-fsanitize=address",
            "-Xarch_host", "-fsanitize=undefined", *[o for o, _, _ in results], *dev, "-o", exe]
    r = subprocess.run(link, capture_output=True, text=True)
    assert r.returncode == 0, f"link failed:\n{r.stderr[-3000:]}"
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:halt_on_error=1:abort_on_error=0"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    env["HIP_VISIBLE_DEVICES"] = ""  # host-only: the driver never needs a device
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    report = (r.stdout + r.stderr)[-6000:]
    assert r.returncode == 0, report
    assert "all checks passed" in r.stdout, report
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, report
