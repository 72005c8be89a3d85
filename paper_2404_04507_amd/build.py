"""Build libiwfpm.so (HIP for gfx950 + host C++) in-tree.

    python -m paper_2404_04507_amd.build [-j N]

Every apply kernel is compiled once per (kernel, precision, extent class)
from csrc/apply_tu.hip, in parallel.  Objects go to _build/ at the repo root;
the library lands next to this file.
"""

from __future__ import annotations

import argparse
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(ROOT, "_build")
LIB = os.path.join(HERE, "libiwfpm.so")

ARCH = "gfx950"
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
# packed-FP32 instructions stay off in all device code
EXTRA = os.environ.get("IWFPM_EXTRA_FLAGS", "").split()
DEVICE_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}", *EXTRA,
                "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                "-I", os.path.join(ROOT, "include"), "-I", CSRC]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-pthread", f"--offload-arch={ARCH}",
              "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
              "-I", os.path.join(ROOT, "include"), "-I", CSRC]

HOST_SOURCES = ["plan.cpp", "batch.cpp", "lobpcg.cpp", "learned.cpp"]
# the eigensolver's host side (small dense Hermitian algebra): inline complex
# products (no Annex G NaN recovery calls) and contracted multiply-adds; the
# plan keeps exact, uncontracted arithmetic for its window ties
HOST_FAST = {"lobpcg.cpp", "learned.cpp"}
FAST_FLAGS = ["-O3", "-fcx-limited-range", "-ffp-contract=fast"]
DEVICE_SOURCES = ["blas_kernels.hip", "learned_kernels.hip", "eigfun.hip", "noalloc.hip"]
APPLY_TUS = [(k, r, m) for k in range(6) for r in ("float", "double") for m in (16, 32, 64)]


def _jobs():
    jobs = []
    for k, r, m in APPLY_TUS:
        obj = os.path.join(BUILD, f"apply_{k}_{r}_{m}.o")
        cmd = [HIPCC, *DEVICE_FLAGS, f"-DIWFPM_TU_KERNEL={k}", f"-DIWFPM_TU_REAL={r}",
               f"-DIWFPM_TU_MAXS={m}", "-c", os.path.join(CSRC, "apply_tu.hip"), "-o", obj]
        jobs.append((obj, cmd))
    for src in DEVICE_SOURCES:
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        jobs.append((obj, [HIPCC, *DEVICE_FLAGS, "-c", os.path.join(CSRC, src), "-o", obj]))
    for src in HOST_SOURCES:
        obj = os.path.join(BUILD, os.path.splitext(src)[0] + ".o")
        flags = HOST_FLAGS + FAST_FLAGS if src in HOST_FAST else HOST_FLAGS
        jobs.append((obj, [HIPCC, *flags, "-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]))
    return jobs


def _run(job):
    obj, cmd = job
    r = subprocess.run(cmd, capture_output=True, text=True)
    err = "\n".join(l for l in r.stderr.splitlines() if "packed-fp32-ops" not in l and l.strip())
    return obj, r.returncode, err, cmd


def build(jobs: int | None = None, verbose: bool = False) -> str:
    os.makedirs(BUILD, exist_ok=True)
    todo = _jobs()
    n = jobs or min(16, os.cpu_count() or 4)
    failed = []
    with ThreadPoolExecutor(max_workers=n) as ex:
        for obj, rc, err, cmd in ex.map(_run, todo):
            if rc != 0:
                failed.append((obj, err, cmd))
            elif verbose and err:
                print(err, file=sys.stderr)
    if failed:
        for obj, err, cmd in failed:
            print("FAILED:", " ".join(cmd), "\n", err, file=sys.stderr)
        raise RuntimeError(f"{len(failed)} compilation unit(s) failed")
    objs = [o for o, _ in todo]
    tmp = LIB + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "-pthread", f"--offload-arch={ARCH}", *objs, "-o", tmp]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("link failed:\n" + r.stderr)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    ap = argparse.ArgumentParser()
    ap.add_argument("-j", type=int, default=None)
    ap.add_argument("-v", action="store_true")
    a = ap.parse_args()
    print(build(a.j, a.v))
