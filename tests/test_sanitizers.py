"""CPU-only runs under AddressSanitizer and UndefinedBehaviorSanitizer:

* the FP64 oracle (built with gcc -fsanitize=address,undefined) solving a
  small problem, its adjoint and a bare sweep, loaded into a child Python
  with the gcc ASan runtime preloaded;
* the host side of the HIP library (every .hip source compiled by hipcc with
  the sanitizers on the host pass only) driven through its C ABI on a
  host-only context by tests/sanitize/host_abi_driver.cpp.

A sanitizer report makes the child exit non-zero."""
import os
import shutil
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

ORACLE_SCRIPT = r"""
import sys
sys.path.insert(0, ROOT)
import numpy as np
import oracle
oracle._LIB = LIBPATH
from paper_1811_12391_amd import inputs as I
prob = I.make_problem("tiny")
r = oracle.solve_problem(prob, tol=1e-8)
assert np.all(np.isfinite(r.dose)) and r.dose.max() > 0
roi = np.zeros(prob.phantom.C); roi[prob.phantom.C // 2] = 1.0
a = oracle.adjoint_problem(prob, roi, tol=1e-8)
assert np.all(np.isfinite(a.d_density))
ph = prob.phantom
sig = np.full((ph.nz, ph.ny, ph.nx), 0.5)
q = np.ones((prob.N, ph.nz, ph.ny, ph.nx))
psi, leak, nfix = oracle.sweep((ph.nx, ph.ny, ph.nz), (ph.dx, ph.dy, ph.dz), sig, prob.dirs, q)
assert np.all(np.isfinite(psi)) and np.all(np.isfinite(leak))
print("oracle ok")
"""


def _gcc_asan_runtime():
    r = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True)
    p = r.stdout.strip()
    return p if r.returncode == 0 and os.path.isabs(p) and os.path.exists(p) else None


def test_oracle_under_asan_ubsan():
    asan = _gcc_asan_runtime()
    if asan is None:
        pytest.skip("gcc ASan runtime not available")
    with tempfile.TemporaryDirectory() as td:
        lib = os.path.join(td, "liboracle_asan.so")
        subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-fPIC", "-shared", "-fopenmp", "-ffp-contract=off",
                               "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                               "-fno-omit-frame-pointer", os.path.join(ROOT, "oracle", "dct_oracle.c"),
                               "-o", lib, "-lm"])
        env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
                   UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1", OMP_NUM_THREADS="2")
        script = f"ROOT = {ROOT!r}\nLIBPATH = {lib!r}\n" + ORACLE_SCRIPT
        r = subprocess.run([sys.executable, "-c", script], env=env, capture_output=True, text=True, timeout=600)
        assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
        assert "oracle ok" in r.stdout


def test_host_abi_under_asan_ubsan():
    if shutil.which(HIPCC) is None and not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    csrc = os.path.join(ROOT, "paper_1811_12391_amd", "csrc")
    srcs = [os.path.join(csrc, f) for f in ("runtime.hip", "k_trace.hip", "k_source.hip", "k_maps.hip",
                                            "k_sweep.hip")]
    san = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
           "-Xarch_host", "-fno-sanitize-recover=undefined", "-Xarch_host", "-fno-omit-frame-pointer"]
    with tempfile.TemporaryDirectory() as td:
        exe = os.path.join(td, "host_abi_driver")
        objs = []
        procs = []
        for src in srcs + [os.path.join(ROOT, "tests", "sanitize", "host_abi_driver.cpp")]:
            obj = os.path.join(td, os.path.basename(src) + ".o")
            objs.append(obj)
            lang = ["-x", "hip"] if src.endswith(".hip") else []
            cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
                   "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                   "-I", os.path.join(ROOT, "include"), *san, *lang, "-c", src, "-o", obj]
            procs.append(subprocess.Popen(cmd, stdout=subprocess.PIPE, stderr=subprocess.STDOUT, text=True))
        for p in procs:
            out, _ = p.communicate(timeout=600)
            assert p.returncode == 0, out[-3000:]
        subprocess.check_call([HIPCC, "--offload-arch=gfx950", *san, *objs, "-o", exe])
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
                   UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
        r = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=300)
        assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
        assert "ok (0 failures)" in r.stdout
