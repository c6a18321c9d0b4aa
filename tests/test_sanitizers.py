"""AddressSanitizer + UndefinedBehaviorSanitizer builds of the host code,
run on the CPU: the FP64 oracle (gcc) over solves, residuals, Jacobians and
LU calls of every mechanism kind, and the library's host runtime (hipcc,
sanitizers on the host pass only; the device code is built as usual) under
the ABI's host-side tests.  Each build is cached under _build/sanitize/ and
redone when its sources change; each run is a subprocess with the sanitizer
runtime preloaded, and any sanitizer report fails the test."""
import glob
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
OUT = os.path.join(ROOT, "_build", "sanitize")
ORACLE = os.path.join(ROOT, "oracle")
CSRC = os.path.join(ROOT, "paper_2005_11468_amd", "csrc")
REPORT_MARKS = ("ERROR: AddressSanitizer", "runtime error:", "ERROR: LeakSanitizer")


def _stale(target, sources):
    if not os.path.exists(target):
        return True
    return max(os.path.getmtime(s) for s in sources) > os.path.getmtime(target)


def _run(script, preload):
    env = dict(os.environ)
    env["LD_PRELOAD"] = preload
    env["ASAN_OPTIONS"] = "detect_leaks=0:verify_asan_link_order=0:abort_on_error=0:halt_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    r = subprocess.run([sys.executable, "-c", script], env=env, capture_output=True, text=True,
                       timeout=900, cwd=ROOT)
    text = r.stdout + r.stderr
    assert r.returncode == 0, text[-4000:]
    for mark in REPORT_MARKS:
        assert mark not in text, text[-4000:]
    return text


ORACLE_SCRIPT = r"""
import sys, numpy as np
sys.path.insert(0, {root!r})
from oracle import oracle as O
O.LIB_PATH = {lib!r}
O.build = lambda force=False: O.LIB_PATH
from psr_inputs import workload
from tests import tiny_mechs as tm
for name in ("isothermal", "energy", "soot"):
    mech, cond, x0, energy = workload(name, 3)
    M = O.Mechanism(mech)
    b = 1
    args = (cond["P"][b], cond["tau"][b], cond["T_in"][b], cond["Y_in"][:, b].copy(), energy)
    x = x0[:, b].copy()
    F = M.residual(*args, x)
    J = M.jacobian(*args, x)
    Jc = M.jacobian(*args, x, complex_step=True)
    M.scaled_residual(*args, x)
    M.mass_diag(*args, x)
    lu, piv, info = O.lu_factor(J + np.eye(len(x)))
    O.lu_solve(lu, piv, F)
    assert np.all(np.isfinite(F)) and np.all(np.isfinite(J))
    opts = O.default_opts(max_lin=60 if name == "soot" else 1500)
    xs, st = O.solve_batch(mech, cond, x0, energy, idx=np.array([0]), opts=opts)
mech = tm.small_network()
cond = {{"P": np.full(2, 101325.0), "tau": np.array([1e-3, 1e-2]), "T_in": np.full(2, 1400.0),
        "Y_in": np.full((mech["species_elems"].shape[0], 2), 1.0 / mech["species_elems"].shape[0])}}
O.sweep_batch(mech, cond, cond["Y_in"].copy(), False, "tau", np.array([[1e-3, 1e-2], [2e-3, 2e-2]]))
print("oracle sanitizer run done")
"""


@pytest.mark.timeout(900)
def test_oracle_under_address_and_undefined_sanitizers():
    os.makedirs(OUT, exist_ok=True)
    lib = os.path.join(OUT, "liboracle_asan.so")
    srcs = [os.path.join(ORACLE, f) for f in ("psr_oracle.c", "psr_oracle.h", "residual_body.inc")]
    if _stale(lib, srcs):
        subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-fPIC", "-shared", "-fno-omit-frame-pointer",
                        "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
                        "-o", lib, os.path.join(ORACLE, "psr_oracle.c"), "-lm"], check=True)
    pre = " ".join(subprocess.run(["gcc", f"-print-file-name={n}"], capture_output=True, text=True,
                                  check=True).stdout.strip() for n in ("libasan.so", "libubsan.so"))
    out = _run(ORACLE_SCRIPT.format(root=ROOT, lib=lib), pre)
    assert "oracle sanitizer run done" in out


HOST_SCRIPT = r"""
import sys
sys.path.insert(0, {root!r})
import paper_2005_11468_amd._lib as L
L.LIB_PATH = {lib!r}
import pytest
sys.exit(pytest.main(["-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu",
                      {root!r} + "/tests/test_abi_cpu.py"]))
"""


@pytest.mark.timeout(900)
def test_host_runtime_under_address_and_undefined_sanitizers():
    rt = sorted(glob.glob("/opt/rocm/lib/llvm/lib/clang/*/lib/linux/libclang_rt.asan-x86_64.so"))
    if not rt or not os.path.exists("/opt/rocm/bin/hipcc"):
        pytest.skip("hipcc or its AddressSanitizer runtime is not installed")
    os.makedirs(OUT, exist_ok=True)
    lib = os.path.join(OUT, "libpsr_asan.so")
    srcs = glob.glob(os.path.join(CSRC, "*"))
    if _stale(lib, srcs):
        cmd = ["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC", "-shared",
               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
               "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
               "-Xarch_host", "-fno-omit-frame-pointer", "-Wno-unused-result", "-Wno-unused-value",
               "-o", lib + ".tmp", os.path.join(CSRC, "psr_lib.hip")]
        subprocess.run(cmd, check=True, capture_output=True)
        os.replace(lib + ".tmp", lib)
    out = _run(HOST_SCRIPT.format(root=ROOT, lib=lib), rt[-1])
    assert " passed" in out and " failed" not in out, out[-2000:]
