"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer, and the
no-underflow condition (R29) of the binary32 reference.

* The oracle's C sources, built with -fsanitize=address,undefined, run every
  oracle pin in a child pytest (the sanitizer runtimes preloaded into it).
* The C ABI's host code (tpc_api.cpp: argument validation, workspace
  carving) is built with g++ and the same sanitizers against stand-in
  launchers that check every carved workspace array lies inside the
  caller's workspace (tests/sanitize/), and driven over a range of sizes and
  invalid arguments.
* R29: no operation of the binary32 oracle delivers a subnormal (the IEEE
  underflow flag stays clear) on the tracking and refit workloads, so the
  production build's flushing of subnormals cannot change a result there
  and the deterministic build's gradual underflow is never exercised.
"""
import os
import subprocess
import sys
import tempfile

import numpy as np
import pytest

import oracle
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-fno-sanitize-recover=all"]


def _runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True).stdout
    return p.strip()


def test_oracle_pins_under_address_and_ub_sanitizers():
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not (os.path.isabs(asan) and os.path.isabs(ubsan)):
        pytest.skip("gcc sanitizer runtimes not found")
    with tempfile.TemporaryDirectory(prefix="orc_san_") as d:
        lib = oracle.build(out=os.path.join(d, "liboracle.so"), extra=tuple(SAN))
        env = dict(os.environ, TPC_ORACLE_LIB=lib, LD_PRELOAD=f"{asan}:{ubsan}",
                   ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
                   UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
        r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                            "tests/test_oracle_pins.py", "tests/test_oracle_refit.py"],
                           cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
        assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
        assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr


def test_abi_host_code_under_address_and_ub_sanitizers():
    with tempfile.TemporaryDirectory(prefix="abi_san_") as d:
        exe = os.path.join(d, "abi_harness")
        cmd = ["g++", "-std=c++17", "-O1", "-g", *SAN, "-D__HIP_PLATFORM_AMD__",
               "-I/opt/rocm/include", "-I", os.path.join(ROOT, "include"),
               "-I", os.path.join(ROOT, "paper_2511_17018_amd", "csrc"),
               os.path.join(ROOT, "tests", "sanitize", "abi_harness.cpp"),
               os.path.join(ROOT, "tests", "sanitize", "stub_launchers.cpp"),
               os.path.join(ROOT, "paper_2511_17018_amd", "csrc", "tpc_api.cpp"), "-o", exe]
        subprocess.run(cmd, check=True, capture_output=True, text=True)
        r = subprocess.run([exe], capture_output=True, text=True, timeout=600,
                           env=dict(os.environ, ASAN_OPTIONS="detect_leaks=1"))
        assert r.returncode == 0, r.stdout + r.stderr
        assert "abi harness ok" in r.stdout


def test_binary32_reference_never_underflows():
    G = synth.geometry()
    P = dict(oracle.DEFAULT_PARAMS)
    # the flag works: a curvature step of a tiny q/pT delivers a subnormal
    oracle.underflow_raised(True)
    oracle.propagate(G, P, [0, 0, 0.1, 0.2, 1e-36], np.eye(5)[np.tril_indices(5)], 100.0,
                     101.0, prec=32)
    assert oracle.underflow_raised(True)
    for ev in (synth.config1(), synth.config2(), synth.config4(n_inst=6)):
        oracle.underflow_raised(True)
        oracle.track(G, P, ev.inst_off, ev.y, ev.z, ev.row, prec=32)
        assert not oracle.underflow_raised(True), ev.name
    ev = synth.config5(n_found=2000)
    oracle.underflow_raised(True)
    oracle.refit(G, P, ev, ev.extra["hit_off"], ev.extra["hit_clu"], ev.extra["seed_par"],
                 ev.extra["D_true"], prec=32)
    assert not oracle.underflow_raised(True)
