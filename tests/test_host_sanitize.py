"""The host-side C++ (gate lowering, Pauli decomposition, the state-vector schedule builder
for forward and reverse sweeps, the tensor-network plan builder) runs clean under
AddressSanitizer and UndefinedBehaviorSanitizer: the library is rebuilt with both on its
host code, and sanitize_driver.py drives every host-only entry point over the benchmark
circuits, random circuits with every gate type, QAOA light-cone networks with the planner's
trees and slicings, and malformed inputs, in a child process that aborts on the first
report. No GPU is used."""
import os
import subprocess
import sys

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.mark.timeout(900)
def test_host_code_is_clean_under_asan_and_ubsan():
    from paper_2301_05451_amd import build

    try:
        lib_path = build.build_sanitized()
        runtime = build.sanitizer_runtime()
    except RuntimeError as e:
        pytest.skip(f"no sanitizer toolchain: {e}")
    env = dict(os.environ)
    env.update(TQ_LIBRARY=lib_path, LD_PRELOAD=runtime,
               ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([sys.executable, os.path.join(HERE, "sanitize_driver.py")], env=env, capture_output=True,
                       text=True, timeout=600)
    assert r.returncode == 0 and "sanitize driver: done" in r.stdout, (r.stdout[-2000:], r.stderr[-6000:])
