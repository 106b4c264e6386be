"""Host-side logic of the library under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

tests/host/host_logic_check.cpp includes paper_1711_05152_amd/csrc/host_logic.h (the distinct-row
check of a plan, the prime search and L_max of Alg. 1, the SplitMix64 streams of the method's
draws, the caching allocator's bookkeeping) and is built here with g++ and the sanitizers; the
random-stream values it prints are compared with the oracle's independent implementation."""
import os
import shutil
import subprocess

import pytest

from oracle import rng as R

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "tests", "host", "host_logic_check.cpp")
CSRC = os.path.join(ROOT, "paper_1711_05152_amd", "csrc")


@pytest.fixture(scope="module")
def run_output(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("no host C++ compiler")
    exe = str(tmp_path_factory.mktemp("host") / "host_logic_check")
    subprocess.run([gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=all", "-I" + CSRC, SRC, "-o", exe], check=True, capture_output=True,
                   text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    res = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert res.returncode == 0, res.stderr[-4000:]
    assert "ERROR: AddressSanitizer" not in res.stderr and "runtime error" not in res.stderr, res.stderr[-4000:]
    return res.stdout.splitlines()


def test_sanitized_checks_pass(run_output):
    for name in ("distinct_rows", "primes", "streams", "cache"):
        assert f"ok {name}" in run_output


def test_streams_match_oracle(run_output):
    keys, draws, ints = {}, 0, 0
    for line in run_output:
        f = line.split()
        if f[0] == "key":
            seed, k = int(f[1]), int(f[2])
            assert k == R.key(seed, R.Z, 3, 1, 7)
            keys[seed] = k
        elif f[0] == "draw":
            seed, c, v, u = int(f[1]), int(f[2]), int(f[3]), float(f[4])
            assert v == R.draw(keys[seed], c)
            assert u == R.uniform01(keys[seed], c)
            draws += 1
        elif f[0] == "int":
            seed, M, v, ctr = (int(x) for x in f[1:5])
            assert (v, ctr) == R.uniform_int(keys[seed], 0, M)
            ints += 1
    assert len(keys) == 3 and draws == 12 and ints == 15
