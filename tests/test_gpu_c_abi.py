"""The C ABI from plain C, without the Python binding: tests/c_abi_example.c, compiled by the host C
compiler against include/mr1l.h and libmr1l.so, runs one forward and one adjoint transform on the
GPU, and its results match the oracle."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from gpu_util import require_gpu
from oracle import mr1l as O
from workloads import rng_for, transform_problem

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_plain_c_program_matches_oracle(tmp_path):
    require_gpu()
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no host C compiler")
    from paper_1711_05152_amd import _lib
    pkg = os.path.dirname(_lib.LIB_PATH)
    exe = tmp_path / "c_abi_example"
    subprocess.run([cc, "-std=c99", "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(ROOT, "include"),
                    "-I", "/opt/rocm/include", os.path.join(ROOT, "tests", "c_abi_example.c"), "-L", pkg, "-lmr1l",
                    "-L/opt/rocm/lib", "-lamdhip64", f"-Wl,-rpath,{pkg}:/opt/rocm/lib", "-o", str(exe)], check=True)
    p = transform_problem(rng_for(305), 3000, 7, 30, 5, 3000, 6000, n_rhs=1)
    n, d = p.freqs.shape
    sm = int(p.M.sum())
    np.array([d, n, len(p.M), sm], np.int64).tofile(tmp_path / "shape")
    np.ascontiguousarray(p.freqs, np.int32).tofile(tmp_path / "freqs")
    np.ascontiguousarray(p.M, np.int64).tofile(tmp_path / "M")
    np.ascontiguousarray(p.z, np.int64).tofile(tmp_path / "z")
    np.ascontiguousarray(p.samples[0], np.complex128).tofile(tmp_path / "samples")
    np.ascontiguousarray(p.coeffs[0], np.complex128).tofile(tmp_path / "coeffs")
    print("running the plain-C example", flush=True)
    r = subprocess.run([str(exe), str(tmp_path)], capture_output=True, text=True, timeout=120)
    print(r.stdout, r.stderr, flush=True)
    assert r.returncode == 0, r.stderr
    c = np.fromfile(tmp_path / "coeffs_out", np.complex128)
    y = np.fromfile(tmp_path / "samples_out", np.complex128)
    c_ref = O.forward(p.freqs, p.M, p.z, p.samples[0])
    y_ref = O.adjoint(p.freqs, p.M, p.z, p.coeffs[0])
    assert np.abs(c - c_ref).max() <= 1e-11 * max(1.0, np.abs(c_ref).max())
    assert np.abs(y - y_ref).max() <= 1e-11 * max(1.0, np.abs(y_ref).max())
