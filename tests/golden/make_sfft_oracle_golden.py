"""Write the oracle's results for the full-size sparse-FFT parity cases (Alg. 3) to
tests/golden/sfft_oracle_<case>.npz.

Only the CPU oracle (``oracle/``) and the seeded input generators (``workloads``) run here; the
GPU tests compare the library's solve of the same inputs with these files.  The oracle needs
about a minute per d = 20 case on one core, which is why its results are stored rather than
recomputed inside the GPU tests.

    python tests/golden/make_sfft_oracle_golden.py [case ...]
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle.sfft import PlantedBlackBox, sfft  # noqa: E402
from workloads import S0, planted_c3, sweep_t52, sweep_t54  # noqa: E402

STEP_KEYS = ("t", "n_It", "n_J", "L", "sumM", "calls", "uncovered", "redraws")


def cases():
    """name -> (planted polynomial, keyword arguments of Alg. 3)."""
    return {
        # d = 20, box [-32,32]^20, s = 1000, |c| in [1,10], r = 5, delta = 1e-3 (noise-free, sigma 1e-2)
        "c3_sigma0": (lambda: planted_c3(0.0), dict(delta=1e-3, s=1000, r=5, b=10, seed=1711051523)),
        "c3_sigma1e-2": (lambda: planted_c3(1e-2), dict(delta=1e-3, s=1000, r=5, b=10, seed=1711051523)),
        # setting of Table 5.2 (d = 5, N = 32, s = 1000, unit moduli): r = 2, delta = 0.1
        "t52_r2_delta0.1": (lambda: sweep_t52(0), dict(delta=0.1, s=1000, r=2, b=10, seed=S0 + 52000)),
        # setting of Table 5.4 (d = 10, N = 32, s = 1000, unit moduli, SNR 30 dB): r = 2, delta = 1e-12
        "t54_snr30_r2": (lambda: sweep_t54(0, 30.0), dict(delta=1e-12, s=1000, r=2, b=10, seed=S0 + 54000)),
    }


def input_digest(p) -> str:
    h = hashlib.sha256()
    for a in (np.ascontiguousarray(p.freqs, np.int64), np.ascontiguousarray(p.coeffs, np.complex128),
              np.ascontiguousarray(p.lo, np.int64), np.ascontiguousarray(p.hi, np.int64)):
        h.update(a.tobytes())
    h.update(repr((float(p.sigma), int(p.noise_seed))).encode())
    return h.hexdigest()


def path(name: str) -> str:
    return os.path.join(HERE, f"sfft_oracle_{name}.npz")


def make(name: str) -> None:
    mk, kw = cases()[name]
    p = mk()
    bb = PlantedBlackBox(p.freqs, p.coeffs, p.sigma, p.noise_seed)
    t0 = time.time()
    res = sfft(p.lo, p.hi, bb, kw["delta"], kw["s"], kw["s"], r=kw["r"], b=kw["b"], seed=kw["seed"])
    steps = np.array([[int(st.get(k, 0)) for k in STEP_KEYS] for st in res.steps], np.int64)
    np.savez_compressed(path(name), freqs=res.freqs.astype(np.int32), coeffs=res.coeffs.astype(np.complex128),
                        steps=steps, step_keys=np.array(STEP_KEYS), samples=np.int64(res.samples),
                        samples_full=np.int64(res.samples_full), margin=np.float64(res.margin),
                        digest=np.array(input_digest(p)),
                        kwargs=np.array(repr(sorted(kw.items()))))
    print(f"{name}: {res.freqs.shape[0]} frequencies, {res.samples} samples, margin {res.margin:.3e}, "
          f"{time.time() - t0:.1f} s", flush=True)


if __name__ == "__main__":
    for n in (sys.argv[1:] or list(cases())):
        make(n)
