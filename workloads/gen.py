"""Seeded synthetic workloads for the multiple rank-1 lattice FFT and the sparse FFT driver.

Everything here is an *input*: frequency sets drawn uniformly from boxes without replacement,
prime lattice sizes and generating vectors for the standalone transforms, complex Gaussian
sample vectors and planted sparse trigonometric polynomials of the kinds used in the paper's
numerical section (Sec. 5.1 random sparse polynomials; Sec. 5.2 unit-modulus coefficients with
additive complex Gaussian noise).  None of the method's arithmetic lives here.

All draws use numpy's PCG64 seeded from ``SeedSequence([S0, workload_id, *extra])`` so that the
CPU oracle, the GPU tests and the benchmark see bit-identical inputs.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "S0", "rng_for", "primes_between", "distinct_freqs", "cn01", "TransformProblem",
    "PlantedPoly", "transform_problem", "standalone_c2", "planted_c1", "planted_c3",
    "batched_c4", "lsq_c5", "random_planted", "sweep_t52", "sweep_t54",
]

S0 = 1711051520  # base seed for every synthetic workload


def rng_for(workload: int, *extra: int) -> np.random.Generator:
    """Independent PCG64 stream for ``(S0, workload, *extra)``."""
    return np.random.Generator(np.random.PCG64(np.random.SeedSequence([S0, workload, *extra])))


def primes_between(lo: int, hi: int) -> np.ndarray:
    """All primes p with lo <= p <= hi (input-side helper: picks lattice sizes for the
    standalone-transform workloads, which the paper draws at random from a range)."""
    hi = int(hi)
    sieve = np.ones(hi + 1, dtype=bool)
    sieve[:2] = False
    for q in range(2, int(math.isqrt(hi)) + 1):
        if sieve[q]:
            sieve[q * q:: q] = False
    out = np.nonzero(sieve)[0]
    return out[out >= lo].astype(np.int64)


def _row_keys(rows: np.ndarray, lo: int) -> np.ndarray:
    """64-bit polynomial hash of integer rows (distinct rows collide with probability ~2^-64)."""
    h = np.zeros(rows.shape[0], np.uint64)
    mult = np.uint64(0x9E3779B97F4A7C15)
    with np.errstate(over="ignore"):
        for c in range(rows.shape[1]):
            h = h * mult + (rows[:, c].astype(np.int64) - lo).astype(np.uint64) + np.uint64(1)
    return h


def distinct_freqs(rng: np.random.Generator, n: int, d: int, lo: int, hi: int) -> np.ndarray:
    """n distinct integer vectors drawn uniformly without replacement from the box [lo, hi]^d,
    returned in draw order as int32 [n, d] (later repeats of an earlier row are dropped)."""
    span = hi - lo + 1
    if n > span ** d:
        raise ValueError("box too small for the requested number of distinct frequencies")
    if n == 0:
        return np.zeros((0, d), np.int32)
    acc = np.zeros((0, d), np.int32)
    while acc.shape[0] < n:
        batch = rng.integers(lo, hi + 1, size=(max(64, 2 * (n - acc.shape[0])), d),
                             dtype=np.int64).astype(np.int32)
        allrows = np.concatenate([acc, batch])
        if span ** d <= (1 << 62):
            keys = np.zeros(allrows.shape[0], np.int64)     # exact mixed-radix code of the row
            for c in range(d):
                keys = keys * span + (allrows[:, c].astype(np.int64) - lo)
        else:
            keys = _row_keys(allrows, lo)
        _, first = np.unique(keys, return_index=True)
        acc = allrows[np.sort(first)]          # unique rows, in order of first draw
    return np.ascontiguousarray(acc[:n])


def cn01(rng: np.random.Generator, shape) -> np.ndarray:
    """Standard circular complex Gaussian CN(0,1): (N(0,1) + i N(0,1)) / sqrt(2)."""
    return ((rng.standard_normal(shape) + 1j * rng.standard_normal(shape)) / math.sqrt(2.0)).astype(
        np.complex128)


@dataclass
class TransformProblem:
    """One multiple rank-1 lattice transform instance: frequency set, lattices and samples."""
    freqs: np.ndarray        # int32 [n, d]
    M: np.ndarray            # int64 [L]
    z: np.ndarray            # int64 [L, d]
    samples: np.ndarray      # complex128 [n_rhs, sum(M)]
    coeffs: np.ndarray       # complex128 [n_rhs, n] (random coefficients for adjoint tests)

    @property
    def n(self) -> int:
        return int(self.freqs.shape[0])

    @property
    def d(self) -> int:
        return int(self.freqs.shape[1])


def transform_problem(rng: np.random.Generator, n: int, d: int, box: int, L: int,
                      m_lo: int, m_hi: int, n_rhs: int = 1, prime: bool = True,
                      with_data: bool = True) -> TransformProblem:
    """Frequencies uniform in [-box, box]^d without replacement; L distinct lattice sizes drawn
    uniformly among the primes (or all integers) in [m_lo, m_hi]; generators uniform in
    [0, M_l - 1]^d; samples and coefficients CN(0,1) (left empty when ``with_data`` is False,
    for consumers that draw them on the device)."""
    freqs = distinct_freqs(rng, n, d, -box, box)
    pool = primes_between(m_lo, m_hi) if prime else np.arange(m_lo, m_hi + 1, dtype=np.int64)
    if len(pool) < L:
        raise ValueError("not enough lattice sizes in range")
    M = np.sort(rng.choice(pool, size=L, replace=False)).astype(np.int64)
    M = rng.permutation(M)
    z = np.stack([rng.integers(0, m, size=d, dtype=np.int64) for m in M]) if L else np.zeros((0, d), np.int64)
    if with_data:
        samples = cn01(rng, (n_rhs, int(M.sum())))
        coeffs = cn01(rng, (n_rhs, n))
    else:
        samples = np.zeros((n_rhs, 0), np.complex128)
        coeffs = np.zeros((n_rhs, 0), np.complex128)
    return TransformProblem(freqs, M, z.astype(np.int64), samples, coeffs)


def standalone_c2(n: int = 1 << 16, d: int = 10, box: int = 64, L: int = 16) -> TransformProblem:
    """Standalone transform workload: |I| = 2^16 frequencies uniform in [-64,64]^10, L = 16
    distinct primes uniform in [|I|, 2|I|], complex Gaussian samples."""
    return transform_problem(rng_for(2), n, d, box, L, n, 2 * n)


@dataclass
class PlantedPoly:
    """Sparse trigonometric polynomial p(x) = sum_h c_h exp(2 pi i h.x) (the black box)."""
    freqs: np.ndarray        # int32 [s, d]
    coeffs: np.ndarray       # complex128 [s]
    lo: np.ndarray           # int32 [d] search box lower corner
    hi: np.ndarray           # int32 [d] search box upper corner
    sigma: float = 0.0       # complex Gaussian noise level on every sample
    noise_seed: int = 0      # seed of the counter-based noise stream

    @property
    def d(self) -> int:
        return int(self.freqs.shape[1])

    @property
    def s(self) -> int:
        return int(self.freqs.shape[0])


def random_planted(rng: np.random.Generator, d: int, N: int, s: int, mag: str = "unit",
                   sigma: float = 0.0, noise_seed: int = 0) -> PlantedPoly:
    """s distinct frequencies uniform in [-N, N]^d.  ``mag``: "unit" = exp(2 pi i phi) with phi
    uniform in [0,1) (Sec. 5.1 Example 5.3, Sec. 5.2); "u1_10" = modulus uniform in [1,10] with
    uniform phase; "box" = uniform in [-1,1) + [-1,1)i rejecting modulus < 1e-6 (Sec. 5.1)."""
    freqs = distinct_freqs(rng, s, d, -N, N)
    if mag == "unit":
        c = np.exp(2j * np.pi * rng.random(s))
    elif mag == "u1_10":
        c = rng.uniform(1.0, 10.0, s) * np.exp(2j * np.pi * rng.random(s))
    elif mag == "box":
        c = np.empty(s, np.complex128)
        i = 0
        while i < s:
            v = complex(rng.uniform(-1, 1), rng.uniform(-1, 1))
            if abs(v) >= 1e-6:
                c[i] = v
                i += 1
    else:
        raise ValueError(mag)
    lo = np.full(d, -N, np.int32)
    hi = np.full(d, N, np.int32)
    return PlantedPoly(freqs, c.astype(np.complex128), lo, hi, sigma, noise_seed)


def planted_c1() -> PlantedPoly:
    """Plain sparse FFT workload: d=5, box [-8,8]^5, s=50 unit-modulus coefficients, no noise."""
    return random_planted(rng_for(1), 5, 8, 50, "unit")


def planted_c3(sigma: float = 0.0) -> PlantedPoly:
    """Sparse FFT at scale: d=20, box [-32,32]^20, s=1000, modulus uniform in [1,10], random
    phase; optional complex Gaussian noise sigma (noise stream seeded from S0 + 3)."""
    return random_planted(rng_for(3), 20, 32, 1000, "u1_10", sigma, S0 + 3)


def batched_c4(count: int = 512, d: int = 15, box: int = 32, seed_extra: int = 0,
               log2_lo: float = 8.0, log2_hi: float = 18.0, with_data: bool = True) -> list[TransformProblem]:
    """Batched workload: ``count`` independent transforms, |I_b| = round(2^U), U uniform in
    [log2_lo, log2_hi]; frequencies uniform in [-32,32]^15; L_b = ceil(log2 |I_b|) distinct
    primes uniform in [|I_b|, 2|I_b|]."""
    rng = rng_for(4, seed_extra)
    out = []
    for _ in range(count):
        n = int(round(2.0 ** rng.uniform(log2_lo, log2_hi)))
        L = int(math.ceil(math.log2(n)))
        out.append(transform_problem(rng, n, d, box, L, n, 2 * n, with_data=with_data))
    return out


def sweep_t52(rep: int) -> PlantedPoly:
    """Success-rate sweep instance (setting of Table 5.2): d = 5, box [-32,32]^5, s = 1000
    frequencies, coefficients e^{2 pi i phi}, phi uniform in [0,1); repetition ``rep``."""
    return random_planted(rng_for(6, rep), 5, 32, 1000, "unit")


def sweep_t54(rep: int, snr_db: float) -> PlantedPoly:
    """Noise sweep instance (setting of Table 5.4): d = 10, box [-32,32]^10, s = 1000,
    coefficients e^{2 pi i phi}, complex Gaussian noise with sigma = sqrt(s / SNR),
    SNR = 10^(snr_db / 10); noise stream seeded per repetition."""
    sigma = math.sqrt(1000.0 / 10.0 ** (snr_db / 10.0))
    return random_planted(rng_for(7, rep), 10, 32, 1000, "unit", sigma, S0 + 7000 + rep)


def lsq_c5(n: int = 1 << 20, d: int = 30, box: int = 16, L: int = 20, n_rhs: int = 64):
    """Least-squares workload frame: frequencies, lattices and the seed for the planted
    coefficients / noise (drawn on the device by the consumer because of their size)."""
    rng = rng_for(5)
    freqs = distinct_freqs(rng, n, d, -box, box)
    pool = primes_between(n, 2 * n)
    M = rng.permutation(np.sort(rng.choice(pool, size=L, replace=False))).astype(np.int64)
    z = np.stack([rng.integers(0, m, size=d, dtype=np.int64) for m in M]).astype(np.int64)
    return freqs, M, z, int(rng.integers(0, 2**62))
