"""Counter-based random streams used for every random draw of the method (oracle side).

The paper draws generating vectors "uniformly at random" (Alg. 1) and anchor components
"uniformly at random" (Alg. 3, steps 1, 2a and 2c) without naming a generator.  Both sides of
this project use the same published generator, each with its own implementation: the output
function of SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number generators",
OOPSLA 2014) applied to a counter.

  GAMMA          = 0x9E3779B97F4A7C15
  mix64(x)       : x ^= x >> 30; x *= 0xBF58476D1CE4E5B9; x ^= x >> 27;
                   x *= 0x94D049BB133111EB; x ^= x >> 31            (all mod 2^64)
  key(seed, f_1..f_m) : k = seed; for each field f: k = mix64(k + GAMMA * (f + 1))
  draw(k, c)     = mix64(k + GAMMA * (c + 1))        (c-th output of SplitMix64 seeded with k)
  uniform01(k,c) = (draw(k, c) >> 11) * 2^-53                   in [0, 1)
  uniform_int(k, c, M): take draws c, c+1, ... until u >= (2^64 mod M); return u mod M
                        (unbiased rejection; the counter advances past every draw consumed)

Streams (purpose tag, then fields):
  Z        = 1 : (t, attempt, L)  generating vector of lattice L of construction call ``attempt``
                 at dimension step t; components drawn in order with uniform_int.
  ANCHOR1D = 2 : (t, i)  1-D projection anchors at step t, repetition i: component c (0-based)
                 is uniform01(key, c), component t-1 unused.
  ANCHOR   = 3 : (t, i)  lattice-step anchors x'_{t+1..d}: component c is uniform01(key, c).
  NOISE    = 4 : (kind, t, i)  complex Gaussian noise of sample g (kind 0: 1-D projection
                 samples, kind 1: lattice samples): Box-Muller from u1 = uniform01(key, 2g),
                 u2 = uniform01(key, 2g+1): eta = sigma/sqrt(2) * sqrt(-2 ln(1-u1)) *
                 (cos 2 pi u2 + i sin 2 pi u2)   (noise model of Sec. 5.2).
  ZREDRAW  = 5 : (t, attempt, L, a)  a-th redraw (a >= 1) of the generating vector of lattice L
                 in the construction variant that redraws z_L until the lattice reconstructs a
                 frequency not yet covered (the earlier construction the paper compares Alg. 1
                 with); a = 0 is the Z stream.
"""
from __future__ import annotations

import numpy as np

MASK = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15
C1 = 0xBF58476D1CE4E5B9
C2 = 0x94D049BB133111EB

Z, ANCHOR1D, ANCHOR, NOISE, ZREDRAW = 1, 2, 3, 4, 5


def mix64(x: int) -> int:
    x &= MASK
    x ^= x >> 30
    x = (x * C1) & MASK
    x ^= x >> 27
    x = (x * C2) & MASK
    x ^= x >> 31
    return x


def key(seed: int, *fields: int) -> int:
    k = seed & MASK
    for f in fields:
        k = mix64(k + GAMMA * (int(f) + 1))
    return k


def draw(k: int, c: int) -> int:
    return mix64(k + GAMMA * (int(c) + 1))


def uniform01(k: int, c: int) -> float:
    return (draw(k, c) >> 11) * (2.0 ** -53)


def uniform_int(k: int, c: int, M: int) -> tuple[int, int]:
    """Unbiased integer in [0, M) from the stream; returns (value, next counter)."""
    if M <= 0:
        raise ValueError("M must be positive")
    floor_reject = (1 << 64) % M
    while True:
        u = draw(k, c)
        c += 1
        if u >= floor_reject:
            return u % M, c


# ---- vectorised forms (numpy uint64 arithmetic wraps mod 2^64) ---------------------------------

def _mix64_vec(x: np.ndarray) -> np.ndarray:
    x = x.astype(np.uint64, copy=True)
    x ^= x >> np.uint64(30)
    x *= np.uint64(C1)
    x ^= x >> np.uint64(27)
    x *= np.uint64(C2)
    x ^= x >> np.uint64(31)
    return x


def uniform01_vec(k: int, ctr: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        x = np.uint64(k) + np.uint64(GAMMA) * (ctr.astype(np.uint64) + np.uint64(1))
        u = _mix64_vec(x)
    return (u >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def gaussian_noise(seed: int, kind: int, t: int, i: int, g: np.ndarray, sigma: float) -> np.ndarray:
    """Complex Gaussian noise for sample indices g (Box-Muller on the NOISE stream)."""
    k = key(seed, NOISE, kind, t, i)
    g = np.asarray(g, dtype=np.uint64)
    u1 = uniform01_vec(k, np.uint64(2) * g)
    u2 = uniform01_vec(k, np.uint64(2) * g + np.uint64(1))
    rad = np.sqrt(-2.0 * np.log1p(-u1))
    return (sigma / np.sqrt(2.0)) * rad * (np.cos(2.0 * np.pi * u2) + 1j * np.sin(2.0 * np.pi * u2))
