"""Oracle for Alg. 1: reconstructing multiple rank-1 lattices with pairwise distinct prime sizes.

Steps, in the paper's order (Alg. 1, Sec. 2.1):
  1. L_max = ceil(c^2/(c-1)^2 * (ln|I| - ln gamma) / 2)
  2. lambda = c (|I| - 1)
  3. P^I_{lambda,L_max}: the L_max smallest primes p > lambda for which k -> (k mod p)
     (componentwise) is injective on I (definition of P^I and of P^I_{lambda,L_max}, Sec. 2.1)
  4. for L = 1..L_max: M_L = p_L; z_L uniform in [0, M_L - 1]^d; I_L = frequencies of I whose
     residue modulo M_L is not shared; I~ = I~ u I_L; stop once I~ = I.
  Output: all lattices drawn so far (also those that added nothing to I~; Alg. 2 averages over
  every l with k in I_l).

Alg. 3 step 2b calls Alg. 1 with c = 2, gamma = 1/2 and repeats it until the result is
reconstructing, at most b calls in total (reading R3 of "up to b-1 times"); if none of the b
calls covers I the last one is kept (reading R4) and the uncovered frequencies have counter 0.

The generating vectors come from the Z stream of ``oracle.rng`` keyed by (t, attempt, L).

Variant (``redraw`` > 0): the earlier construction that Alg. 1 modifies (remark after Alg. 1)
checks, after drawing z_L, whether Lambda(z_L, M_L) reconstructs a frequency of I not yet in I~;
if not, z_L is drawn again (ZREDRAW stream, redraw a = 1, 2, ...) and the lattice is kept only
once it adds a frequency.  Reading: at most ``redraw`` redraws per lattice, after which the last
draw is kept (the unbounded loop of the original could run forever when no generating vector
separates a remaining frequency).
"""
from __future__ import annotations

import math

import numpy as np

from . import rng as R
from .mr1l import unaliased_sets

__all__ = ["lmax", "lam", "is_prime", "prime_sizes", "construct", "construct_retry", "b_rule",
           "r_rule", "b_rule_r1", "sample_bound"]


def lmax(n: int, c: float = 2.0, gamma: float = 0.5) -> int:
    """Maximal number of rank-1 lattices (Alg. 1, first step)."""
    return int(math.ceil(c * c / ((c - 1.0) * (c - 1.0)) * (math.log(n) - math.log(gamma)) / 2.0))


def lam(n: int, c: float = 2.0) -> float:
    """Lower bound for the lattice sizes (Alg. 1, second step)."""
    return c * (n - 1)


def is_prime(p: int) -> bool:
    if p < 2:
        return False
    if p % 2 == 0:
        return p == 2
    q = 3
    while q * q <= p:
        if p % q == 0:
            return False
        q += 2
    return True


def _injective_mod(freqs: np.ndarray, p: int) -> bool:
    """|{k mod p : k in I}| == |I| (componentwise mod), the membership test of P^I."""
    if freqs.shape[0] <= 1:
        return True
    expansion = int((freqs.max(axis=0) - freqs.min(axis=0)).max())
    if p > expansion:
        # two distinct k differ in some component by 0 < |k_j - h_j| <= expansion < p
        return True
    red = np.mod(freqs.astype(np.int64), p)
    return len({tuple(r) for r in red.tolist()}) == freqs.shape[0]


def prime_sizes(freqs: np.ndarray, lam_value: float, count: int) -> list[int]:
    """The ``count`` smallest primes p > lambda that lie in P^I (eq. defining P^I_{lambda,L_max})."""
    out: list[int] = []
    p = int(math.floor(lam_value)) + 1
    while len(out) < count:
        if is_prime(p) and _injective_mod(freqs, p):
            out.append(p)
        p += 1
    return out


def _draw_z(k: int, d: int, M: int) -> list[int]:
    ctr = 0
    z = []
    for _ in range(d):
        v, ctr = R.uniform_int(k, ctr, M)
        z.append(v)
    return z


def construct(freqs, c: float = 2.0, gamma: float = 0.5, seed: int = 0, t: int = 0,
              attempt: int = 0, redraw: int = 0, stats: dict | None = None):
    """One call of Alg. 1 (``redraw`` > 0: the redraw variant of the module docstring).
    Returns (M [L], z [L, d], covered); ``stats['redraws']`` counts the redraws."""
    freqs = np.asarray(freqs, dtype=np.int64)
    n, d = freqs.shape
    if n == 0:
        return np.zeros(0, np.int64), np.zeros((0, d), np.int64), True
    L_max = lmax(n, c, gamma)
    primes = prime_sizes(freqs, lam(n, c), L_max)
    Ms: list[int] = []
    zs: list[list[int]] = []
    covered = np.zeros(n, bool)
    for L in range(1, L_max + 1):
        M_L = primes[L - 1]
        z_L = _draw_z(R.key(seed, R.Z, t, attempt, L), d, M_L)
        _, uniq, _ = unaliased_sets(freqs, [M_L], [z_L])
        a = 0
        while redraw > 0 and a < redraw and not (uniq[0] & ~covered).any():
            a += 1
            z_L = _draw_z(R.key(seed, R.ZREDRAW, t, attempt, L, a), d, M_L)
            _, uniq, _ = unaliased_sets(freqs, [M_L], [z_L])
        if stats is not None:
            stats["redraws"] = stats.get("redraws", 0) + a
        Ms.append(M_L)
        zs.append(z_L)
        covered |= uniq[0]
        if covered.all():
            break
    return np.array(Ms, np.int64), np.array(zs, np.int64).reshape(len(Ms), d), bool(covered.all())


def construct_retry(freqs, b: int, c: float = 2.0, gamma: float = 0.5, seed: int = 0, t: int = 0,
                    redraw: int = 0, stats: dict | None = None):
    """Alg. 1 called until reconstructing, at most b calls (Alg. 3 step 2b).
    Returns (M, z, covered, calls)."""
    result = None
    for attempt in range(max(1, b)):
        result = construct(freqs, c, gamma, seed, t, attempt, redraw, stats)
        if result[2]:
            return result + (attempt + 1,)
    return result + (max(1, b),)


def b_rule(d: int, eps: float, gamma: float = 0.5) -> int:
    """Number of Alg. 1 calls from the lemma on repeated lattice searches (Sec. 4.1):
    ceil((log 3 + log d - log eps)/|log gamma|), the least b with gamma^b <= eps/(3d)."""
    return int(math.ceil((math.log(3) + math.log(d) - math.log(eps)) / abs(math.log(gamma))))


def b_rule_r1(d: int, eps: float) -> int:
    """b for the r = 1 setting of Sec. 4.3: ceil((log d - log eps)/log 2), the least b with
    2^-b <= eps/d."""
    return int(math.ceil((math.log(d) - math.log(eps)) / math.log(2)))


def r_rule(supp: int, d: int, eps: float) -> int:
    """Detection iterations from the lemma and theorem of Sec. 4.1:
    ceil(2 |supp| (log 3 + log d + log |supp| - log eps)); enough for the union bound
    |supp| q^r <= eps/(3d) with q <= 3|supp|/(3|supp| + 2)."""
    return int(math.ceil(2 * supp * (math.log(3) + math.log(d) + math.log(supp) - math.log(eps))))


def sample_bound(r: int, s: int, N: int) -> float:
    """Upper bound of Sec. 3.2 on |X^(1..t)|: 2 Lt max{2(rs(2N+1)-1), 4 Lt ln Lt},
    Lt = ceil(2 ln(rs(2N+1)) + 2 ln 2)."""
    m = r * s * (2 * N + 1)
    Lt = int(math.ceil(2 * math.log(m) + 2 * math.log(2)))
    return 2 * Lt * max(2 * (m - 1), 4 * Lt * math.log(Lt))
