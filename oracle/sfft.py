"""Oracle for the dimension-incremental sparse FFT on multiple rank-1 lattices (Alg. 3, "MLFFT").

Steps in the paper's order (Alg. 3, Sec. 3.1; general scheme Sec. 2.2):

  step 1   K_1 = max P_1(Gamma) - min P_1(Gamma) + 1.  For i = 1..r: draw anchors x'_2..x'_d,
           p~_{1,k} = (1/K_1) sum_l p(l/K_1, x'_2, .., x'_d) e^{-2 pi i l k/K_1},
           I^(1) gets the (up to) s_local largest |p~_{1,k}| >= delta.
  step 2   for t = 2..d:
     2a    same 1-D detection for component t (anchors on all other components) -> I^(t);
           the factor 1/K_t is used here too (reading R1: it is printed in step 1 only, but the
           aliasing identity for the 1-D projections holds with it).
     2b    J_t = (I^(1..t-1) x I^(t)) (the intersection with the projected box is the product
           itself for a box search space); Alg. 1 with c = 2, gamma = 1/2, repeated until
           reconstructing, at most b calls (readings R3, R4).
     2c-e  r~ = r, s~ = s_local if t < d, else r~ = 1, s~ = s.  For i = 1..r~: draw anchors
           x'_{t+1..d}, sample p on the lattice nodes with the anchors appended, compute
           p~_{(1..t),k}, k in J_t, with Alg. 2, and add the (up to) s~ largest |p~| >= delta to
           I^(1..t).
  step 3   output I^(1..d) and the coefficients of the final (t = d, r~ = 1) transform.

Selection (reading R6): keep k with re^2 + im^2 >= delta^2 (IEEE double, no fused multiply-add),
order by that value descending, ties by ascending position in the lexicographically sorted
candidate list, keep the first s.  Sets are kept lexicographically sorted (reading R8).
Empty I^(t) or J_t ends the run with the empty set (reading R14).  For d = 1 the output is
I^(1) with the coefficients of the last repetition.

Component order (the remark that any permutation of the components may be used): with
``order`` = (pi_1, .., pi_d), step t works on component pi_t, i.e. the run above on the search
space and black box with their components permuted; every random stream is keyed by the step t.
The output frequencies are returned in the original components, in the lexicographic order of
the processing order (reading R20).  ``redraw`` selects the construction variant of
``oracle.construct`` for step 2b.

The black box is a planted sparse polynomial; its samples on a lattice come either from direct
evaluation at explicit nodes (tier 0) or from the identity
  p(j z/M mod 1, x~) = sum_h [c_h e^{2 pi i h_{t+1..d} . x~}] e^{2 pi i j (h_{1..t} . z mod M)/M}
evaluated with a library inverse FFT of length M (tier 1).
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import rng as R
from .construct import construct_retry
from .mr1l import forward, forward_direct, residues, sample_offsets, lattice_nodes, unaliased_sets

__all__ = ["PlantedBlackBox", "select_top", "decision_margin", "projection_1d", "sfft", "SfftResult"]


def _sqabs(v: np.ndarray) -> np.ndarray:
    v = np.asarray(v, np.complex128)
    re = v.real.copy()
    im = v.imag.copy()
    return re * re + im * im


def decision_margin(vals: np.ndarray, delta: float, s: int) -> float:
    """Smallest relative distance of a selection decision of ``select_top`` from a flip: of each
    |v|^2 from delta^2, and, when more than s pass the threshold, of the s-th largest from the
    (s+1)-th.  inf when nothing is decided by a comparison of values."""
    key = _sqabs(vals)
    m = np.inf
    if delta > 0.0 and len(key):
        m = float(np.min(np.abs(key - delta * delta)) / (delta * delta))
    above = np.sort(key[key >= delta * delta])[::-1]
    if len(above) > s >= 1:
        m = min(m, float((above[s - 1] - above[s]) / max(above[s - 1], np.finfo(float).tiny)))
    return m


def select_top(vals: np.ndarray, delta: float, s: int) -> np.ndarray:
    """Positions of the (up to) s largest |v| >= delta (reading R6), ascending."""
    key = _sqabs(vals)
    cand = np.nonzero(key >= delta * delta)[0]
    if len(cand) > s:
        order = np.lexsort((cand, -key[cand]))      # primary: key descending, then position
        cand = np.sort(cand[order[:s]])
    return cand


class PlantedBlackBox:
    """p(x) = sum_h c_h e^{2 pi i h . x} plus optional complex Gaussian noise per sample."""

    def __init__(self, freqs, coeffs, sigma: float = 0.0, noise_seed: int = 0):
        self.freqs = np.asarray(freqs, np.int64)
        self.coeffs = np.asarray(coeffs, np.complex128)
        self.sigma = float(sigma)
        self.noise_seed = int(noise_seed)
        self.d = self.freqs.shape[1]

    def eval_nodes(self, nodes: np.ndarray) -> np.ndarray:
        """Direct evaluation at explicit nodes [m, d] (tier 0)."""
        out = np.zeros(nodes.shape[0], np.complex128)
        for a in range(0, nodes.shape[0], 4096):
            ph = nodes[a:a + 4096] @ self.freqs.T.astype(np.float64)
            out[a:a + 4096] = np.exp(2j * np.pi * ph) @ self.coeffs
        return out

    def permuted(self, order) -> "PlantedBlackBox":
        """The same polynomial with its components in the processing order ``order``."""
        return PlantedBlackBox(self.freqs[:, np.asarray(order)], self.coeffs, self.sigma, self.noise_seed)

    def _noise(self, kind, t, i, count):
        if self.sigma == 0.0:
            return 0.0
        return R.gaussian_noise(self.noise_seed, kind, t, i, np.arange(count), self.sigma)

    def sample_1d(self, t: int, i: int, anchors: np.ndarray, K: int) -> np.ndarray:
        """Samples at (x'_1, .., l/K, .., x'_d), l = 0..K-1, component t (1-based) varying.
        Phases h_t l / K are reduced in integers."""
        h = self.freqs
        c = t - 1
        other = np.delete(np.arange(self.d), c)
        base = np.exp(2j * np.pi * (h[:, other].astype(np.float64) @ anchors[other])) * self.coeffs
        ell = np.arange(K, dtype=np.int64)
        q = np.mod(np.multiply.outer(ell, h[:, c]), K).astype(np.float64) / K
        y = np.exp(2j * np.pi * q) @ base
        return y + self._noise(0, t, i, K)

    def sample_lattice(self, t: int, i: int, M, z, anchors_tail: np.ndarray, tier: int = 1):
        """Samples on the stacked lattices (components 1..t) with anchors x'_{t+1..d}."""
        M = np.asarray(M, np.int64)
        off = sample_offsets(M)
        y = np.zeros(int(off[-1]), np.complex128)
        h = self.freqs
        if tier == 0:
            for l in range(len(M)):
                nodes = np.zeros((int(M[l]), self.d))
                nodes[:, :t] = lattice_nodes(z[l], M[l])
                nodes[:, t:] = anchors_tail
                y[off[l]:off[l + 1]] = self.eval_nodes(nodes)
        else:
            w = self.coeffs * np.exp(2j * np.pi * (h[:, t:].astype(np.float64) @ anchors_tail))
            for l in range(len(M)):
                Ml = int(M[l])
                bins = np.zeros(Ml, np.complex128)
                np.add.at(bins, residues(h[:, :t], z[l], Ml), w)
                y[off[l]:off[l + 1]] = np.fft.ifft(bins) * Ml
        return y + self._noise(1, t, i, len(y))


def projection_1d(y: np.ndarray, lo: int, hi: int) -> np.ndarray:
    """p~_{t,k} = (1/K) sum_l y[l] e^{-2 pi i l k / K} for k = lo..hi, K = hi - lo + 1, written
    out term by term with l k reduced mod K in integers (Alg. 3 steps 1 and 2a, reading R1)."""
    K = hi - lo + 1
    ks = np.arange(lo, hi + 1, dtype=np.int64)
    ell = np.arange(K, dtype=np.int64)
    q = np.mod(np.multiply.outer(ks, ell), K).astype(np.float64) / K
    return (np.exp(-2j * np.pi * q) @ y) / K


@dataclass
class SfftResult:
    freqs: np.ndarray
    coeffs: np.ndarray
    steps: list = field(default_factory=list)
    samples: int = 0            # distinct nodes: sum over steps of r K_t and r~ (1 - L + sum M)
    samples_full: int = 0       # values drawn when every lattice is sampled in full
    margin: float = np.inf      # smallest decision_margin over every selection of the run


def sfft(box_lo, box_hi, black_box, delta: float, s: int, s_local: int | None = None,
         r: int = 1, b: int = 10, seed: int = 0, tier: int = 1, zero_anchors: bool = False,
         redraw: int = 0, order=None, delta_1d: float | None = None, c: float = 2.0,
         gamma: float = 0.5) -> SfftResult:
    """Alg. 3 on the box search space [box_lo, box_hi] (inclusive, per component).
    ``zero_anchors``: anchor components fixed to 0 instead of drawn (the r = 1 setting of the
    remark on coefficients with a common sign of real or imaginary part, Sec. 3.1).
    ``redraw``: construction variant (see ``oracle.construct``); ``order``: component order.
    ``delta_1d``: threshold of the 1-D detections (steps 1 and 2a) when it differs from
    ``delta`` (the threshold-based truncation of Sec. 5.3 uses delta / 10 there).
    ``c``, ``gamma``: the parameters step 2b passes to Alg. 1 (Alg. 3 fixes 2 and 1/2).  Each step
    records ``uncovered``, the frequencies of J_t in no I_l of the kept lattices (reading R4)."""
    if order is not None and list(order) != list(range(len(box_lo))):
        order = np.asarray(order, np.int64)
        assert sorted(order.tolist()) == list(range(len(box_lo))), "order must be a permutation"
        res = sfft(np.asarray(box_lo)[order], np.asarray(box_hi)[order], black_box.permuted(order), delta, s,
                   s_local, r, b, seed, tier, zero_anchors, redraw, None, delta_1d, c, gamma)
        orig = np.empty_like(res.freqs)
        orig[:, order] = res.freqs
        res.freqs = orig
        return res
    lo = np.asarray(box_lo, np.int64)
    hi = np.asarray(box_hi, np.int64)
    d = len(lo)
    s_local = s if s_local is None else s_local
    delta_1d = delta if delta_1d is None else delta_1d
    res = SfftResult(np.zeros((0, d), np.int32), np.zeros(0, np.complex128))

    def detect_1d(t):
        K = int(hi[t - 1] - lo[t - 1] + 1)
        flags = np.zeros(K, bool)
        last = None
        for i in range(1, r + 1):
            k1 = R.key(seed, R.ANCHOR1D, t, i)
            anchors = np.zeros(d) if zero_anchors else np.array([R.uniform01(k1, c) for c in range(d)])
            y = black_box.sample_1d(t, i, anchors, K)
            pt = projection_1d(y, int(lo[t - 1]), int(hi[t - 1]))
            flags[select_top(pt, delta_1d, s_local)] = True
            res.margin = min(res.margin, decision_margin(pt, delta_1d, s_local))
            last = pt
        res.samples += r * K
        res.samples_full += r * K
        ks = np.arange(lo[t - 1], hi[t - 1] + 1, dtype=np.int64)
        return ks[flags], last[flags]

    I1, c1 = detect_1d(1)
    prev = I1.reshape(-1, 1)
    res.steps.append(dict(t=1, n_It=len(I1)))
    if d == 1:
        res.freqs = prev.astype(np.int32)
        res.coeffs = c1
        return res
    if len(I1) == 0:
        return res
    last_coeffs = None
    for t in range(2, d + 1):
        It, _ = detect_1d(t)
        if len(It) == 0 or prev.shape[0] == 0:
            res.steps.append(dict(t=t, n_It=len(It), n_J=0))
            return res
        J = np.concatenate([np.repeat(prev, len(It), axis=0),
                            np.tile(It, prev.shape[0]).reshape(-1, 1)], axis=1)
        cstats: dict = {}
        M, z, covered, calls = construct_retry(J, b, c=c, gamma=gamma, seed=seed, t=t, redraw=redraw,
                                               stats=cstats)
        uncovered = int(np.count_nonzero(unaliased_sets(J, M, z)[2] == 0))
        r_t, s_t = (r, s_local) if t < d else (1, s)
        flags = np.zeros(J.shape[0], bool)
        for i in range(1, r_t + 1):
            k1 = R.key(seed, R.ANCHOR, t, i)
            tail = np.zeros(d - t) if zero_anchors else np.array([R.uniform01(k1, c) for c in range(t, d)])
            y = black_box.sample_lattice(t, i, M, z, tail, tier=tier)
            pt = forward(J, M, z, y) if tier == 1 else forward_direct(J, M, z, y)
            flags[select_top(pt, delta, s_t)] = True
            res.margin = min(res.margin, decision_margin(pt, delta, s_t))
            last_coeffs = pt
            res.samples += 1 - len(M) + int(np.sum(M))
            res.samples_full += int(np.sum(M))
        res.steps.append(dict(t=t, n_It=len(It), n_J=J.shape[0], L=len(M), sumM=int(np.sum(M)),
                              calls=calls, covered=covered, uncovered=uncovered, M=M, z=z,
                              redraws=cstats.get("redraws", 0)))
        prev = J[flags]
    res.freqs = prev.astype(np.int32)
    res.coeffs = last_coeffs[flags]
    return res
