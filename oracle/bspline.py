"""Oracle for the B-spline test function of Sec. 5.3 and its relative L2 approximation error.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The univariate factor (Sec. 5.3) is the periodic B-spline of order m,

    N_m(x) = C_m sum_{k in Z} sinc(pi k / m)^m (-1)^k e^{2 pi i k x},   sinc(u) = sin(u) / u,

with C_m > 0 chosen so that the L2(T) norm of N_m is one.  The test function of the section is

    f(x) = prod_{t in {1,3,8}} N_2(x_t) + prod_{t in {2,5,6,10}} N_4(x_t) + prod_{t in {4,7,9}} N_6(x_t)

on T^10.  This module handles any weighted sum of such products: term tau is described by one
row of an integer matrix ``orders[tau, c]``, the order m of the factor N_m(x_c) of component c, or
0 for a factor 1.

Closed form used for point evaluation: the coefficients C_m sinc(pi k/m)^m (-1)^k are, up to the
factor C_m m, those of the 1-periodisation of the cardinal B-spline B_m (support [0, m], order m)
compressed by m: N_m(x) = C_m m B_m(m (x mod 1)).  B_m is written out with truncated powers,

    B_m(u) = 1/(m-1)! sum_{j=0..m} (-1)^j binom(m, j) (u - j)_+^(m-1),

evaluated only for u <= m/2 (by the symmetry B_m(u) = B_m(m - u)) so that few terms cancel.
The normalisation C_m is computed from its definition: C_m^-2 = sum_k sinc(pi k/m)^(2m)
(Parseval), the series summed to |k| <= 10^5 (tail below 10^-16 for m >= 2; for m = 1 every
term but k = 0 vanishes).

Fourier coefficients of f: term tau contributes w_tau prod_c N^_{m_tau,c}(k_c) when k_c = 0 on every
component with no factor, else nothing.  The squared norm ||f||^2 = sum_{tau,tau'} w w' prod_c
<g_tau,c, g_tau',c> uses <N_m, 1> = N^_m(0) = C_m and <N_m, N_m'> = sum_k N^_m(k) N^_m'(k).

Relative L2 error of an approximation p = sum_{k in I} p~_k e^{2 pi i k.x} (Sec. 5.3, by Parseval):

    ||f - p|| / ||f|| = sqrt(||f||^2 - sum_{k in I} |f^_k|^2 + sum_{k in I} |p~_k - f^_k|^2) / ||f||.
"""
from __future__ import annotations

import math

import numpy as np

from .mr1l import lattice_nodes, sample_offsets

__all__ = ["cardinal_bspline", "norm_const", "N", "N_hat", "TensorBsplineSum", "paper_f10_orders"]

_SERIES_K = 100_000


def cardinal_bspline(m: int, u) -> np.ndarray:
    """B_m(u), the cardinal B-spline of order m on [0, m] (zero outside), from truncated powers."""
    u = np.asarray(u, np.float64)
    v = np.where(u <= 0.5 * m, u, m - u)           # symmetry about m/2
    out = np.zeros_like(v)
    inside = (v >= 0.0) & (u < m)
    for j in range(0, m // 2 + 1):
        w = v - j
        if m == 1:
            term = (w >= 0.0).astype(np.float64)     # (u - j)_+^0 = [u >= j]
        else:
            term = np.where(w > 0.0, w, 0.0) ** (m - 1)
        out += (-1) ** j * math.comb(m, j) * term
    return np.where(inside, out / math.factorial(m - 1), 0.0)


_CM: dict[int, float] = {}


def norm_const(m: int) -> float:
    """C_m with ||N_m||_{L2(T)} = 1: C_m^-2 = sum_k sinc(pi k/m)^(2m) (Parseval on the series)."""
    if m not in _CM:
        if m == 1:
            _CM[m] = 1.0
        else:
            k = np.arange(_SERIES_K, 0, -1, dtype=np.float64)      # smallest terms first
            a = np.pi * k / m
            terms = (np.sin(a) / a) ** (2 * m)
            _CM[m] = 1.0 / math.sqrt(1.0 + 2.0 * math.fsum(terms))
    return _CM[m]


def N(m: int, x) -> np.ndarray:
    """The periodic B-spline N_m(x) of Sec. 5.3 at real x (any real; taken mod 1)."""
    x = np.asarray(x, np.float64)
    return norm_const(m) * m * cardinal_bspline(m, m * np.mod(x, 1.0))


def N_hat(m: int, k) -> np.ndarray:
    """Fourier coefficient C_m sinc(pi k/m)^m (-1)^k of N_m at integer k (Sec. 5.3)."""
    k = np.asarray(k, np.int64)
    a = np.pi * k.astype(np.float64) / m
    with np.errstate(invalid="ignore", divide="ignore"):
        sinc = np.where(k == 0, 1.0, np.sin(a) / np.where(k == 0, 1.0, a))
    # sin(pi k/m) vanishes exactly at nonzero multiples of m
    sinc = np.where((k != 0) & (k % m == 0), 0.0, sinc)
    sign = np.where(k % 2 == 0, 1.0, -1.0)
    return norm_const(m) * sinc ** m * sign


def _inner(m1: int, m2: int) -> float:
    """<g1, g2> on T for factors N_m1 and N_m2 (0 meaning the constant 1)."""
    if m1 == 0 and m2 == 0:
        return 1.0
    if m1 == 0 or m2 == 0:
        return norm_const(m1 or m2)                     # integral of N_m = N^_m(0)
    if m1 == m2:
        return 1.0
    k = np.arange(_SERIES_K, 0, -1, dtype=np.int64)
    return float(N_hat(m1, 0) * N_hat(m2, 0) + 2.0 * math.fsum(N_hat(m1, k) * N_hat(m2, k)))


def paper_f10_orders() -> np.ndarray:
    """orders matrix of the test function of Sec. 5.3 on T^10 (components 1-based in the paper)."""
    o = np.zeros((3, 10), np.int32)
    for t in (1, 3, 8):
        o[0, t - 1] = 2
    for t in (2, 5, 6, 10):
        o[1, t - 1] = 4
    for t in (4, 7, 9):
        o[2, t - 1] = 6
    return o


class TensorBsplineSum:
    """f(x) = sum_tau w_tau prod_c N_{orders[tau, c]}(x_c) (factor 1 where the order is 0), with the
    black-box interface of ``oracle.sfft`` (explicit nodes; no noise)."""

    def __init__(self, orders, weights=None):
        self.orders = np.asarray(orders, np.int64)
        assert self.orders.ndim == 2 and (self.orders >= 0).all()
        self.T, self.d = self.orders.shape
        self.weights = np.ones(self.T) if weights is None else np.asarray(weights, np.float64)

    # -- point values ---------------------------------------------------------------------------
    def eval_nodes(self, nodes: np.ndarray) -> np.ndarray:
        nodes = np.asarray(nodes, np.float64)
        out = np.zeros(nodes.shape[0])
        for tau in range(self.T):
            prod = np.full(nodes.shape[0], self.weights[tau])
            for c in range(self.d):
                m = int(self.orders[tau, c])
                if m > 0:
                    prod = prod * N(m, nodes[:, c])
            out += prod
        return out.astype(np.complex128)

    def permuted(self, order) -> "TensorBsplineSum":
        return TensorBsplineSum(self.orders[:, np.asarray(order)], self.weights)

    def sample_1d(self, t: int, i: int, anchors: np.ndarray, K: int) -> np.ndarray:
        """Values at (x'_1, .., l/K, .., x'_d), l = 0..K-1, component t (1-based) varying."""
        nodes = np.tile(np.asarray(anchors, np.float64), (K, 1))
        nodes[:, t - 1] = np.arange(K, dtype=np.float64) / K
        return self.eval_nodes(nodes)

    def sample_lattice(self, t: int, i: int, M, z, anchors_tail: np.ndarray, tier: int = 1):
        """Values on the stacked lattices (components 1..t) with anchors x'_{t+1..d}; always by
        point evaluation at the explicit nodes (``tier`` only selects the transform)."""
        M = np.asarray(M, np.int64)
        off = sample_offsets(M)
        y = np.zeros(int(off[-1]), np.complex128)
        for l in range(len(M)):
            nodes = np.zeros((int(M[l]), self.d))
            nodes[:, :t] = lattice_nodes(z[l], M[l])
            nodes[:, t:] = anchors_tail
            y[off[l]:off[l + 1]] = self.eval_nodes(nodes)
        return y

    # -- Fourier side ---------------------------------------------------------------------------
    def fhat(self, freqs) -> np.ndarray:
        """f^_k for the rows k of ``freqs`` [n, d]."""
        k = np.asarray(freqs, np.int64).reshape(-1, self.d)
        out = np.zeros(k.shape[0])
        for tau in range(self.T):
            v = np.full(k.shape[0], self.weights[tau])
            for c in range(self.d):
                m = int(self.orders[tau, c])
                v = v * (N_hat(m, k[:, c]) if m > 0 else (k[:, c] == 0).astype(np.float64))
            out += v
        return out

    def norm2(self) -> float:
        """||f||^2 over T^d."""
        tot = 0.0
        for a in range(self.T):
            for b in range(self.T):
                p = self.weights[a] * self.weights[b]
                for c in range(self.d):
                    p *= _inner(int(self.orders[a, c]), int(self.orders[b, c]))
                tot += p
        return tot

    def rel_l2_error(self, freqs, coeffs) -> float:
        """||f - p|| / ||f|| for p = sum_{k in I} coeffs_k e^{2 pi i k.x} (Sec. 5.3, Parseval)."""
        fh = self.fhat(freqs)
        c = np.asarray(coeffs, np.complex128).reshape(-1)
        nf2 = self.norm2()
        e2 = nf2 - float(np.sum(fh * fh)) + float(np.sum(np.abs(c - fh) ** 2))
        return math.sqrt(max(e2, 0.0) / nf2)
