"""Oracle for the inverse multiple rank-1 lattice FFT (Alg. 2), its adjoint and the Fourier matrix.

Notation (Sec. 2.1): a rank-1 lattice is Lambda(z, M) = { j z / M mod 1 : j = 0..M-1 }; a
multiple rank-1 lattice stacks L of them.  Samples are stored lattice after lattice, so lattice
l owns the slice [off_l, off_l + M_l) of a vector of length sum_l M_l, and entry j of that slice
is the value at the node j z_l / M_l mod 1 (Sec. 2.1, definition of Lambda(z, M)).

The residue of frequency k in lattice l is r_l(k) = (k . z_l) mod M_l.  k belongs to the
unaliased set I_l when no other h in I has the same residue (Alg. 1 and Alg. 2, definition of
I_l), and counter[k] is the number of lattices whose I_l contains k (Alg. 2).

Two weightings share the machinery:
  "paper": F, Alg. 2:  c_k = (1/counter_k) sum_{l : k in I_l} (1/M_l) sum_j y_l[j] e^{-2 pi i j r_l(k)/M_l},
           c_k = 0 when counter_k = 0 (reading R5: Alg. 2 assumes every k is covered).
           Its adjoint F*: y_l[j] = (1/M_l) sum_{k in I_l} (c_k/counter_k) e^{+2 pi i j r_l(k)/M_l}.
  "eval":  the Fourier matrix A(X, I) = (e^{2 pi i k.x})_{x in X, k in I} of Sec. 2.1 on the
           stacked lattice nodes: (A c)_l[j] = sum_k c_k e^{2 pi i j r_l(k)/M_l}, and
           (A* y)_k = sum_l sum_j y_l[j] e^{-2 pi i j r_l(k)/M_l}.

Tier 0 (``*_direct``) evaluates the sums term by term with phases reduced exactly in integers;
tier 1 uses numpy's FFT of each lattice slice (a library DFT of length M_l, Alg. 2 "rank-1
lattice FFT") followed by indexing at the residues.  Tier 1 is checked against tier 0 in the
tests before it is trusted.
"""
from __future__ import annotations

import numpy as np

__all__ = [
    "residues", "alias_counts", "unaliased_sets", "sample_offsets", "forward", "adjoint",
    "forward_direct", "adjoint_direct", "lattice_nodes", "fourier_matrix", "unaliased_sets_pairwise",
]


def _as_rhs(a: np.ndarray) -> tuple[np.ndarray, bool]:
    a = np.asarray(a)
    if a.ndim == 1:
        return a[None, :], True
    return a, False


def residues(freqs: np.ndarray, z: np.ndarray, M: int) -> np.ndarray:
    """r(k) = (k . z) mod M in [0, M) for every row k of ``freqs`` (exact integers)."""
    freqs = np.asarray(freqs, dtype=np.int64)
    z = np.asarray(z, dtype=np.int64)
    M = int(M)
    bound = int(np.abs(freqs).max(initial=0)) * int(np.abs(z).sum())
    if bound < (1 << 62):
        return np.mod(freqs @ z, M).astype(np.int64)
    # exact fallback with Python integers
    return np.array([sum(int(a) * int(b) for a, b in zip(k, z)) % M for k in freqs], dtype=np.int64)


def alias_counts(res: np.ndarray, M: int) -> np.ndarray:
    """Histogram cnt[m] = #{k : r(k) = m}, m = 0..M-1."""
    return np.bincount(np.asarray(res, dtype=np.int64), minlength=int(M))


def unaliased_sets(freqs, M, z):
    """Residues [L, n], membership of k in I_l as bool [L, n] and counter [n] (Alg. 2)."""
    freqs = np.asarray(freqs)
    L = len(M)
    n = freqs.shape[0]
    res = np.zeros((L, n), np.int64)
    uniq = np.zeros((L, n), bool)
    for l in range(L):
        res[l] = residues(freqs, z[l], M[l])
        cnt = alias_counts(res[l], M[l])
        uniq[l] = cnt[res[l]] == 1
    counter = uniq.sum(axis=0).astype(np.int64)
    return res, uniq, counter


def unaliased_sets_pairwise(freqs, M, z):
    """Same membership as ``unaliased_sets`` but straight from the definition of I_l: k is in
    I_l iff no h != k in I has k.z_l == h.z_l (mod M_l).  O(n^2) Python-integer arithmetic, for
    tiny inputs only."""
    freqs = [tuple(int(v) for v in row) for row in np.asarray(freqs)]
    L = len(M)
    n = len(freqs)
    uniq = np.ones((L, n), bool)
    for l in range(L):
        zl = [int(v) for v in z[l]]
        Ml = int(M[l])
        dots = [sum(a * b for a, b in zip(k, zl)) for k in freqs]
        for a in range(n):
            for b in range(n):
                if a != b and (dots[a] - dots[b]) % Ml == 0:
                    uniq[l, a] = False
                    break
    return uniq, uniq.sum(axis=0)


def sample_offsets(M) -> np.ndarray:
    """off[l] = sum_{l' < l} M_l' (length L + 1)."""
    return np.concatenate([[0], np.cumsum(np.asarray(M, dtype=np.int64))]).astype(np.int64)


def forward(freqs, M, z, samples, weights: str = "paper") -> np.ndarray:
    """Tier 1: F y (Alg. 2) or A* y, with a library FFT of every lattice slice."""
    y, squeeze = _as_rhs(samples)
    res, uniq, counter = unaliased_sets(freqs, M, z)
    off = sample_offsets(M)
    n = res.shape[1]
    out = np.zeros((y.shape[0], n), np.complex128)
    for l in range(len(M)):
        ghat = np.fft.fft(y[:, off[l]:off[l + 1]], axis=1)
        if weights == "paper":
            ghat = ghat / float(M[l])
            sel = uniq[l]
            out[:, sel] += ghat[:, res[l][sel]]
        elif weights == "eval":
            out += ghat[:, res[l]]
        else:
            raise ValueError(weights)
    if weights == "paper":
        cov = counter > 0
        out[:, cov] /= counter[cov]
        out[:, ~cov] = 0.0
    return out[0] if squeeze else out


def adjoint(freqs, M, z, coeffs, weights: str = "paper") -> np.ndarray:
    """Tier 1: F* c or A c, by filling the residue bins of every lattice and applying the
    library inverse FFT of length M_l."""
    c, squeeze = _as_rhs(coeffs)
    res, uniq, counter = unaliased_sets(freqs, M, z)
    off = sample_offsets(M)
    out = np.zeros((c.shape[0], int(off[-1])), np.complex128)
    for l in range(len(M)):
        Ml = int(M[l])
        bins = np.zeros((c.shape[0], Ml), np.complex128)
        if weights == "paper":
            sel = uniq[l]
            bins[:, res[l][sel]] = c[:, sel] / counter[sel]
            out[:, off[l]:off[l + 1]] = np.fft.ifft(bins, axis=1)       # (1/M) sum_m bins e^{+}
        elif weights == "eval":
            for r in range(c.shape[0]):
                np.add.at(bins[r], res[l], c[r])
            out[:, off[l]:off[l + 1]] = np.fft.ifft(bins, axis=1) * Ml   # sum_m bins e^{+}
        else:
            raise ValueError(weights)
    return out[0] if squeeze else out


def _phase_table(M: int, j: np.ndarray, r: np.ndarray, sign: float) -> np.ndarray:
    """e^{sign 2 pi i (j r mod M)/M} with the product reduced exactly in integers."""
    if M >= (1 << 31):
        raise ValueError("tier-0 phases need M < 2^31 so that j*r fits in int64")
    q = np.mod(np.multiply.outer(j.astype(np.int64), np.asarray(r, np.int64)), M).astype(np.float64)
    return np.exp(sign * 2j * np.pi * q / M)


def forward_direct(freqs, M, z, samples, weights: str = "paper", subset=None) -> np.ndarray:
    """Tier 0: the sums of Alg. 2 (or of A*) evaluated term by term.  ``subset`` restricts the
    output to the given frequency indices (the unaliased sets still use the whole of I)."""
    y, squeeze = _as_rhs(samples)
    res, uniq, counter = unaliased_sets(freqs, M, z)
    off = sample_offsets(M)
    idx = np.arange(res.shape[1]) if subset is None else np.asarray(subset)
    out = np.zeros((y.shape[0], len(idx)), np.complex128)
    for l in range(len(M)):
        Ml = int(M[l])
        j = np.arange(Ml, dtype=np.int64)
        ks = idx if weights == "eval" else idx[uniq[l][idx]]
        pos = np.arange(len(idx)) if weights == "eval" else np.nonzero(uniq[l][idx])[0]
        for chunk in range(0, len(ks), 64):
            kk = ks[chunk:chunk + 64]
            E = _phase_table(Ml, j, res[l][kk], -1.0)                  # [M, chunk]
            g = y[:, off[l]:off[l + 1]] @ E
            if weights == "paper":
                g = g / Ml
            out[:, pos[chunk:chunk + 64]] += g
    if weights == "paper":
        cnt = counter[idx]
        cov = cnt > 0
        out[:, cov] /= cnt[cov]
        out[:, ~cov] = 0.0
    return out[0] if squeeze else out


def adjoint_direct(freqs, M, z, coeffs, weights: str = "paper") -> np.ndarray:
    """Tier 0: F* c or A c evaluated term by term."""
    c, squeeze = _as_rhs(coeffs)
    res, uniq, counter = unaliased_sets(freqs, M, z)
    off = sample_offsets(M)
    out = np.zeros((c.shape[0], int(off[-1])), np.complex128)
    for l in range(len(M)):
        Ml = int(M[l])
        j = np.arange(Ml, dtype=np.int64)
        if weights == "paper":
            sel = np.nonzero(uniq[l])[0]
            w = c[:, sel] / counter[sel]
        else:
            sel = np.arange(res.shape[1])
            w = c
        E = _phase_table(Ml, j, res[l][sel], +1.0)                     # [M, |sel|]
        blk = w @ E.T
        if weights == "paper":
            blk = blk / Ml
        out[:, off[l]:off[l + 1]] = blk
    return out[0] if squeeze else out


def lattice_nodes(z, M) -> np.ndarray:
    """Nodes x_j = (j z mod M) / M of the rank-1 lattice Lambda(z, M), j = 0..M-1 (Sec. 2.1)."""
    z = np.asarray(z, dtype=np.int64)
    j = np.arange(int(M), dtype=np.int64)
    return np.mod(np.multiply.outer(j, z), int(M)).astype(np.float64) / float(M)


def fourier_matrix(nodes: np.ndarray, freqs: np.ndarray) -> np.ndarray:
    """A(X, I) = (exp(2 pi i k . x))_{x in X, k in I} (Sec. 2.1), from explicit real nodes."""
    return np.exp(2j * np.pi * (np.asarray(nodes, np.float64) @ np.asarray(freqs, np.float64).T))
