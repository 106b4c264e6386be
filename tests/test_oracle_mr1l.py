"""Pins of the oracle's transforms against the mathematics (no GPU).

Each test checks the oracle against something other than itself: brute-force definitions,
the dense Fourier matrix of Sec. 2.1 built from explicit real nodes, exact recovery of
polynomials supported on I from a reconstructing multiple rank-1 lattice (Alg. 2 and the
identity for projected coefficients in Sec. 4.1), a textbook special case, and the adjoint
identity.
"""
import numpy as np
import pytest

from oracle import mr1l as O
from workloads import rng_for, transform_problem, distinct_freqs, cn01


def _small(seed, n=40, d=3, box=6, L=4, mlo=50, mhi=120, n_rhs=2):
    return transform_problem(rng_for(100, seed), n, d, box, L, mlo, mhi, n_rhs=n_rhs)


@pytest.mark.parametrize("seed", range(4))
def test_residues_bruteforce(seed):
    p = _small(seed)
    for l in range(len(p.M)):
        r = O.residues(p.freqs, p.z[l], p.M[l])
        ref = [sum(int(a) * int(b) for a, b in zip(k, p.z[l])) % int(p.M[l]) for k in p.freqs]
        assert r.tolist() == ref
        assert r.min() >= 0 and r.max() < p.M[l]


def test_residues_negative_and_large():
    freqs = np.array([[-5, 3], [7, -9], [0, 0], [-1, -1]], np.int32)
    z = np.array([2**40 + 3, 2**41 - 1], np.int64)
    M = 2**45 + 59
    r = O.residues(freqs, z, M)
    ref = [(int(a) * int(z[0]) + int(b) * int(z[1])) % M for a, b in freqs]
    assert r.tolist() == ref


@pytest.mark.parametrize("seed", range(4))
def test_unaliased_sets_match_pairwise_definition(seed):
    p = _small(seed, n=60, mlo=40, mhi=90)
    res, uniq, counter = O.unaliased_sets(p.freqs, p.M, p.z)
    uniq2, counter2 = O.unaliased_sets_pairwise(p.freqs, p.M, p.z)
    assert np.array_equal(uniq, uniq2)
    assert np.array_equal(counter, counter2)
    for l in range(len(p.M)):
        cnt = O.alias_counts(res[l], p.M[l])
        assert cnt.sum() == p.n                              # every k lands in one bin
        assert (cnt == 1).sum() == uniq[l].sum()             # singleton bins <-> I_l


def _poly_samples(freqs, M, z, c):
    """Samples of p(x) = sum_k c_k e^{2 pi i k.x} on the stacked lattices from the dense
    Fourier matrix on explicit real nodes (independent of residues)."""
    return np.concatenate([O.fourier_matrix(O.lattice_nodes(z[l], M[l]), freqs) @ c
                           for l in range(len(M))])


@pytest.mark.parametrize("seed", range(3))
def test_forward_exact_recovery(seed):
    """Alg. 2 returns the coefficients of a polynomial supported on I at every covered k."""
    p = _small(seed, n=50, L=6, mlo=100, mhi=200)
    _, _, counter = O.unaliased_sets(p.freqs, p.M, p.z)
    c = p.coeffs[0]
    y = _poly_samples(p.freqs, p.M, p.z, c)
    for got in (O.forward_direct(p.freqs, p.M, p.z, y), O.forward(p.freqs, p.M, p.z, y)):
        cov = counter > 0
        assert np.abs(got[cov] - c[cov]).max() < 1e-12
        assert np.all(got[~cov] == 0)


@pytest.mark.parametrize("seed", range(3))
def test_forward_is_dense_left_inverse(seed):
    """F A(Lambda, I) = identity on covered columns, zero rows for uncovered k."""
    p = _small(seed, n=30, L=3, mlo=40, mhi=80)
    _, _, counter = O.unaliased_sets(p.freqs, p.M, p.z)
    A = np.concatenate([O.fourier_matrix(O.lattice_nodes(p.z[l], p.M[l]), p.freqs)
                        for l in range(len(p.M))])
    FA = np.stack([O.forward(p.freqs, p.M, p.z, A[:, col]) for col in range(p.n)], axis=1)
    expect = np.diag((counter > 0).astype(float))
    assert np.abs(FA - expect).max() < 1e-12


@pytest.mark.parametrize("weights", ["paper", "eval"])
@pytest.mark.parametrize("seed", range(3))
def test_tier1_matches_tier0(weights, seed):
    p = _small(seed, n=80, L=5, mlo=60, mhi=150)
    f1 = O.forward(p.freqs, p.M, p.z, p.samples, weights)
    f0 = O.forward_direct(p.freqs, p.M, p.z, p.samples, weights)
    assert np.abs(f1 - f0).max() < 1e-12 * max(1.0, np.abs(f0).max())
    a1 = O.adjoint(p.freqs, p.M, p.z, p.coeffs, weights)
    a0 = O.adjoint_direct(p.freqs, p.M, p.z, p.coeffs, weights)
    assert np.abs(a1 - a0).max() < 1e-12 * max(1.0, np.abs(a0).max())


def test_eval_mode_is_fourier_matrix():
    p = _small(7, n=35, L=3, mlo=30, mhi=70)
    A = np.concatenate([O.fourier_matrix(O.lattice_nodes(p.z[l], p.M[l]), p.freqs)
                        for l in range(len(p.M))])
    c = p.coeffs[0]
    y = p.samples[0]
    assert np.abs(O.adjoint(p.freqs, p.M, p.z, c, "eval") - A @ c).max() < 1e-11
    assert np.abs(O.forward(p.freqs, p.M, p.z, y, "eval") - A.conj().T @ y).max() < 1e-11


@pytest.mark.parametrize("weights", ["paper", "eval"])
def test_adjoint_identity(weights):
    p = _small(11, n=200, d=4, box=10, L=6, mlo=200, mhi=400, n_rhs=1)
    y = p.samples[0]
    c = p.coeffs[0]
    lhs = np.vdot(c, O.forward(p.freqs, p.M, p.z, y, weights))     # <F y, c>
    rhs = np.vdot(O.adjoint(p.freqs, p.M, p.z, c, weights), y)     # <y, F* c>
    assert abs(lhs - rhs) <= 1e-13 * max(1.0, abs(lhs))


def test_special_case_single_lattice_is_dft():
    """L = 1, d = 1, z = 1, I = {-(M-1)/2..(M-1)/2}: F y is the DFT of y divided by M,
    re-indexed by k mod M (textbook DFT via numpy's FFT)."""
    M = 97
    freqs = np.arange(-(M - 1) // 2, (M - 1) // 2 + 1, dtype=np.int32).reshape(-1, 1)
    y = cn01(rng_for(101), M)
    got = O.forward_direct(freqs, [M], [[1]], y)
    ref = np.fft.fft(y)[np.mod(freqs[:, 0], M)] / M
    assert np.abs(got - ref).max() < 1e-13


def test_special_case_crt_lattice_is_2d_dft():
    """d = 2, coprime n1, n2, z = (n2, n1), M = n1 n2: by the Chinese remainder theorem the nodes
    (j/n1 mod 1, j/n2 mod 1) run through the full n1 x n2 tensor grid, every k in the box
    {0..n1-1} x {0..n2-1} is unaliased, and F y is the textbook 2-D DFT of the grid samples
    divided by M."""
    n1, n2 = 7, 5
    M = n1 * n2
    k1, k2 = np.meshgrid(np.arange(n1), np.arange(n2), indexing="ij")
    freqs = np.stack([k1.ravel(), k2.ravel()], axis=1).astype(np.int32)
    y = cn01(rng_for(102), M)
    Y = np.zeros((n1, n2), np.complex128)
    for j in range(M):
        Y[j % n1, j % n2] = y[j]
    ref = np.fft.fft2(Y) / M
    for got in (O.forward_direct(freqs, [M], [[n2, n1]], y), O.forward(freqs, [M], [[n2, n1]], y)):
        assert np.abs(got - ref[freqs[:, 0], freqs[:, 1]]).max() < 1e-13


def test_uncovered_frequency_gives_zero():
    """Reading R5: counter 0 -> coefficient 0 (and the adjoint ignores it)."""
    freqs = np.array([[0], [5], [10]], np.int32)   # all congruent mod 5
    M, z = [5], [[1]]
    y = cn01(rng_for(103), 5)
    out = O.forward(freqs, M, z, y)
    assert np.all(out == 0)
    assert np.all(O.adjoint(freqs, M, z, np.ones(3)) == 0)


def test_distinct_freqs_generator():
    f = distinct_freqs(rng_for(104), 100, 3, -2, 2)
    assert len(np.unique(f, axis=0)) == 100 and f.min() >= -2 and f.max() <= 2
