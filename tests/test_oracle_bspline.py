"""Pins of the B-spline test function oracle (Sec. 5.3): closed forms, textbook values, exact
quadrature of piecewise polynomials, FFTs of samples, and the sparse FFT driver on it.  CPU only."""
import math
from fractions import Fraction

import numpy as np
import pytest

from oracle import bspline as B
from oracle import sfft as S


def _central_value(order: int, u: int) -> Fraction:
    """Cardinal B-spline of the given order at integer u, exactly (truncated powers in rationals)."""
    s = Fraction(0)
    for j in range(order + 1):
        w = Fraction(u - j)
        if w > 0:
            s += (-1) ** j * math.comb(order, j) * w ** (order - 1)
    return s / math.factorial(order - 1)


def _gl_cells(n_cells: int, pts: int):
    """Gauss-Legendre nodes and weights on each of n_cells equal cells of [0, 1]."""
    g, w = np.polynomial.legendre.leggauss(pts)
    x = ((np.arange(n_cells)[:, None] + 0.5 * (g[None, :] + 1.0)) / n_cells).ravel()
    wt = np.tile(0.5 * w / n_cells, n_cells)
    return x, wt


# ---- the univariate factor -------------------------------------------------------------------------

def test_textbook_central_bspline_values():
    # central values of the cardinal B-splines of orders 4, 8, 12 (standard table values)
    assert _central_value(4, 2) == Fraction(2, 3)
    assert _central_value(8, 4) == Fraction(151, 315)
    assert _central_value(12, 6) == Fraction(655177, 1663200)


@pytest.mark.parametrize("m", [2, 3, 4, 5, 6, 8])
def test_norm_const_matches_closed_form(m):
    # sum_k sinc(pi k/m)^(2m) = m B_2m(m) (Poisson summation of the autocorrelation B_m * B_m = B_2m)
    cm = B.norm_const(m)
    assert abs(cm * cm * m * float(_central_value(2 * m, m)) - 1.0) < 1e-14


@pytest.mark.parametrize("m", [1, 2, 3, 4, 6])
def test_unit_norm_and_mean_by_exact_quadrature(m):
    # N_m is a polynomial of degree m-1 on each cell [i/m, (i+1)/m]: m-point Gauss-Legendre per
    # cell integrates N_m^2 exactly
    x, w = _gl_cells(m, m + 1)
    v = B.N(m, x)
    assert abs(np.sum(w * v * v) - 1.0) < 1e-14
    assert abs(np.sum(w * v) - B.norm_const(m)) < 1e-14        # mean = N^_m(0) = C_m


def test_order_two_is_the_normalised_hat():
    x = np.random.default_rng(3).random(1000)
    hat = math.sqrt(3.0) * (1.0 - np.abs(2.0 * x - 1.0))
    assert np.max(np.abs(B.N(2, x) - hat)) < 1e-15
    assert np.all(B.N(1, x) == 1.0)


@pytest.mark.parametrize("m", [2, 3, 4, 6])
def test_closed_form_matches_fourier_series(m):
    # the paper's definition as a partial Fourier series; its tail is bounded by
    # 2 C_m sum_{k>K} (m/(pi k))^m <= 2 C_m (m/pi)^m K^(1-m) / (m-1)
    rng = np.random.default_rng(10 + m)
    x = np.concatenate([rng.random(40), [0.0, 0.5, 1.0 / m, 0.999999]])
    K = 20000
    k = np.arange(-K, K + 1)
    ser = np.exp(2j * np.pi * np.outer(x, k)) @ B.N_hat(m, k)
    bound = 2 * B.norm_const(m) * (m / math.pi) ** m * K ** (1 - m) / (m - 1) + 1e-12
    assert np.max(np.abs(ser - B.N(m, x))) <= bound
    assert np.max(np.abs(ser.imag)) < 1e-12                       # N_m is real and even about 1/2


@pytest.mark.parametrize("m", [2, 3, 4, 6])
def test_fft_of_samples_gives_the_coefficients(m):
    P = 1 << 14
    v = B.N(m, np.arange(P) / P)
    c = np.fft.fft(v) / P
    k = np.arange(-50, 51)
    alias = 2 * B.norm_const(m) * (m / math.pi) ** m * 1.7 * (P - 50.0) ** (-m) + 1e-15
    assert np.max(np.abs(c[k % P] - B.N_hat(m, k))) <= alias
    assert B.N_hat(m, np.array([m, 2 * m, -3 * m])).tolist() == [0.0, 0.0, 0.0]


# ---- tensor-product sums ---------------------------------------------------------------------------

def test_tensor_coefficients_by_fft():
    orders = np.array([[3, 4, 0], [0, 0, 6], [4, 0, 5]])
    f = B.TensorBsplineSum(orders, [1.0, -0.5, 2.0])
    P = 96
    g = np.arange(P) / P
    X = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    F = np.fft.fftn(f.eval_nodes(X).real.reshape(P, P, P)) / P ** 3
    k = np.random.default_rng(4).integers(-7, 8, size=(200, 3))
    k = np.concatenate([k, [[0, 0, 0], [1, 0, 0], [0, 2, 0], [0, 0, 3], [5, 0, 0], [2, 3, 0]]])
    got = F[k[:, 0] % P, k[:, 1] % P, k[:, 2] % P]
    assert np.max(np.abs(got - f.fhat(k))) < 3e-6                  # aliasing of the order-3 factor
    assert np.max(np.abs(got.imag)) < 1e-12


def _quad2(fun, cells=12, pts=8):
    x, w = _gl_cells(cells, pts)
    X = np.stack(np.meshgrid(x, x, indexing="ij"), axis=-1).reshape(-1, 2)
    W = np.outer(w, w).ravel()
    return float(np.sum(W * fun(X)))


def test_norm2_by_exact_quadrature():
    # breakpoints of orders 2, 3, 4, 6 all lie on multiples of 1/12; f^2 has degree <= 10 per
    # variable on each cell, which 8-point Gauss-Legendre integrates exactly
    orders = np.array([[2, 4], [6, 0], [0, 3]])
    f = B.TensorBsplineSum(orders, [1.0, 0.7, -1.3])
    q = _quad2(lambda X: f.eval_nodes(X).real ** 2)
    assert abs(q - f.norm2()) < 1e-12 * q
    p = B.TensorBsplineSum(B.paper_f10_orders())
    assert p.d == 10 and p.T == 3
    assert sorted((p.orders > 0).sum(axis=1).tolist()) == [3, 3, 4]
    assert ((p.orders > 0).sum(axis=0) == 1).all()


def test_rel_l2_error_by_quadrature():
    orders = np.array([[2, 4], [6, 0]])
    f = B.TensorBsplineSum(orders, [1.0, 0.7])
    ks = np.array([(a, b) for a in range(-3, 4) for b in range(-3, 4)])
    rng = np.random.default_rng(7)
    coeffs = f.fhat(ks) + 0.01 * (rng.standard_normal(len(ks)) + 1j * rng.standard_normal(len(ks)))

    def sq_err(X):
        p = np.exp(2j * np.pi * (X @ ks.T.astype(np.float64))) @ coeffs
        return np.abs(f.eval_nodes(X) - p) ** 2

    direct = math.sqrt(_quad2(sq_err, cells=12, pts=16) / _quad2(lambda X: f.eval_nodes(X).real ** 2))
    assert abs(f.rel_l2_error(ks, coeffs) - direct) < 1e-10
    # the best coefficients for a set are f^ itself; the error then is the tail of Parseval's sum
    best = f.rel_l2_error(ks, f.fhat(ks))
    assert abs(best - math.sqrt(1.0 - np.sum(f.fhat(ks) ** 2) / f.norm2())) < 1e-14


# ---- the sparse FFT on a B-spline sum ------------------------------------------------------------

def test_sfft_threshold_variant_on_smooth_sum():
    # smooth factors (orders 4 and 6) alias little, so the threshold decides the support: every
    # frequency of the box with |f^_k| >= 2 delta is found, none below delta / 2, and the
    # coefficients are close to f^
    f = B.TensorBsplineSum(np.array([[4, 4, 0], [0, 0, 6]]))
    delta = 1e-3
    res = S.sfft([-8] * 3, [8] * 3, f, delta, s=10 ** 6, r=3, seed=17, delta_1d=delta / 10)
    box = np.array([(a, b, c) for a in range(-8, 9) for b in range(-8, 9) for c in range(-8, 9)])
    fh = f.fhat(box)
    found = {tuple(k) for k in res.freqs.tolist()}
    must = {tuple(k) for k in box[np.abs(fh) >= 2 * delta].tolist()}
    never = {tuple(k) for k in box[np.abs(fh) < delta / 2].tolist()}
    assert must <= found and not (found & never)
    assert np.max(np.abs(res.coeffs - f.fhat(res.freqs))) < 1e-4
    best = f.rel_l2_error(res.freqs, f.fhat(res.freqs))
    assert f.rel_l2_error(res.freqs, res.coeffs) < 1.05 * best
    assert res.margin > 0.0
