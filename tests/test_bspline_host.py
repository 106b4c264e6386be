"""Host-only entry points of the B-spline test function (Fourier coefficients, norm, relative L2
error of Sec. 5.3) against the oracle.  They launch no kernel, so they run without a GPU."""
import numpy as np

from oracle import bspline as OB


def test_host_coefficients_and_error_match_oracle():
    from paper_1711_05152_amd.sfft import BsplineSum, paper_f10
    f, of = paper_f10(), OB.TensorBsplineSum(OB.paper_f10_orders())
    rng = np.random.default_rng(5)
    k = rng.integers(-40, 41, size=(3000, 10))
    k[::2, 3:] = 0
    k = np.unique(k, axis=0)
    assert np.abs(f.coeffs(k) - of.fhat(k)).max() <= 1e-15
    c = of.fhat(k) + 1e-4 * (rng.standard_normal(len(k)) + 1j * rng.standard_normal(len(k)))
    e, n2 = f.rel_l2_error(k, c)
    assert abs(e - of.rel_l2_error(k, c)) <= 1e-12 and abs(n2 - of.norm2()) <= 1e-13
    g, og = BsplineSum([[2, 4], [6, 0], [0, 3]], [1.0, 0.7, -1.3]), OB.TensorBsplineSum([[2, 4], [6, 0], [0, 3]],
                                                                                        [1.0, 0.7, -1.3])
    assert abs(g.rel_l2_error(np.zeros((0, 2), np.int32), [])[1] - og.norm2()) <= 1e-13
