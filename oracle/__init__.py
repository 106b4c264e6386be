"""CPU oracle for the multiple rank-1 lattice FFT and the dimension-incremental sparse FFT.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg
of ``bench.py`` may import this package.  The product path (the HIP library and its Python
binding) never imports, calls or links anything from here, and this package imports nothing
from the product.  The only code the two sides share is the input generator package
``workloads`` (which holds none of the method's arithmetic).

Plain, slow, obviously correct implementations in IEEE double precision, each function citing
the passage of Kaemmerer, Potts, Volkmer, "High-dimensional sparse FFT based on sampling along
multiple rank-1 lattices" (arXiv 1711.05152) that it follows:

* ``rng``       counter-based SplitMix64 streams for the method's random draws (generating
                vectors, anchors) and for sample noise.
* ``mr1l``      residues, alias histograms, unaliased sets I_l and counters, the inverse
                multiple rank-1 lattice FFT (Alg. 2) in a brute-force tier and an FFT tier, its
                adjoint, and the Fourier matrix A(X, I) of Sec. 2.1 with its adjoint.
* ``construct`` the randomized construction of reconstructing multiple rank-1 lattices with
                distinct prime sizes (Alg. 1) and the parameter rules around it.
* ``sfft``      the dimension-incremental sparse FFT (Alg. 3 "MLFFT") with the planted
                polynomial black box, 1-D projections, thresholding and top-s selection.
* ``bspline``   the periodic B-splines N_m and the tensor-product test function of Sec. 5.3
                (point values, Fourier coefficients, norm, relative L2 approximation error),
                usable as a black box of ``sfft``.
"""
