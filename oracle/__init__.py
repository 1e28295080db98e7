"""FP64 CPU oracle for Chebyshev-filtered subspace iteration (Levitt & Torrent, arXiv:1406.4350).

TEST INFRASTRUCTURE ONLY. Nothing in the product path imports, links or runs this package: only the
tests, ``__graft_entry__.smoke()`` and the cpu_baseline leg of ``bench.py`` do.

It computes, slowly and plainly, what the GPU path computes:

* ``dense``   -- explicit H and S on tiny grids (naive separable DFT, no FFT library), their dense
                 generalized eigendecomposition, and the Chebyshev filter written through it.
* ``matfree`` -- matrix-free operators (Alg. 1 with numpy FFTs), the Woodbury inverse of S (Sec. 5.1),
                 the filter of Alg. 2 (Sec. 4.2), Rayleigh-Ritz, the Lanczos upper bound and the outer
                 loop (Sec. 5.3).
* ``grad``    -- the adjoint of filter + Rayleigh-Ritz (an addition beyond the paper).

Every function cites the passage it follows. Shared with the GPU path: only the seeded input
generator, which holds none of this arithmetic.
"""
