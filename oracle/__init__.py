"""FP64 CPU oracle for the approximated-observation CS-SAR method.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import anything from this package; the
product path (the HIP library and its Python binding) never does, and this
package never imports the product path.  The two share no code: the only
common module is the seeded input generator package ``inputs``, which holds
none of the method's arithmetic.

What is computed, and where in the paper it comes from:

* ``dft``     -- the DFT matrices F and F^H of eq. (RDA) in Section III.C,
                 written out as explicit matrices (no FFT), unitary scaling.
* ``csa``     -- the matched-filter focusing chain M and the approximated
                 observation G = M^{-1} (Section III.B, eqs. (focus) and
                 G = M^{-1}), built for the chirp-scaling algorithm named in
                 Section III.D with the inversion rules i)-ii) of Section
                 III.C.  Theorem 1 (G^H = M) holds exactly for this chain.
* ``ita``     -- the complex soft threshold (eq. (L12)), the iteration
                 eq. (th2d) / Algorithm 1 with X^(0) = 0, and the sparsity
                 rule for lambda of Section IV.B.
* ``sim``     -- the exact stripmap echo model of eq. (obf) with exact slant
                 range (Section V.A), periodised on the grid, and the dense
                 exact observation matrix H of eq. (ob2d) for tiny grids.
* ``metrics`` -- PSLR and IRW as defined in Section V.A.2.
* ``grad``    -- the adjoint (reverse-mode) gradient of ||X_K - X_true||^2
                 through K unrolled iterations of eq. (th2d).

Parity pins for every function are in tests/test_oracle_*.py.
"""

from . import dft, csa, ita, sim, metrics  # noqa: F401
