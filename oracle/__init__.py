"""FP64 CPU oracle for image-space gridding and nonrigid SENSE.

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only the test-suite, the smoke check
and the benchmark's CPU-baseline leg may import or run anything in this
package.  The HIP library never calls it and shares no code with it: no
kernels, no tables, no helpers.  The only thing both sides take from a common
place is the seeded input generator in ``synth`` (which holds none of the
method's arithmetic).

Each function restates one passage of the paper (Jang, Malave, Nishimura,
"Image-Space Gridding for Nonrigid Motion-Corrected MR Image Reconstruction",
arXiv:2501.16713) in plain NumPy/SciPy FP64 code, with no blocking, fusion or
reordering beyond what the equation states:

* ``kernel``  - the interpolation kernel c(x) and its transform C(k)
                (notation table; deapodization, section "k-space Gridding").
* ``grid``    - the Projection Core P (spread) and the Backprojection Core B
                (gather) on a periodic oversampled grid (Eq. 1, 3; Fig. 1).
* ``warp``    - image-space gridding: forward T (Eq. 9) and adjoint T^H
                (Eq. 7-8), the displacement-field warp they approximate
                (Eq. 5), and the derivative of T x with respect to d.
* ``kspace``  - inverse k-space gridding G (Eq. 3), k-space gridding G^H
                (Eq. 1-2), and the direct NDFT that G approximates.
* ``sense``   - nonrigid SENSE A_p = G_p S T_p, its adjoint, the stacked
                model (Eq. 10) and the l2 normal operator of Eq. 11.
* ``cg``      - conjugate gradients on the l2 form of Eq. 11.
* ``dense``   - brute-force dense matrices of T and G from explicit sums
                (no FFT), used only to pin the FFT-based functions.
* ``wavelet`` - the orthonormal multi-level Haar transform W of the
                l1 terms of Eq. 11 and Eq. 13.
* ``fista``   - wavelet-FISTA for Eq. 11 / Eq. 13 and the power iteration
                for its step size.
* ``inversion`` - Appendix 1: naive and iterative inversion of T (Eq. 12-13).
* ``register``  - gradient-descent registration with T_d as the warp (the
                gradient-based alternative to the demons step).
* ``gridrecon`` - bulk-translation linear phase, Pipe-Menon density
                compensation and direct gridding reconstruction (section
                "Motion Capturing for Segmented Data Acquisitions").

Every function is pinned in ``tests/test_oracle_*.py`` against something
other than itself: adjoint identities, brute-force sums, exact special cases
(integer shifts), textbook routines (Fourier shift, NDFT), closed forms and
finite differences.  The one function without such a pin is listed in its
module header as "parity unpinned".
"""
from . import kernel, grid, warp, kspace, sense, cg, dense  # noqa: F401
from . import wavelet, fista, inversion, register, gridrecon  # noqa: F401
