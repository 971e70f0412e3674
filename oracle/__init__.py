"""Plain FP64 CPU oracle for the major-cycle measurement operator of
"A Decentralized Framework for Radio-Interferometric Image Reconstruction"
(Wang, Mignot, Prunet, Di Mascolo, Spinelli, Ferrari; arXiv 2507.22128).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import anything from here.  The
HIP library never calls, links or imports this package, and this package
imports nothing from the HIP library: the two implementations share no code.

Everything is NumPy / SciPy in float64 / complex128, written for a reader who
checks it against the paper by eye:

* ``geometry``   - the coordinate chain (wavelengths, grid cells, Fourier pixels)
* ``es_kernel``  - exponential-of-semicircle kernel and its gridding correction
* ``dft``        - the direct Fourier sum of Eq. 1 with the w and D terms
                   dropped (Section 2): the plain definition of the operator
* ``gridding``   - the kernel-based gridded operator (same algorithm as the
                   GPU, in FP64) and its exact adjoint
* ``imaging``    - weighting, spatial-frequency partition (Fig. 3), dirty and
                   residual images (Eq. 2), PSF
* ``decentral``  - filters Gamma, PSF convolution H, pseudo-full-resolution
                   composition (Eq. 7), aggregate rho (Eq. 5), combination
* ``msclean``    - multi-scale CLEAN minor cycle (Eq. 6)
* ``wavelets``   - orthonormal Daubechies filters and periodized transforms
* ``fista``      - FISTA for the wavelet-l1 problems of Eqs. 4 and 5
* ``pool``       - runs ``gridding``'s degrid / grid unchanged over chunks
                   of large visibility sets on several host processes

Parity status of each function is stated in its docstring; items whose
definition is a reading of a silent or ambiguous passage say so.
"""

from . import geometry, es_kernel, dft, gridding, imaging, decentral, msclean, wavelets, fista, pool  # noqa: F401,E501
