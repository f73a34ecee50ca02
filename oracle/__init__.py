"""FP64 CPU oracle for the TripoSH bispectrum-multipole estimator.

TEST INFRASTRUCTURE ONLY. This package is the plain, slow reference that the
HIP path is checked against. Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import it. The product path
(``paper_1803_02132_amd``) never imports, calls or links anything here, and this
package never imports the product path.

Everything follows Sugiyama, Saito, Beutler & Seo (2019), "A complete FFT-based
decomposition formalism for the redshift-space bispectrum" (arXiv:1803.02132):

* ``angular``   -- Wigner 3j symbols, normalised harmonics y_l^m, Legendre
                   polynomials, selection rules (Sec. 2, Table 1, App. A).
* ``estimator`` -- weights, y-weighted density fields, mass assignment, FFTs,
                   shell filters, the 3j-weighted triple-product reduction and
                   the normalisation (Sec. 4.1, 4.2, 4.4, 5.2), plus the direct
                   triangle sum that the FFT form rewrites (Sec. 4.2, eq. 35).
* ``shotnoise`` -- the shot noise of the estimator: the coincident-index terms
                   of its particle description (Sec. 4.2, eqs. 43-46).
* ``threepoint`` -- the three-point-function multipoles (Sec. 4.3, eqs. 47-48)
                   and the window multipoles of the randoms (Sec. 6.1, eq. 58).
* ``masked``    -- the masked model (Sec. 6.2): the 9j coupling of window and
                   model multipoles (eq. 63, App. A), the integral constraint
                   (eq. 64) and the Hankel transform to the bispectrum (eq. 68).

Every function states the passage it follows. Readings of passages that are
silent or ambiguous are listed in each module's header (R1..R12, S1..S5,
T1..T4, M1..M4).

Parity status per function is stated in each module header; every function is
pinned by a ``-m "not gpu"`` test against closed forms, library routines,
brute force or values printed in the paper; the conventions listed there are
pinned by exact properties they imply.
"""
