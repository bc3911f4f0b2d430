"""CPU oracle for the tetrahedral-stencil FFT homogenization solver (Finel, arXiv 2405.11168).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the tests, the smoke check and the benchmark's
CPU-baseline leg use it.  It shares no code with the HIP library; the one
thing both sides use is the seeded input module ``hz_synth``.

Everything here is plain, slow FP64 numpy written to be checked against the
paper by eye:

* ``tetra``    -- Algorithm 1 (displacement-based basic scheme, Sec. 2.6) in
                  the paper's own Fourier form: D(q) of eq. Dq, the Green
                  operator of eq. Green_tensor, the update of eq.
                  basic_scheme_dep_2 and the criterion of eqs. L2-norm and
                  tolerance; also the strain-based Algorithm 2 and the strain
                  Green operators G^d, G^nd and Gamma of Sec. 2.6.
* ``stencil``  -- the real-space tetrahedral finite-difference operators of
                  eqs. DA1-DA2 and the corner force density of eq. L2-norm.
* ``dense``    -- the plain definition: direct minimisation of the collapsed
                  energy of eq. Elast_energy on tiny grids.
* ``laminate`` -- closed-form effective response of an axis-aligned laminate.
* ``comparison`` -- the comparison discretisations of Sec. 3.2 and Appendix B
                  (Willot's rotated scheme, eq. Dq_rotated, and the
                  continuous-frequency operator of Moulinec-Suquet) as
                  displacement-based basic schemes with one strain field.
* ``voigt``    -- Voigt <-> tensor bookkeeping.

Pins (see tests/test_oracle_*.py) tie each part to something other than
itself: naive DFT sums, the closed form of |D|^2, the real-space stencils,
the dense minimiser, the laminate closed form, Voigt/Reuss bounds and
symmetries.  Iteration *counts* versus contrast are parity unpinned: the
paper prints them only as a figure.
"""
