"""Plain FP64 CPU oracle for the constrained-realization solve.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or
execute this package: only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it. It shares no code with the HIP
library (no kernels, headers, tables or helpers) and it imports nothing from
the product package.

What it computes (Eskilt et al. 2023, arXiv:2306.15511, Sect. 2.2.1 and
App. A):

* ``healpix``  - RING geometry of HEALPix (Gorski et al. 2005).
* ``legendre`` - normalised associated Legendre functions lambda_lm(z) =
  Delta_lm P_lm(z) (App. A definition of P~_lm), by the textbook three-term
  recurrence carried out in extended-exponent arithmetic so nothing underflows.
* ``sht``      - synthesis Y, its exact transpose Y^T (no quadrature weight),
  ring-factored: Legendre sums by BLAS per m, azimuthal sums by numpy FFT.
* ``dense``    - the same Y built as an explicit matrix from SciPy's
  ``sph_harm_y`` (an independent implementation), and the dense Cholesky
  solve of the constrained-realization system.
* ``cr``       - the operator A = S^-1 + B Y^T N^-1 Y B, its right-hand side,
  the Jacobi diagonal and preconditioned conjugate gradients; the
  harmonic-diagonal model and its closed forms.
* ``joint``    - the joint (C_l amplitude, sky) Metropolis move and ln pi.
* ``grad``     - gradients of chi^2 with respect to a_lm and of ln pi with
  respect to binned C_l (adjoint CG).
* ``spin2``    - spin-2 functions W, X (+-2Y = (W +- X) e^{i m phi}) and the
  polarised synthesis (a_E, a_B) -> (Q, U) with its transpose.
* ``cr_tqu``   - the T+Q+U constrained-realization operator with 3x3 spectra
  blocks and per-component N^-1.

All arithmetic is float64 / complex128.
"""
