"""FP64 CPU oracle for the data-space Hessian build and inversion.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or links
anything in this package: only the test suite, the smoke check and the CPU
baseline leg of the benchmark use it.  It shares no code, tables or constants
with the HIP library; the only common input is the seeded generator module
``synth`` (velocity models, receivers, frequencies, residuals), which holds none
of the method's arithmetic.

Layout:
  fd.py       medium set-up, the acoustic FD recurrence, Green-function samples,
              the DFT at arbitrary frequencies, forward/adjoint operators S, S^T
  hessian.py  frequency-domain Hessians (Toeplitz-limit form R1, finite-record
              form R2, the literal Fourier-diagonal algorithm) and the explicit
              time-domain Hessian from products of Toeplitz matrices
  solve.py    penalty, Cholesky factorisation, per-frequency multi-source solve
  krylov.py   the iterative baseline: CG on the time-domain system, two PDE
              solves per iteration

Every function cites the passage of the paper it follows.  Pins (tests that
check the oracle against something other than itself) live under tests/ and are
listed per function in each module's docstring.
"""
