"""FP64 CPU oracle for the implicit-complementarity interior-point method.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
link anything in this package; only the test-suite, the smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the HIP path:
the only common module is ``qpgen`` (seeded problem generators, which hold
none of the method's arithmetic).

Everything here is plain, dense and slow on purpose: one QP at a time, NumPy
arrays in float64 (a ``dtype`` argument exists only to time the same code in
float32 as the plain per-QP baseline), dense LU (``numpy.linalg.solve``) for
every linear system.  Each function names the passage of the paper it
follows.

Modules
-------
retraction   softplus retraction b_kappa and its derivatives (section 4.1, appendix C)
kkt          KKT residuals and the Newton matrices (section 2.1, 2.2, 4.2, appendix B)
implicit     Algorithm 1 (solve) and Algorithm 2 (relax) with Newton steps from
             the uncondensed implicit system
standard     the standard Mehrotra predictor-corrector IPM (ablation arm) and its
             central-path relaxation
gradients    implicit-function-theorem vector-Jacobian product (appendix A,
             Algorithm 3's parameter formulas) and central finite differences
reference    closed forms and brute force: unconstrained and equality-only QPs,
             box QPs, active-set enumeration, the hard-projection Jacobian
             (appendix D)

Pins: every function is checked in ``tests/test_oracle_*.py`` against values
fixed by the mathematics (closed forms, brute force, identities, finite
differences), not against itself.  Parity unpinned: iteration counts (the
paper reports none) and the default centering factor sigma (the paper gives
none).
"""
from . import retraction, kkt, implicit, standard, gradients, reference  # noqa: F401
