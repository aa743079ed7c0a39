"""FP64 CPU oracle for two-level nonlinear restricted additive Schwarz.

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain reference that the
HIP path is checked against.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the product path never does.
It shares no code with the HIP library: both read the same seeded inputs
from ``synth`` and nothing else.

Layout
  p1.py       P1 finite elements for -div((1+beta u^2) kappa grad u) = f
              (eq. 1), residual F(u) and Jacobian DF(u) (eq. 3).
  nh.py       Q1 finite elements for 2-D compressible Neo-Hooke elasticity
              (eq. 2), two dofs per node, nodal traction loads.
  guess.py    learned initial guess of the local solves: features,
              lifting, training targets, the network, Adam, the judge.
  schwarz.py  overlapping subdomains and transfer operators, local nonlinear
              corrections T_i (eq. 4), RASPEN residual (eqs. 5, 8), GDSW
              and RGDSW coarse spaces, coarse correction T_0 (eq. 9),
              additive and hybrid couplings (eqs. 10, 11), exact tangents
              (eqs. 6, 7, 12), GMRES and the outer
              Newton iteration on the tangent system (eq. 13), and a
              brute-force global Newton solve as the plain definition of the
              end result; load stepping.
  nks.py      the Newton-Krylov-Schwarz comparator: Newton on F(u) = 0 with
              GMRES right-preconditioned by linear two-level Schwarz.

Every function cites the passage of the paper it follows; where the paper is
silent the docstring states the reading taken.  Pins (independent checks of
this code against mathematics) live in tests/test_oracle_*.py.
"""
from .nh import NHProblem  # noqa: F401
from .p1 import P1Problem  # noqa: F401
from .schwarz import Schwarz, gmres_mgs, global_newton  # noqa: F401
from .nks import NKS  # noqa: F401
