"""FP64 CPU oracle for the IterNCGP hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never calls it, and this package imports nothing from the
product path.

Contents (each function cites the passage of Tatzel et al., "Accelerating
Non-Conjugate Gaussian Processes By Trading Off Computation For Uncertainty",
TMLR 2025, that it follows):

* ``kernels``    -- RBF / Matern kernel functions and dense kernel matrices.
* ``likelihood`` -- softmax likelihood, gradient, Hessian blocks W_n and the
  explicit pseudo-inverse W_n^+ (appendix lemma on the pseudo-inverse);
  Poisson and Gaussian likelihoods.
* ``newton``     -- O-exact: the Newton step as the solve of
  (K + W^+) v = yhat - m with a dense Cholesky (Proposition "Reformulation of
  the Newton Step"); the textbook Newton step for cross-checks.
* ``itergp``     -- O-method: Algorithms 1, 2 and 3 (IterNCGP outer loop,
  IterGP inner loop, virtual solver run with compression).
* ``predict``    -- predictive mean / marginal variance (eqs. for m_{i,j} and
  k_{i,j}) and the probit approximation.

Parity status: every function here is pinned by ``tests/test_oracle_*.py``
against facts the paper or textbook mathematics fix (see the module headers).
"""
from . import kernels, likelihood, newton, itergp, predict  # noqa: F401
