"""FP64 CPU oracle for Fourier-basis kernel ridge regression.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the CPU
baseline leg of the benchmark may import this package.  The product path (the
HIP library and its Python binding) never calls it and shares no code with it.

Everything here is the plain definition of what the fast method computes,
evaluated slowly in float64 on the CPU:

* ``fourier``  - the Gram generator M[q] = n^-1 sum_j exp(+i q.X_j) and the
  right-hand side b_k = n^-1 sum_j Y_j exp(-i k.X_j) as direct sums (Sec. 2.3,
  "Covariance vector" and "Covariance matrix"), plus the additive-model block
  Gram (Sec. 5, "Complexity").
* ``penalty``  - the Sobolev weights (Sec. 3.1), the low-bias identity (Sec. 3.2),
  the physics-informed penalty lambda S^2 + mu D^* C D on a box for any linear
  constant-coefficient operator (Sec. 4, "Tractable domains"), its collocation form (Sec. 4, intractable domains) and the
  additive block penalty (Sec. 5).
* ``solve``    - the normal equations of eq. (kenrel_reg) solved by an FP64
  LAPACK Cholesky (zpotrf/zpotrs through scipy).
* ``cg``       - the product Sigma x by its dense definition and the textbook
  Jacobi-preconditioned conjugate-gradient iteration (Sec. 2.3, "Matrix inversion").
* ``predict``  - f_theta(x) = sum_k theta_k exp(+i k.x) by direct sum (Sec. 2.1).
* ``krr``      - kernel ridge regression in its n x n kernel form (Sec. 2.1), an
  independent route to theta for small n.
* ``grad``     - held-out MSE and its gradients with respect to log lambda, the
  penalty weights and theta.

Conventions (the readings of the paper taken here):
* points are in torus radians: x = pi X_raw / (2L), so the basis is exp(i k.x);
* M[q] uses the + sign and the system is A[k, l] = M[l - k] + lambda P[k, l];
* b uses the - sign (the sign that the paper's own design matrix implies);
* mode arrays are row-major over (k_1, ..., k_d), each running -m..m, k_d fastest;
  the generator M runs over -2m..2m in each coordinate.

Parity status: every function here is pinned by the tests in
``tests/test_oracle_*.py`` against closed forms, a different library routine,
brute force or a high-precision sum; none is "parity unpinned".
"""
from .fourier import (modes, gram_generator, rhs, fourier_entry, fourier_entries, toeplitz_matrix, design_matrix,
                      additive_blocks, additive_rhs)
from .penalty import (sobolev_weights, sobolev_bessel_weights, piml_box_fourier_matrix,
                      heat_symbol, piml_heat_penalty, pde_symbol, piml_box_penalty, additive_penalty,
                      collocation_penalty)
from .solve import system_matrix, solve_system, condition_number, fit
from .cg import toeplitz_apply, toeplitz_apply_rows, pcg
from .predict import predict, predict_additive
from .krr import krr_theta
from .grad import heldout_mse, heldout_mse_quadratic, mse_gradients, theta_path_gradients

__all__ = [
    "modes", "gram_generator", "rhs", "fourier_entry", "fourier_entries", "toeplitz_matrix", "design_matrix",
    "additive_blocks", "additive_rhs",
    "sobolev_weights", "sobolev_bessel_weights", "piml_box_fourier_matrix", "heat_symbol",
    "piml_heat_penalty", "pde_symbol", "piml_box_penalty", "additive_penalty", "collocation_penalty",
    "system_matrix", "solve_system", "condition_number", "fit", "toeplitz_apply", "toeplitz_apply_rows", "pcg",
    "predict", "predict_additive", "krr_theta",
    "heldout_mse", "heldout_mse_quadratic", "mse_gradients", "theta_path_gradients",
]
