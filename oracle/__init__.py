"""FP64 CPU oracle for the randomized low-rank covariance inverse.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import, call or run
anything in this package: only the test-suite, the smoke check and the
benchmark's CPU-baseline leg use it. It shares no code with the HIP library
(no kernels, headers, helpers, tables or pre/post-processing); the two meet only
through the seeded input generators in ``workloads``.

It is written to be read against the paper (Banerjee, Vogelstein, Dunson,
"Parallel inversion of huge covariance matrices"):

* ``kernels``  squared-exponential and Matern covariances (Sec. 5.1, Sec. 4.1).
* ``srht``     the Walsh-Hadamard matrix by the Sylvester recursion and the
               structured random matrix Omega = c R T P (Def. 1, Sec. 3.2).
* ``transforms`` the discrete cosine and Hartley forms of the same
               structured Omega, for any n (Sec. 3.2; Sec. 5, Table 3).
* ``sketch``   Y = (K_f + nu I) Omega (Sec. 3.1-3.2).
* ``qr``       Householder QR and the binary-tree blocked QR, Eq. (1)-(4)
               (Sec. 3.3).
* ``lowrank``  the Woodbury-form approximate inverse applied to A, and the
               log-determinant / Gaussian log-likelihood (Sec. 1, Sec. 3.1
               reading; see the module docstring).
* ``grad``     gradients of the approximate log-likelihood and of the solve
               with respect to (log ell, log s, log sigma2).

Everything is float64 NumPy. Library primitives (matmul, LU, triangular solve,
eigenvalues) are used as single steps only; no blocking or fusion is added
beyond what the definitions state.

Parity pins: every function is pinned by ``tests/test_oracle_*.py`` against
values the paper prints (Tables 1-2), closed forms, library routines and
brute force on small inputs; the module headers list the pins.
"""
from . import kernels, srht, transforms, sketch, qr, lowrank, grad  # noqa: F401
