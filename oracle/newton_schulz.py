"""Plain dense Newton-Schulz sign iteration in float64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper computes the sign function (Eq. 13) iteratively but does not name
the iteration; the one used on the hot path is the
Newton-Schulz map X <- 1/2 X (3I - X^2), which converges to sign(X_0) for every
symmetric X_0 whose eigenvalues are non-zero with |lambda| < sqrt(3).  This
module states the iteration and its stopping rule exactly as the GPU path runs
them, so iteration counts can be compared:

    X_0 = T / c        (c >= spectral radius, e.g. the Gershgorin bound)
    repeat:  A = X_k^2;  r_k = ||A - I||_F;  stop if r_k < tol
             X_{k+1} = 1/2 X_k (3I - A)
    the number of iterations is the number of updates applied.
"""
from __future__ import annotations

import numpy as np

__all__ = ["ns_sign", "ns_scalar_iterations", "ns_map"]


def ns_map(x):
    """Scalar Newton-Schulz map g(x) = x (3 - x^2) / 2."""
    return 0.5 * x * (3.0 - x * x)


def ns_sign(T: np.ndarray, c: float, tol: float = 1e-10, max_iter: int = 100):
    """Dense float64 Newton-Schulz on T / c.  Returns (X, iterations, residual
    history)."""
    n = T.shape[0]
    X = T / c
    I = np.eye(n)
    hist = []
    for k in range(max_iter + 1):
        A = X @ X
        r = float(np.linalg.norm(A - I))
        hist.append(r)
        if r < tol or k == max_iter:
            return X, k, hist
        X = 0.5 * (X @ (3.0 * I - A))
    return X, max_iter, hist


def ns_scalar_iterations(d: np.ndarray, c: float, tol: float = 1e-10, max_iter: int = 100):
    """For a diagonal T = diag(d) every iterate stays diagonal and the matrix
    iteration is the scalar map applied entrywise; the residual is
    sqrt(sum_p (x_p^2 - 1)^2).  Returns the iteration count."""
    x = np.asarray(d, dtype=np.float64) / c
    for k in range(max_iter + 1):
        r = float(np.sqrt(np.sum((x * x - 1.0) ** 2)))
        if r < tol or k == max_iter:
            return k
        x = ns_map(x)
    return max_iter
