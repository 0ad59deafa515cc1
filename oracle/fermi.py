"""FP64 submatrix method with a finite-temperature occupation function.

TEST INFRASTRUCTURE ONLY (see the package docstring): never imported by the
product path.

Paper passages followed (arXiv 2205.14741):

* Fig. 2 -- the submatrix method evaluates a general matrix function f on
  every dense principal submatrix T_i and keeps block i's columns of
  f(T_i).  The function used here is the Fermi-Dirac occupation
  f(x) = 1 / (1 + exp(beta x)) at inverse temperature beta, applied to
  T_i = H[idx_i, idx_i] - mu I.  It is the finite-temperature counterpart of
  the step function of Eq. 14: for every x != 0, f(x) tends to
  1/2 (1 - sign(x)) as beta grows.  The paper does not name this f; choosing
  it is a reading of the general f of Fig. 2.
* Section 2 -- mu is set by the electron count.  With a smooth f the count
  Ne(mu) = sum_i sum_{q in block i} f(T_i)_qq is continuous and strictly
  increasing in mu, so a unique mu meets any count in (0, N); it is found
  here by plain bisection (``find_mu_fd``).  Its derivative follows from
  f'(x) = -beta f(x) (1 - f(x)): dNe/dmu = beta sum_i sum_{q in block i}
  [f(T_i) (I - f(T_i))]_qq.

Every f(T_i) is taken by its definition, V diag(f(lam)) V^T from
``numpy.linalg.eigh``; f(x) is evaluated as ``scipy.special.expit(-beta x)``,
which does not overflow for large |beta x|.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.special

from .submatrix import BlockView, global_gershgorin_bracket, submatrix, submatrix_indices

__all__ = ["fermi", "fermi_eigh", "density_matrix_columns_fd", "density_matrix_fd",
           "FermiCache", "find_mu_fd"]


def fermi(x, beta: float):
    """Fermi-Dirac occupation 1 / (1 + exp(beta x)), elementwise."""
    return scipy.special.expit(-beta * np.asarray(x, dtype=np.float64))


def fermi_eigh(T: np.ndarray, beta: float) -> np.ndarray:
    """f(T) = V diag(f(lam)) V^T for symmetric T (Fig. 2's matrix function)."""
    lam, V = np.linalg.eigh(T)
    return (V * fermi(lam, beta)) @ V.T


def density_matrix_columns_fd(view: BlockView, i: int, mu: float, beta: float):
    """Steps 2 and 3 (Fig. 2) for atom i with f = Fermi-Dirac: the b_i columns
    of f(T_i)[:, loc_i : loc_i + b_i] over the rows idx_i.
    Returns (atoms, columns) with columns of shape (n_i, b_i)."""
    atoms, _, loc = submatrix_indices(view, i)
    F = fermi_eigh(submatrix(view, i, mu), beta)
    b = int(view.bs[i])
    return atoms, F[:, loc:loc + b].copy()


def density_matrix_fd(m, mu: float, beta: float, atoms=None) -> np.ndarray:
    """P in the block-column panel layout of H, block column i from
    submatrix i only (not symmetrised).  With ``atoms`` given, only those
    block columns are filled (the others stay NaN)."""
    view = m if isinstance(m, BlockView) else BlockView(m)
    P = np.full_like(view.vals, np.nan)
    todo = range(view.n_atoms) if atoms is None else atoms
    for i in todo:
        rows, cols = density_matrix_columns_fd(view, int(i), mu, beta)
        off = 0
        for r in rows:
            br = int(view.bs[r])
            P[view.panel_slot(r, int(i))] = cols[off:off + br, :]
            off += br
    return P


class FermiCache:
    """Eigendecomposition of every unshifted submatrix, so that the electron
    count and its derivative can be taken at any mu and beta:
    Ne(mu) = sum_i sum_k f(lam_ik - mu) w_ik with w_ik the weight of
    eigenvector k on atom i's own orbitals, and
    dNe/dmu = beta sum_i sum_k f (1 - f) w_ik (f' = -beta f (1 - f))."""

    def __init__(self, m, atoms=None):
        self.view = m if isinstance(m, BlockView) else BlockView(m)
        todo = range(self.view.n_atoms) if atoms is None else atoms
        lam, wts = [], []
        for i in todo:
            _, _, loc = submatrix_indices(self.view, int(i))
            w, V = np.linalg.eigh(submatrix(self.view, int(i), 0.0))
            b = int(self.view.bs[i])
            lam.append(w)
            wts.append(np.sum(V[loc:loc + b, :] ** 2, axis=0))
        self.lam = np.concatenate(lam)
        self.wts = np.concatenate(wts)

    def ne(self, mu: float, beta: float) -> float:
        return math.fsum((self.wts * fermi(self.lam - mu, beta)).tolist())

    def dne(self, mu: float, beta: float) -> float:
        f = fermi(self.lam - mu, beta)
        return beta * math.fsum((self.wts * f * (1.0 - f)).tolist())


def find_mu_fd(m, n_target: float, beta: float, tol: float = 1e-8, max_steps: int = 200,
               cache: FermiCache | None = None):
    """The mu with Ne(mu) = n_target, by bisection inside the global
    Gershgorin bracket (widened by 40 / beta on each side, where the
    occupations are within e^-40 of 0 and 1), until |Ne - n_target| <= tol or
    the bracket stops shrinking.  Returns (mu, steps, Ne)."""
    cache = cache or FermiCache(m)
    lo, hi = global_gershgorin_bracket(m)
    lo -= 40.0 / beta
    hi += 40.0 / beta
    mid, ne = 0.5 * (lo + hi), float("nan")
    for step in range(1, max_steps + 1):
        mid = 0.5 * (lo + hi)
        ne = cache.ne(mid, beta)
        if abs(ne - n_target) <= tol or not (lo < mid < hi):
            return mid, step, ne
        if ne < n_target:
            lo = mid
        else:
            hi = mid
    return mid, max_steps, ne
