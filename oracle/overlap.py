"""FP64 submatrix method with a non-orthogonal basis (S != I), from the paper.

TEST INFRASTRUCTURE ONLY (see the package docstring): never imported by the
product path.

Paper passages followed (arXiv 2205.14741):

* Eq. 12 -- the sign of the 2 x 2 block matrix [[0, A], [I, 0]] has the
  off-diagonal blocks A^(1/2) and A^(-1/2); this is how the inverse square
  root of an overlap matrix is obtained from a sign evaluation.  Here the
  sign is taken by its definition (Eq. 13): M (M^2)^(-1/2), where
  M^2 = diag(A, A), with (A)^(-1/2) from the eigendecomposition of A.
* Eq. 13 -- sign(A) = A (A^2)^(-1/2).
* Eq. 14 -- P = 1/2 (I - sign(S^-1 H - mu I)) S^-1.  For symmetric H and
  symmetric positive definite S, S^-1 H is similar to
  K = S^(-1/2) H S^(-1/2), and P = 1/2 S^(-1/2) (I - sign(K - mu I)) S^(-1/2)
  = sum over the eigenpairs H c = lam S c (c^T S c = 1) with lam < mu of
  c c^T, with weight 1/2 for lam = mu (sign(0) := 0).  That last form, by
  the generalized symmetric eigendecomposition, is the plain definition used
  here.
* Fig. 2 -- the submatrix method: one dense principal submatrix per atom
  block, over the index set of that block column; the matrix function of
  the submatrix pair (T_i(H), T_i(S)) is Eq. 14 applied to the pair, and only
  block i's columns are kept.  The electron count in a non-orthogonal basis
  is tr(P S) (P = C C^T with C^T S C = I, so tr(P S) counts the occupied
  states).

The index sets come from H's pattern; S must be stored on the same pattern
(the synthetic overlaps are generated that way).
"""
from __future__ import annotations

import math

import numpy as np
import scipy.linalg

from .submatrix import BlockView, submatrix, submatrix_indices

__all__ = ["inv_sqrt_eigh", "sqrt_eigh", "block_sign_eq12", "overlap_submatrix",
           "density_matrix_columns_overlap", "density_matrix_overlap", "traces_overlap",
           "full_P_overlap"]


def inv_sqrt_eigh(A: np.ndarray) -> np.ndarray:
    """A^(-1/2) of a symmetric positive definite A: V diag(lam^(-1/2)) V^T."""
    lam, V = np.linalg.eigh(A)
    if lam[0] <= 0:
        raise ValueError("matrix is not positive definite")
    return (V / np.sqrt(lam)) @ V.T


def sqrt_eigh(A: np.ndarray) -> np.ndarray:
    """A^(1/2) of a symmetric positive definite A."""
    lam, V = np.linalg.eigh(A)
    if lam[0] <= 0:
        raise ValueError("matrix is not positive definite")
    return (V * np.sqrt(lam)) @ V.T


def block_sign_eq12(A: np.ndarray) -> np.ndarray:
    """sign([[0, A], [I, 0]]) by the definition of Eq. 13, M (M^2)^(-1/2):
    M^2 = diag(A, A), so (M^2)^(-1/2) = diag(A^(-1/2), A^(-1/2)) and the
    result is [[0, A A^(-1/2)], [A^(-1/2), 0]] (Eq. 12's right-hand side)."""
    n = A.shape[0]
    M = np.zeros((2 * n, 2 * n))
    M[:n, n:] = A
    M[n:, :n] = np.eye(n)
    Ri = inv_sqrt_eigh(A)
    R = np.zeros_like(M)
    R[:n, :n] = Ri
    R[n:, n:] = Ri
    return M @ R


def overlap_submatrix(view_s: BlockView, i: int) -> np.ndarray:
    """T_i(S) = S[idx_i, idx_i] (no shift)."""
    return submatrix(view_s, i, 0.0)


def density_matrix_columns_overlap(view_h: BlockView, view_s: BlockView, i: int, mu: float):
    """Eq. 14 on the submatrix pair of atom i: the b_i columns of
    P_i = sum_{lam < mu} c c^T (+ 1/2 for lam == mu) with H_i c = lam S_i c,
    c^T S_i c = 1, over the rows idx_i.  Returns (atoms, columns)."""
    atoms, idx, loc = submatrix_indices(view_h, i)
    Hi = submatrix(view_h, i, 0.0)
    Si = overlap_submatrix(view_s, i)
    lam, C = scipy.linalg.eigh(Hi, Si)
    w = np.where(lam < mu, 1.0, np.where(lam == mu, 0.5, 0.0))
    b = int(view_h.bs[i])
    cols = (C * w) @ C[loc:loc + b, :].T
    return atoms, cols


def density_matrix_overlap(mh, ms, mu: float, atoms=None) -> np.ndarray:
    """P (S != I) in H's block-column panel layout; block column i from
    submatrix i only (not symmetrised).  ``atoms``: only those block columns
    (others NaN)."""
    vh = mh if isinstance(mh, BlockView) else BlockView(mh)
    vs = ms if isinstance(ms, BlockView) else BlockView(ms)
    P = np.full_like(vh.vals, np.nan)
    todo = range(vh.n_atoms) if atoms is None else atoms
    for i in todo:
        rows, cols = density_matrix_columns_overlap(vh, vs, int(i), mu)
        off = 0
        for r in rows:
            br = int(vh.bs[r])
            P[vh.panel_slot(r, int(i))] = cols[off:off + br, :]
            off += br
    return P


def traces_overlap(mh, ms, P: np.ndarray):
    """E = tr(P H) and Ne = tr(P S): sums over the stored entries of P .* H
    and P .* S (H, S symmetric, stored on the same pattern), compensated
    (math.fsum) per block column, then over the columns."""
    vh = mh if isinstance(mh, BlockView) else BlockView(mh)
    vs = ms if isinstance(ms, BlockView) else BlockView(ms)
    e_cols, n_cols = [], []
    for c in range(vh.n_atoms):
        a, b = int(vh.panel_off[c]), int(vh.panel_off[c + 1])
        e_cols.append(math.fsum((P[a:b] * vh.vals[a:b]).tolist()))
        n_cols.append(math.fsum((P[a:b] * vs.vals[a:b]).tolist()))
    return math.fsum(e_cols), math.fsum(n_cols)


def full_P_overlap(H: np.ndarray, S: np.ndarray, n_occ: int) -> np.ndarray:
    """Exact density matrix of the whole pencil: the n_occ lowest generalized
    eigenvectors (c^T S c = 1), P = C_occ C_occ^T."""
    lam, C = scipy.linalg.eigh(H, S)
    Co = C[:, :n_occ]
    return Co @ Co.T
