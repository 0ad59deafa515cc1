"""FP64 submatrix method for P = 1/2 (I - sign(H - mu I)), written from the paper.

TEST INFRASTRUCTURE ONLY (see the package docstring): never imported by the
product path.

Paper passages followed (arXiv 2205.14741):

* Eq. 13 -- the matrix sign function, sign(A) = A (A^2)^(-1/2).  For symmetric
  A = V diag(lam) V^T this is V diag(sign(lam)) V^T, which is how it is
  evaluated here (``numpy.linalg.eigh``), with sign(0) := 0.
* Eq. 14 -- purification P = 1/2 (I - sign(S^-1 H - mu I)) S^-1; every
  workload has an orthogonal basis (S = I), so P = 1/2 (I - sign(H - mu I)).
* Fig. 2 -- the submatrix method.  Each column of the sparse matrix gets a
  small dense matrix: the principal submatrix T_i over every index that the
  column couples to.  The matrix function is evaluated on that dense T_i, and
  only the columns of the result that belong to column i are copied back into
  the sparse output.  Here the unit is an atom block, not a single column:
  the columns of one atom share one index set.
* Section 2 (linear-scaling methods) -- the chemical potential mu separates
  occupied from unoccupied states; the paper gives no rule for finding it, so
  bisection on the electron count tr P is used (see ``find_mu``).

Input layout: a ``synth.BlockSparse``-like object (block sizes, CSC block
pattern with sorted rows and the diagonal present, block-column panels).  Only
its arrays are read.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "BlockView", "index_set", "submatrix_indices", "submatrix", "sign_eigh",
    "gershgorin_bound", "density_matrix", "density_matrix_columns",
    "energy_trace", "SpectralCache", "find_mu", "global_gershgorin_bracket",
    "full_P",
]


class BlockView:
    """Read-only block accessor over the block-column panel layout."""

    def __init__(self, m):
        self.bs = np.asarray(m.block_size, dtype=np.int64)
        self.col_ptr = np.asarray(m.col_ptr, dtype=np.int64)
        self.row_idx = np.asarray(m.row_idx, dtype=np.int64)
        self.panel_off = np.asarray(m.panel_off, dtype=np.int64)
        self.vals = np.asarray(m.vals, dtype=np.float64)
        self.n_atoms = self.bs.shape[0]
        self.orb_off = np.concatenate([[0], np.cumsum(self.bs)])
        # position of every stored block (r, c): (panel start, row offset, height)
        self._where = {}
        for c in range(self.n_atoms):
            rows = self.row_idx[self.col_ptr[c]:self.col_ptr[c + 1]]
            h = int(self.bs[rows].sum())
            ro = 0
            for r in rows:
                self._where[(int(r), c)] = (int(self.panel_off[c]), ro, h)
                ro += int(self.bs[r])

    def rows_of(self, c: int) -> np.ndarray:
        return self.row_idx[self.col_ptr[c]:self.col_ptr[c + 1]]

    def block(self, r: int, c: int):
        """Block H_rc (b_r x b_c) or None when it is not stored."""
        w = self._where.get((int(r), int(c)))
        if w is None:
            return None
        start, ro, h = w
        bc = int(self.bs[c])
        panel = self.vals[start:start + h * bc].reshape(bc, h).T
        return panel[ro:ro + int(self.bs[r]), :]

    def panel_slot(self, r: int, c: int):
        """(flat indices into vals of block (r, c), shape) for writing P."""
        start, ro, h = self._where[(int(r), int(c))]
        br, bc = int(self.bs[r]), int(self.bs[c])
        p = np.arange(br)[:, None]
        q = np.arange(bc)[None, :]
        return start + q * h + ro + p


def index_set(view: BlockView, i: int) -> np.ndarray:
    """Step 1 (Fig. 2): atoms j whose block H_ji is stored, in ascending order.
    This is the structural pattern of block column i; it always contains i."""
    return np.array(sorted(int(j) for j in view.rows_of(i)), dtype=np.int64)


def submatrix_indices(view: BlockView, i: int):
    """Index set I_i, the orbital indices idx_i (ascending atom order), and
    loc_i, the position of atom i's first orbital inside idx_i."""
    atoms = index_set(view, i)
    idx = np.concatenate([np.arange(view.orb_off[a], view.orb_off[a] + view.bs[a])
                          for a in atoms])
    loc = int(sum(int(view.bs[a]) for a in atoms if a < i))
    return atoms, idx, loc


def submatrix(view: BlockView, i: int, mu: float) -> np.ndarray:
    """Step 1 (Fig. 2) with the shift of Eq. 14: T_i = H[idx_i, idx_i] - mu I.
    Blocks not stored in H are zero."""
    atoms, idx, _ = submatrix_indices(view, i)
    n = idx.shape[0]
    T = np.zeros((n, n))
    offs = np.concatenate([[0], np.cumsum(view.bs[atoms])])
    for a, ra in enumerate(atoms):
        for b, cb in enumerate(atoms):
            blk = view.block(ra, cb)
            if blk is not None:
                T[offs[a]:offs[a + 1], offs[b]:offs[b + 1]] = blk
    T[np.arange(n), np.arange(n)] -= mu
    return T


def sign_eigh(T: np.ndarray) -> np.ndarray:
    """Eq. 13: sign(T) = T (T^2)^(-1/2) = V sign(lam) V^T for symmetric T."""
    lam, V = np.linalg.eigh(T)
    return (V * np.sign(lam)) @ V.T


def gershgorin_bound(T: np.ndarray) -> float:
    """max_p sum_q |T_pq|: an upper bound on the spectral radius of T."""
    return float(np.max(np.sum(np.abs(T), axis=1)))


def density_matrix_columns(view: BlockView, i: int, mu: float):
    """Steps 2 and 3 (Fig. 2) for atom i: the b_i columns of
    P_i = 1/2 (E - sign(T_i)[:, loc_i : loc_i + b_i]) over the rows idx_i.
    Returns (atoms, columns) with columns of shape (n_i, b_i)."""
    atoms, idx, loc = submatrix_indices(view, i)
    T = submatrix(view, i, mu)
    S = sign_eigh(T)
    b = int(view.bs[i])
    E = np.zeros((idx.shape[0], b))
    E[loc + np.arange(b), np.arange(b)] = 1.0
    return atoms, 0.5 * (E - S[:, loc:loc + b])


def density_matrix(m, mu: float, atoms=None) -> np.ndarray:
    """P in the same block-column panel layout (and pattern) as H.  Every block
    column i is written only from submatrix i; P is not symmetrised.  With
    ``atoms`` given, only those block columns are filled (others stay NaN)."""
    view = m if isinstance(m, BlockView) else BlockView(m)
    P = np.full_like(view.vals, np.nan)
    todo = range(view.n_atoms) if atoms is None else atoms
    for i in todo:
        rows, cols = density_matrix_columns(view, int(i), mu)
        # rows are ascending and equal the stored pattern of column i, so the
        # columns land in the panel of block column i in the same row order
        off = 0
        for r in rows:
            br = int(view.bs[r])
            P[view.panel_slot(r, i)] = cols[off:off + br, :]
            off += br
    return P


def energy_trace(m, P: np.ndarray):
    """E = tr(P H) and Ne = tr P (Eq. 14 with the energy read as tr(PH), no
    spin factor since P = C C^T).  tr(PH) = sum_{jk} P_jk H_kj = sum over
    stored blocks of P_jk H_jk because H is symmetric, so E is an elementwise
    product over the common pattern.  Sums are exactly rounded (math.fsum)."""
    view = m if isinstance(m, BlockView) else BlockView(m)
    E = math.fsum((np.asarray(P) * view.vals).tolist())
    diag = []
    for c in range(view.n_atoms):
        start, ro, h = view._where[(c, c)]
        b = int(view.bs[c])
        q = np.arange(b)
        diag.append(P[start + q * h + ro + q])
    Ne = math.fsum(np.concatenate(diag).tolist())
    return E, Ne


# ----------------------------------------------------------------------------
# chemical potential
# ----------------------------------------------------------------------------

class SpectralCache:
    """Eigendecomposition of every (unshifted) submatrix H[idx_i, idx_i].

    Shifting by mu does not change eigenvectors, so the submatrix electron
    count is Ne(mu) = sum_i sum_k theta(mu - lam_ik) * || V_ik[loc_i:loc_i+b_i] ||^2
    (the diagonal of P_ii = V theta(mu - lam) V^T summed over atom i's
    orbitals).  It is monotone in mu."""

    def __init__(self, m, atoms=None):
        self.view = m if isinstance(m, BlockView) else BlockView(m)
        todo = range(self.view.n_atoms) if atoms is None else atoms
        lam, wts = [], []
        for i in todo:
            _, _, loc = submatrix_indices(self.view, int(i))
            T = submatrix(self.view, int(i), 0.0)
            w, V = np.linalg.eigh(T)
            b = int(self.view.bs[i])
            lam.append(w)
            wts.append(np.sum(V[loc:loc + b, :] ** 2, axis=0))
        self.lam = np.concatenate(lam)
        self.wts = np.concatenate(wts)

    def ne(self, mu: float) -> float:
        occ = self.lam < mu
        half = self.lam == mu   # sign(0) = 0 -> occupation 1/2
        return math.fsum((self.wts * occ).tolist()) + 0.5 * math.fsum((self.wts * half).tolist())


def global_gershgorin_bracket(m):
    """[min_p (h_pp - R_p), max_p (h_pp + R_p)] with R_p = sum_{q != p} |h_pq|:
    every eigenvalue of H (and of every principal submatrix) lies inside."""
    view = m if isinstance(m, BlockView) else BlockView(m)
    N = int(view.orb_off[-1])
    absrow = np.zeros(N)
    diag = np.zeros(N)
    for c in range(view.n_atoms):
        oc = view.orb_off[c]
        bc = int(view.bs[c])
        for r in view.rows_of(c):
            blk = view.block(r, c)
            # column sums of |H| over column c's orbitals == row sums (symmetry)
            absrow[oc:oc + bc] += np.sum(np.abs(blk), axis=0)
            if r == c:
                diag[oc:oc + bc] = np.diag(blk)
    R = absrow - np.abs(diag)
    return float(np.min(diag - R)), float(np.max(diag + R))


def find_mu(m, n_target: float, max_steps: int = 60, accept: float = 0.5,
            cache: SpectralCache | None = None, mu_start: float | None = None):
    """Bisection for mu (Eq. 14 leaves the rule open): start from the global
    Gershgorin bracket, take midpoints, stop at the first midpoint with
    |Ne(mu) - n_target| < accept, else after ``max_steps`` evaluations.

    ``mu_start`` (a warm start, e.g. the previous geometry's mu) replaces the
    first midpoint: Ne is evaluated there first and, if it is not accepted, it
    becomes the lower or upper end of the bracket (kept inside the Gershgorin
    bracket) before the midpoints continue.  Returns (mu, steps, history)."""
    cache = cache or SpectralCache(m)
    lo, hi = global_gershgorin_bracket(m)
    hist = []
    mid = 0.5 * (lo + hi)
    for step in range(1, max_steps + 1):
        mid = mu_start if (step == 1 and mu_start is not None) else 0.5 * (lo + hi)
        ne = cache.ne(mid)
        hist.append((mid, ne))
        if abs(ne - n_target) < accept:
            return mid, step, hist
        if ne < n_target:
            lo = min(max(lo, mid), hi)
        else:
            hi = max(min(hi, mid), lo)
    return mid, max_steps, hist


# ----------------------------------------------------------------------------
# exact reference (whole matrix)
# ----------------------------------------------------------------------------

def full_P(H: np.ndarray, n_occ: int) -> np.ndarray:
    """Exact projector onto the n_occ lowest eigenvectors of the whole H
    (what the submatrix method approximates)."""
    lam, V = np.linalg.eigh(H)
    Vo = V[:, :n_occ]
    return Vo @ Vo.T
