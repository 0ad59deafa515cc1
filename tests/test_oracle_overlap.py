"""Pins of the S != I oracle (oracle/overlap.py) against closed forms,
invariants and the independent S = I oracle, on the CPU."""
import numpy as np
import pytest
import scipy.linalg

import synth
from oracle import overlap as ov
from oracle import submatrix as om


def test_inv_sqrt_2x2_closed_form():
    """A = [[a, b], [b, a]] has eigenvectors (1, 1)/sqrt 2 and (1, -1)/sqrt 2
    with eigenvalues a + b and a - b, so A^(-1/2) = 1/2 [[p + q, p - q],
    [p - q, p + q]] with p = (a + b)^(-1/2), q = (a - b)^(-1/2)."""
    a, b = 1.3, 0.4
    p, q = (a + b) ** -0.5, (a - b) ** -0.5
    want = 0.5 * np.array([[p + q, p - q], [p - q, p + q]])
    got = ov.inv_sqrt_eigh(np.array([[a, b], [b, a]]))
    assert np.max(np.abs(got - want)) < 1e-15
    assert np.max(np.abs(ov.inv_sqrt_eigh(np.eye(5)) - np.eye(5))) == 0.0
    d = np.array([4.0, 0.25, 9.0])
    assert np.max(np.abs(ov.inv_sqrt_eigh(np.diag(d)) - np.diag([0.5, 2.0, 1.0 / 3.0]))) < 1e-15


def test_inv_sqrt_rejects_indefinite():
    with pytest.raises(ValueError):
        ov.inv_sqrt_eigh(np.array([[1.0, 2.0], [2.0, 1.0]]))


def test_eq12_block_sign():
    """sign([[0, A], [I, 0]]) = [[0, A^(1/2)], [A^(-1/2), 0]]: the result squares
    to I, its zero blocks are exact, its top-right block squared is A and it
    is the inverse of the bottom-left one; for diagonal A the blocks are the
    elementwise square roots."""
    rng = np.random.default_rng(3)
    B = rng.normal(size=(6, 6))
    A = B @ B.T + 6 * np.eye(6)
    n = 6
    Sg = ov.block_sign_eq12(A)
    assert np.max(np.abs(Sg @ Sg - np.eye(2 * n))) < 1e-12
    assert np.all(Sg[:n, :n] == 0) and np.all(Sg[n:, n:] == 0)
    R, Ri = Sg[:n, n:], Sg[n:, :n]
    assert np.max(np.abs(R @ R - A)) < 1e-11
    assert np.max(np.abs(R @ Ri - np.eye(n))) < 1e-12
    d = np.array([4.0, 1.0, 0.25])
    Sd = ov.block_sign_eq12(np.diag(d))
    assert np.max(np.abs(Sd[:3, 3:] - np.diag([2.0, 1.0, 0.5]))) < 1e-15
    assert np.max(np.abs(Sd[3:, :3] - np.diag([0.5, 1.0, 2.0]))) < 1e-15


def test_identity_overlap_reduces_to_orthogonal_oracle():
    """S = I: the generalized-eigenproblem route gives the P of the S = I
    oracle (sign of H - mu I by symmetric eigendecomposition)."""
    m = synth.config1(0)
    S = m.with_vals(np.where(_diag_mask(m), 1.0, 0.0))
    lam = np.linalg.eigvalsh(synth.to_dense(m))
    mu = 0.5 * (lam[m.n_occ - 1] + lam[m.n_occ])
    atoms = [0, 7, 33, 63]
    P1 = ov.density_matrix_overlap(m, S, mu, atoms=atoms)
    P0 = om.density_matrix(m, mu, atoms=atoms)
    sel = ~np.isnan(P0)
    assert np.max(np.abs(P1[sel] - P0[sel])) < 1e-12


def test_diagonal_congruence():
    """S = D^2 with D diagonal positive and H = D K D: H c = lam S c is
    K (D c) = lam (D c), so P(H, S) = D^-1 P(K) D^-1, and since D is diagonal
    this holds submatrix by submatrix; checked against the S = I oracle on K."""
    K = synth.config1(1)
    rng = np.random.default_rng(11)
    dvec = rng.uniform(0.6, 1.7, size=K.n_orb)
    vals_h, vals_s = _congruent_vals(K, dvec)
    Hm, Sm = K.with_vals(vals_h), K.with_vals(vals_s)
    lam = np.linalg.eigvalsh(synth.to_dense(K))
    mu = 0.5 * (lam[K.n_occ - 1] + lam[K.n_occ])
    atoms = [1, 20, 42]
    Pk = om.density_matrix(K, mu, atoms=atoms)
    P = ov.density_matrix_overlap(Hm, Sm, mu, atoms=atoms)
    want, _ = _congruent_vals(K.with_vals(np.nan_to_num(Pk)), 1.0 / dvec)
    sel = ~np.isnan(Pk)
    assert np.max(np.abs(P[sel] - want[sel])) < 1e-12


def test_fully_coupled_is_exact_projector():
    """Every atom couples to every other (2x2x2 lattice, cutoff covers all):
    each submatrix is the whole pencil, so P = C_occ C_occ^T exactly, P S P = P,
    tr(P S) = n_occ and tr(P H) = sum of the n_occ lowest generalized
    eigenvalues."""
    m = synth.fully_coupled_lattice(0)
    s = synth.overlap_for(m, 2)
    Hd, Sd = synth.to_dense(m), synth.to_dense(s)
    lam = scipy.linalg.eigh(Hd, Sd, eigvals_only=True)
    mu = 0.5 * (lam[m.n_occ - 1] + lam[m.n_occ])
    P = ov.density_matrix_overlap(m, s, mu)
    Pd = synth.to_dense(m.with_vals(P))
    Pf = ov.full_P_overlap(Hd, Sd, m.n_occ)
    assert np.max(np.abs(Pd - Pf)) < 1e-12
    assert np.max(np.abs(Pd @ Sd @ Pd - Pd)) < 1e-12
    E, Ne = ov.traces_overlap(m, s, P)
    assert abs(Ne - m.n_occ) < 1e-11
    assert abs(E - lam[:m.n_occ].sum()) < 1e-11


def test_overlap_truncation_decays_with_radius():
    """The submatrix error against the exact pencil projector shrinks as the
    pattern (submatrix radius) grows beyond the couplings' range."""
    errs = []
    for rc in (1.5, 2.0, 2.5):
        base = synth.lattice_system(5, 2, 1.5, seed=4)
        wide = synth.lattice_system(5, 2, rc, seed=4)
        m = _on_pattern(base, wide)
        s = _on_pattern(synth.overlap_for(base, 4), wide)
        Hd, Sd = synth.to_dense(m), synth.to_dense(s)
        lam = scipy.linalg.eigh(Hd, Sd, eigvals_only=True)
        mu = 0.5 * (lam[m.n_occ - 1] + lam[m.n_occ])
        P = ov.density_matrix_overlap(m, s, mu)
        Pf = ov.full_P_overlap(Hd, Sd, m.n_occ)
        errs.append(float(np.max(np.abs(synth.to_dense(m.with_vals(P)) - _restrict(Pf, m)))))
    assert errs[0] > errs[1] > errs[2]


# ---------------------------------------------------------------- helpers

def _diag_mask(m):
    """Entries of the diagonal of m in its panel layout."""
    mask = np.zeros(m.vals.shape[0], dtype=bool)
    for c in range(m.n_atoms):
        rows = m.row_idx[m.col_ptr[c]:m.col_ptr[c + 1]]
        ro = int(m.block_size[rows[rows < c]].sum())
        h = int(m.block_size[rows].sum())
        b = int(m.block_size[c])
        for q in range(b):
            mask[int(m.panel_off[c]) + q * h + ro + q] = True
    return mask


def _congruent_vals(m, d):
    """Panel values of D A D and of D^2 (on A's pattern, zero off the
    diagonal) for A = m and the diagonal d."""
    off = m.orb_off
    out = m.vals.copy()
    s = np.zeros_like(m.vals)
    for c in range(m.n_atoms):
        rows = m.row_idx[m.col_ptr[c]:m.col_ptr[c + 1]]
        h = int(m.block_size[rows].sum())
        b = int(m.block_size[c])
        ridx = np.concatenate([np.arange(off[r], off[r + 1]) for r in rows])
        cidx = np.arange(off[c], off[c + 1])
        panel = out[m.panel_off[c]:m.panel_off[c] + h * b].reshape(b, h)   # [col][row]
        panel *= d[cidx][:, None] * d[ridx][None, :]
        sp = s[m.panel_off[c]:m.panel_off[c] + h * b].reshape(b, h)
        for q in range(b):
            sp[q, np.nonzero(ridx == cidx[q])[0]] = d[cidx[q]] ** 2
    return out, s


def _on_pattern(m, wide):
    """m's values placed on the (superset) pattern of ``wide``: explicit zero
    blocks widen the index sets."""
    dm = synth.to_dense(m)
    out = np.zeros_like(wide.vals)
    off = wide.orb_off
    for c in range(wide.n_atoms):
        rows = wide.row_idx[wide.col_ptr[c]:wide.col_ptr[c + 1]]
        h = int(wide.block_size[rows].sum())
        b = int(wide.block_size[c])
        ridx = np.concatenate([np.arange(off[r], off[r + 1]) for r in rows])
        cidx = np.arange(off[c], off[c + 1])
        out[wide.panel_off[c]:wide.panel_off[c] + h * b] = dm[np.ix_(ridx, cidx)].T.ravel()
    return wide.with_vals(out, name=m.name)


def _restrict(D, m):
    """A dense matrix restricted to m's stored block pattern (zeros elsewhere)."""
    mask = synth.to_dense(m.with_vals(np.ones_like(m.vals))) != 0
    return np.where(mask, D, 0.0)
