"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test is chosen so that a plausible slip in the oracle (a dropped shift, a
wrong sign, a wrong column offset, a transposed block, a missing factor 1/2)
fails at least one of them.  None of them re-types the oracle's formulas.
"""
import json
import math
import os

import numpy as np
import pytest

import synth
from oracle import submatrix as om
from oracle import newton_schulz as ons

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _dense(P_vals, m):
    return synth.to_dense(m.with_vals(P_vals))


# ---------------------------------------------------------------- sign (Eq. 13)

@pytest.mark.parametrize("seed", range(6))
def test_sign_two_by_two_closed_form(seed):
    rng = np.random.default_rng(seed)
    a, d, b = rng.normal(size=3)
    T = np.array([[a, b], [b, d]])
    m = 0.5 * (a + d)
    r = math.sqrt((0.5 * (a - d)) ** 2 + b * b)
    lo, hi = m - r, m + r
    if lo < 0 < hi:
        expect = (T - m * np.eye(2)) / r
    elif lo > 0:
        expect = np.eye(2)
    else:
        expect = -np.eye(2)
    np.testing.assert_allclose(om.sign_eigh(T), expect, atol=1e-14)


def test_sign_diagonal():
    d = np.array([-3.0, 0.25, 1e-3, -1e-6, 7.0])
    np.testing.assert_array_equal(om.sign_eigh(np.diag(d)), np.diag(np.sign(d)))


@pytest.mark.parametrize("n", [3, 17, 64])
def test_sign_invariants(n):
    rng = np.random.default_rng(n)
    A = rng.normal(size=(n, n))
    T = A + A.T
    S = om.sign_eigh(T)
    np.testing.assert_allclose(S, S.T, atol=1e-12)
    np.testing.assert_allclose(S @ S, np.eye(n), atol=1e-12)
    np.testing.assert_allclose(S @ T, T @ S, atol=1e-11 * np.abs(T).max())
    # sign(T) T = |T| is positive semidefinite with the same singular values
    np.testing.assert_allclose(np.sort(np.linalg.eigvalsh(S @ T)),
                               np.sort(np.abs(np.linalg.eigvalsh(T))), atol=1e-11)


def test_gershgorin_bounds_spectral_radius():
    rng = np.random.default_rng(3)
    A = rng.normal(size=(40, 40))
    T = A + A.T
    assert om.gershgorin_bound(T) >= np.max(np.abs(np.linalg.eigvalsh(T))) - 1e-12


# ----------------------------------------------------- method (Fig. 2 + Eq. 14)

def test_three_site_chain_golden():
    g = json.load(open(os.path.join(GOLDEN, "three_site_chain.json")))
    t = g["t"]
    m = synth.from_pairs([1, 1, 1], [(0, 1), (1, 2)], [np.array([[t]]), np.array([[t]])],
                         g["onsite"], n_occ=2)
    v = om.BlockView(m)
    assert list(om.index_set(v, 0)) == [0, 1]
    assert list(om.index_set(v, 1)) == [0, 1, 2]
    assert list(om.index_set(v, 2)) == [1, 2]
    P = om.density_matrix(m, g["mu"])
    Pd = _dense(P, m)
    np.testing.assert_allclose(Pd[0:2, 0], g["P_column_0_rows_0_1"], atol=1e-15)
    np.testing.assert_allclose(Pd[0:3, 1], g["P_column_1_rows_0_1_2"], atol=1e-15)
    np.testing.assert_allclose(Pd[1:3, 2], g["P_column_2_rows_1_2"], atol=1e-15)
    assert Pd[2, 0] == 0.0 and Pd[0, 2] == 0.0   # not in the pattern
    E, Ne = om.energy_trace(m, P)
    assert abs(E - g["E_trace_PH"]) < 1e-14
    assert abs(Ne - g["Ne_trace_P"]) < 1e-14


def test_fully_coupled_is_exact_projector():
    """Every index set is the whole system, so the submatrix method must return
    the exact spectral projector: idempotent, commuting with H, trace n_occ,
    tr(PH) = sum of the n_occ lowest eigenvalues."""
    m = synth.fully_coupled_lattice(seed=4, n_orb=4)
    H = synth.to_dense(m)
    lam = np.linalg.eigvalsh(H)
    mu = 0.5 * (lam[m.n_occ - 1] + lam[m.n_occ])
    assert lam[m.n_occ] - lam[m.n_occ - 1] > 0.1
    P = om.density_matrix(m, mu)
    Pd = _dense(P, m)
    np.testing.assert_allclose(Pd, Pd.T, atol=1e-13)
    np.testing.assert_allclose(Pd @ Pd, Pd, atol=1e-13)
    np.testing.assert_allclose(Pd @ H, H @ Pd, atol=1e-13)
    E, Ne = om.energy_trace(m, P)
    assert abs(Ne - m.n_occ) < 1e-12
    assert abs(E - math.fsum(lam[:m.n_occ])) < 1e-12
    # and the oracle's whole-matrix reference agrees
    np.testing.assert_allclose(om.full_P(H, m.n_occ), Pd, atol=1e-12)


def test_block_diagonal_closed_form():
    """No coupling between atoms (cutoff below the spacing): each submatrix is
    the diagonal onsite block, so P = diag(theta(mu - h_pp))."""
    m = synth.lattice_system(3, 4, 0.5, seed=2)
    assert m.nnzb == m.n_atoms
    h = np.diag(synth.to_dense(m))
    mu = 0.1
    P = om.density_matrix(m, mu)
    np.testing.assert_array_equal(_dense(P, m), np.diag((h < mu).astype(float)))
    E, Ne = om.energy_trace(m, P)
    assert Ne == float(np.sum(h < mu))
    assert abs(E - math.fsum(h[h < mu])) < 1e-13


def test_column_offsets_nonuniform_blocks():
    """Atoms of different sizes: the columns of atom i are taken at loc_i, the
    offset of its first orbital inside the submatrix.  Checked on a system
    where the submatrix of every atom is the whole (fully coupled) system."""
    rng = np.random.default_rng(11)
    bs = [3, 1, 4, 2]
    pairs = [(i, j) for i in range(4) for j in range(i + 1, 4)]
    blocks = [0.3 * rng.normal(size=(bs[i], bs[j])) for i, j in pairs]
    onsite = rng.normal(size=sum(bs)) * 2.0
    m = synth.from_pairs(bs, pairs, blocks, onsite, n_occ=5)
    H = synth.to_dense(m)
    lam, V = np.linalg.eigh(H)
    mu = 0.5 * (lam[4] + lam[5])
    Pd = _dense(om.density_matrix(m, mu), m)
    expect = V[:, :5] @ V[:, :5].T
    np.testing.assert_allclose(Pd, expect, atol=1e-12)


def test_truncated_columns_match_direct_submatrix_projector():
    """On a truncated system, column block i of P equals the spectral
    projector of the (explicitly sliced) dense principal submatrix."""
    m = synth.lattice_system(4, 2, 1.2, seed=5, jitter=0.05)
    H = synth.to_dense(m)
    off = m.orb_off
    view = om.BlockView(m)
    mu = 0.03
    P = _dense(om.density_matrix(m, mu), m)
    for i in (0, 7, 31, 63):
        rows = m.row_idx[m.col_ptr[i]:m.col_ptr[i + 1]]
        idx = np.concatenate([np.arange(off[a], off[a + 1]) for a in sorted(rows)])
        lam, V = np.linalg.eigh(H[np.ix_(idx, idx)])
        Pi = (V * (lam < mu)) @ V.T
        cols = np.arange(off[i], off[i + 1])
        pos = np.searchsorted(idx, cols)
        np.testing.assert_allclose(P[np.ix_(idx, cols)], Pi[:, pos], atol=1e-12)
        mask = np.ones(H.shape[0], bool)
        mask[idx] = False
        assert np.all(P[mask][:, cols] == 0.0)
        assert len(om.index_set(view, i)) == len(rows)


def test_truncation_error_decays_with_submatrix_radius():
    """The same H (couplings within 1.5) on wider structural patterns: the
    submatrix approximation approaches the exact projector."""
    errs = []
    for rc in (1.5, 2.0, 2.5):
        m = synth.lattice_system(6, 4, rc, seed=0, coupling_cutoff=1.5)
        H = synth.to_dense(m)
        lam = np.linalg.eigvalsh(H)
        mu = 0.5 * (lam[m.n_occ - 1] + lam[m.n_occ])
        P = om.density_matrix(m, mu)
        E, Ne = om.energy_trace(m, P)
        Pex = om.full_P(H, m.n_occ)
        Eex = math.fsum(lam[:m.n_occ])
        dP = np.max(np.abs(_dense(P, m) - np.where(_dense(np.ones_like(P), m) != 0, Pex, 0)))
        errs.append((abs(E - Eex) / abs(Eex), dP, abs(Ne - m.n_occ)))
    rel = [e[0] for e in errs]
    assert rel[0] > rel[1] > rel[2]
    assert errs[0][1] > errs[2][1]
    assert rel[2] < 1e-4


def test_symmetrisation_invariance():
    """E and Ne do not change when P is replaced by P^T on the common
    (symmetric) pattern, since H is symmetric."""
    m = synth.lattice_system(4, 2, 1.5, seed=9, jitter=0.05)
    P = om.density_matrix(m, 0.0)
    Pd = _dense(P, m)
    PT = Pd.T
    E1, N1 = om.energy_trace(m, P)
    H = synth.to_dense(m)
    assert abs(E1 - math.fsum((PT * H).ravel().tolist())) < 1e-12
    assert abs(N1 - math.fsum(np.diag(PT).tolist())) < 1e-13


# ------------------------------------------------------------- chemical potential

def test_electron_count_two_routes_and_monotone():
    m = synth.config1()
    cache = om.SpectralCache(m)
    mus = np.linspace(-1.0, 1.0, 9)
    nes = [cache.ne(mu) for mu in mus]
    assert all(b >= a - 1e-12 for a, b in zip(nes, nes[1:]))
    for mu in (-0.7, 0.0013, 0.45):
        _, Ne = om.energy_trace(m, om.density_matrix(m, mu))
        assert abs(Ne - cache.ne(mu)) < 1e-10


def test_gershgorin_bracket_three_site_chain():
    """H = [[-1, t, 0], [t, 1, t], [0, t, -1]], t = 3/4: the row intervals are
    [-1.75, -0.25], [-0.5, 2.5], [-1.75, -0.25], so the bracket is
    [-1.75, 2.5].  (With |h_pp| wrongly counted in the radius it would be
    [-2.75, 3.5].)"""
    g = json.load(open(os.path.join(GOLDEN, "three_site_chain.json")))
    t = g["t"]
    m = synth.from_pairs([1, 1, 1], [(0, 1), (1, 2)], [np.array([[t]]), np.array([[t]])],
                         g["onsite"], n_occ=2)
    assert om.global_gershgorin_bracket(m) == (-1.75, 2.5)


def test_gershgorin_bracket_two_atoms_closed_form():
    """Two atoms of two orbitals, onsite diagonals (2, -1) and (1/4, 3),
    coupling block C = [[1, -2], [1/2, 0]] (rows: atom 0's orbitals):
        H = [[ 2,   0,   1,   -2],
             [ 0,  -1,   1/2,  0],
             [ 1,   1/2, 1/4,  0],
             [-2,   0,   0,    3]]
    Row intervals h_pp -+ R_p: [-1, 5], [-1.5, -0.5], [-1.25, 1.75], [1, 5],
    so the bracket is [-1.5, 5].  A transposed coupling block would give row 2
    the radius 3 and the bracket [-2.75, 5]; |h_pp| in the radius would give
    [-4, 8]."""
    C = np.array([[1.0, -2.0], [0.5, 0.0]])
    m = synth.from_pairs([2, 2], [(0, 1)], [C], [2.0, -1.0, 0.25, 3.0], n_occ=2)
    assert om.global_gershgorin_bracket(m) == (-1.5, 5.0)


def test_find_mu_history_with_outlier_state():
    """An isolated high state (one orbital pushed to +20) stretches the
    Gershgorin bracket upwards, so the first midpoints fall above the gap and
    the bisection has to move hi down several times before it lands in the gap:
    the lo / hi update is exercised, and every midpoint is the centre of the
    bracket the previous decisions leave."""
    m = synth.with_onsite_shift(synth.config1(), 0, 3, 20.0)
    lam = np.linalg.eigvalsh(synth.to_dense(m))
    mu, steps, hist = om.find_mu(m, m.n_occ)
    assert steps >= 4
    assert lam[m.n_occ - 1] < mu < lam[m.n_occ]
    lo, hi = om.global_gershgorin_bracket(m)
    for mid, ne in hist:
        assert mid == 0.5 * (lo + hi)
        if ne < m.n_occ:
            lo = mid
        else:
            hi = mid
    assert any(ne < m.n_occ - 0.5 for _, ne in hist) or any(ne > m.n_occ + 0.5 for _, ne in hist[:-1])


def test_find_mu_warm_start():
    """Warm start: a guess inside the gap is accepted at once (one evaluation,
    mu = the guess); the bracket's own midpoint as the guess reproduces the
    cold history exactly; a guess below the gap (Ne short of the target)
    becomes the lower end, so every later midpoint is the centre of
    [guess, ...] and the search still ends in the gap; a guess outside the
    Gershgorin bracket is clamped to it and changes nothing after step 1."""
    m = synth.with_onsite_shift(synth.config1(), 0, 3, 20.0)
    lam = np.linalg.eigvalsh(synth.to_dense(m))
    cache = om.SpectralCache(m)
    mu_c, steps_c, hist_c = om.find_mu(m, m.n_occ, cache=cache)
    mu_w, steps_w, hist_w = om.find_mu(m, m.n_occ, cache=cache, mu_start=mu_c)
    assert (mu_w, steps_w) == (mu_c, 1)
    lo, hi = om.global_gershgorin_bracket(m)
    assert om.find_mu(m, m.n_occ, cache=cache, mu_start=0.5 * (lo + hi)) == (mu_c, steps_c, hist_c)
    g = lam[m.n_occ // 2]          # inside the occupied band: Ne(g) < n_occ - 0.5
    mu_b, steps_b, hist_b = om.find_mu(m, m.n_occ, cache=cache, mu_start=g)
    assert hist_b[0][0] == g and hist_b[0][1] < m.n_occ - 0.5
    assert hist_b[1][0] == 0.5 * (g + hi)
    assert lam[m.n_occ - 1] < mu_b < lam[m.n_occ]
    a, b = g, hi
    for mid, ne in hist_b[1:]:
        assert mid == 0.5 * (a + b)
        if ne < m.n_occ:
            a = mid
        else:
            b = mid
    # below the whole spectrum: Ne = 0, lo stays at the bracket's lo
    mu_o, steps_o, hist_o = om.find_mu(m, m.n_occ, cache=cache, mu_start=lo - 100.0)
    assert hist_o[0][1] == 0.0 and hist_o[1:] == hist_c


def test_find_mu_config1_lands_in_gap():
    m = synth.config1()
    lam = np.linalg.eigvalsh(synth.to_dense(m))
    mu, steps, hist = om.find_mu(m, m.n_occ)
    assert lam[m.n_occ - 1] < mu < lam[m.n_occ]
    assert abs(hist[-1][1] - m.n_occ) < 0.5
    lo, hi = om.global_gershgorin_bracket(m)
    assert lo <= lam[0] and hi >= lam[-1]


# ----------------------------------------------------------------- index sets

def test_config1_index_sets_closed_form():
    """4x4x4 periodic lattice, cutoff 1.5: 1 + 6 (r = 1) + 12 (r = sqrt 2) = 19
    atoms in every index set, n = 76."""
    m = synth.config1()
    v = om.BlockView(m)
    for i in range(m.n_atoms):
        atoms, idx, loc = om.submatrix_indices(v, i)
        assert len(atoms) == 19 and idx.shape[0] == 76
        assert loc == 4 * int(np.searchsorted(atoms, i))


def test_index_sets_brute_force_geometry():
    m = synth.lattice_system(5, 1, 1.6, seed=3, jitter=0.1, vacancy=0.1)
    v = om.BlockView(m)
    pos, box = m.positions, m.box
    for i in range(m.n_atoms):
        d = pos - pos[i]
        d -= box * np.round(d / box)
        expect = np.nonzero(np.sqrt((d ** 2).sum(1)) <= 1.6)[0]
        assert list(om.index_set(v, i)) == list(expect)


# -------------------------------------------------------------- Newton-Schulz

@pytest.mark.parametrize("n", [5, 40, 120])
def test_newton_schulz_reaches_the_eigh_sign(n):
    rng = np.random.default_rng(100 + n)
    Q, _ = np.linalg.qr(rng.normal(size=(n, n)))
    lam = rng.uniform(0.05, 2.0, size=n) * rng.choice([-1.0, 1.0], size=n)
    T = (Q * lam) @ Q.T
    X, k, hist = ons.ns_sign(T, om.gershgorin_bound(T), tol=1e-10)
    assert hist[-1] < 1e-10
    np.testing.assert_allclose(X, (Q * np.sign(lam)) @ Q.T, atol=1e-11)


@pytest.mark.parametrize("d,tol,expect", [
    # one entry x_0 = 1/2 (d = 1, c = 2).  Hand enumeration of the scalar map
    # g(x) = x (3 - x^2) / 2 in exact fractions:
    #   x_0 = 1/2            r_0 = 3/4                 = 0.75
    #   x_1 = 11/16          r_1 = 135/256             = 0.52734375
    #   x_2 = 7117/8192      r_2 = 16457175/67108864   ~ 0.24523
    #   x_3 ~ 0.97530        r_3                       ~ 0.0488
    ([1.0], 0.8, 0), ([1.0], 0.6, 1), ([1.0], 0.3, 2), ([1.0], 0.1, 3),
    # two entries +-1/2: the residual is the Frobenius norm sqrt(2) |x_k^2 - 1|
    # (r_0 ~ 1.0607, r_1 ~ 0.7458, r_2 ~ 0.3468, r_3 ~ 0.069).  tol 0.3 tells
    # the Frobenius norm (3) from the largest entry (which would give 2).
    ([1.0, -1.0], 1.1, 0), ([1.0, -1.0], 0.75, 1), ([1.0, -1.0], 0.35, 2), ([1.0, -1.0], 0.3, 3),
])
def test_scalar_iteration_count_hand_enumerated(d, tol, expect):
    assert ons.ns_scalar_iterations(np.array(d), 2.0, tol=tol) == expect


def test_scalar_iteration_count_cap():
    assert ons.ns_scalar_iterations(np.array([1.0]), 2.0, tol=0.0, max_iter=3) == 3
    assert ons.ns_scalar_iterations(np.array([2.0, -2.0]), 2.0, tol=1e-12) == 0


def test_newton_schulz_diagonal_iteration_count():
    d = np.array([-0.01, 0.3, 2.0, -4.0, 0.05])
    c = np.max(np.abs(d))
    _, k, _ = ons.ns_sign(np.diag(d), c, tol=1e-10)
    # hand count: the slowest entry is 0.01/4 = 0.0025; the scalar map grows a
    # small x by ~1.5 per step until it nears 1, then converges quadratically
    assert k == ons.ns_scalar_iterations(d, c, tol=1e-10)
    x, kk = 0.0025, 0
    while abs(x * x - 1.0) >= 1e-11:
        x, kk = 0.5 * x * (3 - x * x), kk + 1
    assert abs(k - kk) <= 1
