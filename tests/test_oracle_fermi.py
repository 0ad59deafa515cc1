"""Pins of the finite-temperature oracle (oracle/fermi.py) against closed
forms, limits, invariants and the independent zero-temperature oracle, on
the CPU."""
import math

import numpy as np

import synth
from oracle import fermi as fd
from oracle import submatrix as om


def _f(x, beta):
    return 1.0 / (1.0 + math.exp(beta * x))


def test_fermi_2x2_closed_form():
    """T = m I + N with N traceless symmetric, N^2 = r^2 I, so for any f
    f(T) = (f(m + r) + f(m - r)) / 2 I + (f(m + r) - f(m - r)) / (2 r) N."""
    for a, b, d, beta in [(0.3, -0.7, -1.1, 2.5), (2.0, 0.05, 1.9, 40.0), (-0.4, 1.2, 0.6, 0.3)]:
        T = np.array([[a, b], [b, d]])
        m = 0.5 * (a + d)
        r = math.hypot(0.5 * (a - d), b)
        N = T - m * np.eye(2)
        fp, fm = _f(m + r, beta), _f(m - r, beta)
        want = 0.5 * (fp + fm) * np.eye(2) + (fp - fm) / (2 * r) * N
        assert np.max(np.abs(fd.fermi_eigh(T, beta) - want)) < 1e-15


def test_particle_hole_and_commutation():
    """f(-x) = 1 - f(x), so f(T) + f(-T) = I; f(T) commutes with T and is
    symmetric with every eigenvalue in (0, 1)."""
    rng = np.random.default_rng(5)
    B = rng.normal(size=(9, 9))
    T = B + B.T
    F = fd.fermi_eigh(T, 1.7)
    assert np.max(np.abs(F + fd.fermi_eigh(-T, 1.7) - np.eye(9))) < 1e-14
    assert np.max(np.abs(F @ T - T @ F)) < 1e-13
    assert np.max(np.abs(F - F.T)) < 1e-15
    w = np.linalg.eigvalsh(F)
    assert w.min() > 0 and w.max() < 1


def test_large_beta_gives_the_sign_oracle():
    """With mu in the gap of every sampled submatrix spectrum and beta times
    the distance of the nearest eigenvalue at 60, every occupation is within
    e^-60 of 0 or 1: P equals the zero-temperature P of Eq. 14."""
    m = synth.config1(0)
    lam = np.linalg.eigvalsh(synth.to_dense(m))
    mu = 0.5 * (lam[m.n_occ - 1] + lam[m.n_occ])
    atoms = [0, 5, 17, 40, 63]
    cache = fd.FermiCache(m, atoms=atoms)
    gap = float(np.min(np.abs(cache.lam - mu)))
    assert gap > 0.05
    beta = 60.0 / gap
    P = fd.density_matrix_fd(m, mu, beta, atoms=atoms)
    P0 = om.density_matrix(m, mu, atoms=atoms)
    sel = ~np.isnan(P0)
    assert np.max(np.abs(P[sel] - P0[sel])) < 1e-12


def test_small_beta_gives_half_identity():
    """f(x) = 1/2 - beta x / 4 + O(beta^3): as beta -> 0, P -> 1/2 I on the
    pattern and Ne -> N / 2."""
    m = synth.config1(2)
    beta = 1e-9
    P = fd.density_matrix_fd(m, 0.1, beta)
    want = np.where(_diag_mask(m), 0.5, 0.0)
    assert np.max(np.abs(P - want)) < 1e-8
    _, Ne = om.energy_trace(m, P)
    assert abs(Ne - 0.5 * m.n_orb) < 1e-6


def test_cache_count_matches_the_assembled_P():
    """Two routes to Ne: the eigenvector weights on the atom's own orbitals
    (FermiCache) and the trace of the assembled P (energy_trace)."""
    m = synth.water_system(6, 1.5, seed=2)
    beta, mu = 3.0, -0.4
    P = fd.density_matrix_fd(m, mu, beta)
    _, Ne = om.energy_trace(m, P)
    assert abs(fd.FermiCache(m).ne(mu, beta) - Ne) < 1e-10


def test_derivative_matches_finite_differences():
    m = synth.config1(1)
    cache = fd.FermiCache(m)
    for beta, mu in [(2.0, 0.0), (15.0, -0.3)]:
        h = 1e-5
        fdiff = (cache.ne(mu + h, beta) - cache.ne(mu - h, beta)) / (2 * h)
        assert abs(cache.dne(mu, beta) - fdiff) < 1e-6 * max(1.0, abs(fdiff))
        assert cache.dne(mu, beta) > 0


def test_dense_pattern_is_the_whole_matrix_function():
    """Every atom coupled to every other: each submatrix is the whole
    H - mu I, so P = f(H - mu I) of the dense matrix and
    Ne = sum_k f(lam_k - mu) over its eigenvalues."""
    m = synth.fully_coupled_lattice(4)
    H = synth.to_dense(m)
    beta, mu = 4.0, 0.2
    P = fd.density_matrix_fd(m, mu, beta)
    lam, V = np.linalg.eigh(H)
    occ = np.array([_f(x - mu, beta) for x in lam])
    Pd = (V * occ) @ V.T
    assert np.max(np.abs(synth.to_dense(m.with_vals(P)) - Pd)) < 1e-12
    _, Ne = om.energy_trace(m, P)
    assert abs(Ne - math.fsum(occ.tolist())) < 1e-11


def test_find_mu_fd_meets_the_count():
    """Ne(mu) is continuous and increasing: bisection meets any count to the
    tolerance, and a larger count needs a larger mu."""
    m = synth.config1(0)
    cache = fd.FermiCache(m)
    mus = []
    for target in (m.n_occ - 3.3, m.n_occ, m.n_occ + 2.5):
        mu, steps, ne = fd.find_mu_fd(m, target, 8.0, tol=1e-9, cache=cache)
        assert abs(ne - target) <= 1e-9 and steps < 200
        assert abs(cache.ne(mu, 8.0) - target) <= 1e-9
        mus.append(mu)
    assert mus[0] < mus[1] < mus[2]


def _diag_mask(m):
    mask = np.zeros(m.vals.shape[0], dtype=bool)
    for c in range(m.n_atoms):
        rows = m.row_idx[m.col_ptr[c]:m.col_ptr[c + 1]]
        ro = int(m.block_size[rows[rows < c]].sum())
        h = int(m.block_size[rows].sum())
        b = int(m.block_size[c])
        for q in range(b):
            mask[m.panel_off[c] + q * h + ro + q] = True
    return mask
