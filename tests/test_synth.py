"""Seeded generators: layout, symmetry, determinism, the stated geometry and
the gap that the workloads rely on."""
import math

import numpy as np
import pytest

import synth


def _check_layout(m):
    n = m.n_atoms
    assert m.col_ptr.shape == (n + 1,) and m.panel_off.shape == (n + 1,)
    h = m.panel_height()
    assert np.all(np.diff(m.panel_off) == h * m.block_size)
    assert m.vals.shape == (int(m.panel_off[-1]),)
    for c in range(n):
        rows = m.row_idx[m.col_ptr[c]:m.col_ptr[c + 1]]
        assert np.all(np.diff(rows) > 0) and c in rows


@pytest.mark.parametrize("make", [synth.config1,
                                  lambda: synth.lattice_system(4, 3, 1.8, 1, jitter=0.05, vacancy=0.05),
                                  lambda: synth.water_system(12, 1.4, 0)])
def test_layout_and_symmetry(make):
    m = make()
    _check_layout(m)
    H = synth.to_dense(m)
    assert np.array_equal(H, H.T)
    assert np.all(np.isfinite(H))


def test_seed_determinism():
    a, b, c = synth.config1(0), synth.config1(0), synth.config1(1)
    assert np.array_equal(a.vals, b.vals)
    assert not np.array_equal(a.vals, c.vals)
    w1, w2 = synth.water_system(10, 1.5, 3), synth.water_system(10, 1.5, 3)
    assert np.array_equal(w1.vals, w2.vals) and np.array_equal(w1.positions, w2.positions)


def test_config2_shape_pins_stream_order():
    m = synth.config2(0)
    assert m.n_atoms == 967 and m.n_orb == 5802
    h = m.panel_height()
    assert h.min() == 192 and h.max() == 276


def test_lattice_coupling_law():
    m = synth.lattice_system(3, 2, 1.1, seed=0)
    H = synth.to_dense(m)
    # nearest neighbours at r = 1: entries -exp(-2) U(0.5, 1)
    off = H[0:2, 2:4]  # atoms 0 and 1 are neighbours along z
    assert np.all(off <= -0.5 * math.exp(-2) + 1e-15) and np.all(off >= -math.exp(-2) - 1e-15)
    d = np.diag(H)
    low = d[0::2]
    high = d[1::2]
    assert np.all(low < -0.3) and np.all(high > 0.3)


def test_water_geometry():
    m = synth.water_system(30, 1.0, 2)
    pos, box = m.positions.reshape(30, 3, 3), m.box
    assert abs(box - 30 ** (1 / 3)) < 1e-12

    def mind(a, b):
        d = a - b
        d -= box * np.round(d / box)
        return np.sqrt((d ** 2).sum(-1))

    oh1 = mind(pos[:, 1], pos[:, 0])
    oh2 = mind(pos[:, 2], pos[:, 0])
    np.testing.assert_allclose(oh1, 0.9572 / 3.104, rtol=1e-12)
    np.testing.assert_allclose(oh2, 0.9572 / 3.104, rtol=1e-12)
    hh = mind(pos[:, 1], pos[:, 2])
    ang = 2 * np.arcsin(hh / 2 / oh1)
    np.testing.assert_allclose(np.degrees(ang), 104.52, atol=1e-9)
    O = pos[:, 0]
    dOO = mind(O[:, None], O[None, :]) + np.eye(30) * 10
    assert dOO.min() >= 0.8
    assert list(m.block_size[:6]) == [13, 5, 5, 13, 5, 5]
    assert m.n_occ == 4 * 30


def test_gap_at_target_filling():
    for m, min_gap in ((synth.config1(0), 0.5), (synth.water_system(40, 1.8, 0), 1.0)):
        lam = np.linalg.eigvalsh(synth.to_dense(m))
        assert lam[m.n_occ] - lam[m.n_occ - 1] > min_gap


def test_union_is_block_diagonal():
    a = synth.lattice_system(2, 2, 1.1, 0)
    b = synth.water_system(4, 1.0, 1)
    u = synth.union([a, b])
    _check_layout(u)
    H = synth.to_dense(u)
    na = a.n_orb
    assert np.all(H[:na, na:] == 0)
    assert np.array_equal(H[:na, :na], synth.to_dense(a))
    assert np.array_equal(H[na:, na:], synth.to_dense(b))
    assert u.n_occ == a.n_occ + b.n_occ


def test_trajectory_is_smooth_and_keyed():
    s0 = synth.config5_step(0, n_mol=20, cutoff=1.4)
    s1 = synth.config5_step(1, n_mol=20, cutoff=1.4)
    d = s1.positions - s0.positions
    d -= s0.box * np.round(d / s0.box)
    assert np.max(np.abs(d)) < 0.2
    # same pattern (small moves): values change a little, not wholesale
    if np.array_equal(s0.row_idx, s1.row_idx):
        rel = np.abs(s1.vals - s0.vals).max() / np.abs(s0.vals).max()
        assert 0 < rel < 0.1
    g1 = synth.keyed_normals(7, np.array([1, 2]), np.array([5, 9]), np.array([3, 4]))
    g2 = synth.keyed_normals(7, np.array([2]), np.array([9]), np.array([4]))
    assert np.array_equal(g1[3:], g2)
    big = synth.keyed_normals(1, np.arange(2000), np.arange(2000) + 1, np.full(2000, 50))
    assert abs(big.mean()) < 0.02 and abs(big.std() - 1) < 0.02
