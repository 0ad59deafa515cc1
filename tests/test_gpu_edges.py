"""Degenerate and boundary inputs on the GPU path, against the oracle:

* one atom: a single submatrix, n = b = 5, padded with 27 identity rows;
* no couplings: every submatrix is the atom's own block;
* every index set the whole system: P is the exact projector;
* submatrix dimensions exactly at a tile boundary (n = 64, no padding) and
  one past it (n = 65), for both paddings;
* NaN in H is reported by the sign call that follows build_submatrices.
"""
import numpy as np
import pytest

import synth
from oracle import submatrix as om
from paper_2205_14741_amd import smsign as sm
from gpu_helpers import h_dev, rel, run_fixed_mu

pytestmark = pytest.mark.gpu

PRECS = [("f64", 1e-10), ("f32", 1e-5), ("bf16x3", 1e-4)]   # f64: the iteration stops at ||X^2 - I||_F < 1e-10


def _check(m, mu, prec, tol, pad_to=32):
    P, E, Ne, st, plan = run_fixed_mu(m, mu, prec, pad_to=pad_to)
    Po = om.density_matrix(m, mu)
    Eo, Neo = om.energy_trace(m, Po)
    dP = float(np.max(np.abs(P - Po)))
    assert dP < tol, (prec, dP)
    assert rel(E, Eo) < tol and abs(Ne - Neo) < tol * m.n_orb
    assert np.all(st["status"] >= 1)
    return P, plan


@pytest.mark.parametrize("prec,tol", PRECS)
def test_single_atom(prec, tol, dev):
    onsite = np.array([-2.0, -0.5, 0.7, 1.5, 3.0])
    m = synth.from_pairs([5], [], [], onsite, n_occ=2)
    P, plan = _check(m, 0.1, prec, tol)
    info = plan.info()
    assert info["n"][0] == 5 and info["npad"][0] == 32
    np.testing.assert_allclose(P.reshape(5, 5), np.diag([1.0, 1.0, 0.0, 0.0, 0.0]), atol=tol)


@pytest.mark.parametrize("prec,tol", PRECS)
def test_no_couplings(prec, tol, dev):
    m = synth.lattice_system(3, 4, 0.5, seed=2)          # cutoff below the spacing
    P, plan = _check(m, 0.0, prec, tol)
    assert np.all(plan.info()["n"] == 4)


@pytest.mark.parametrize("prec,tol", PRECS)
def test_fully_coupled_is_exact_projector(prec, tol, dev):
    m = synth.fully_coupled_lattice(seed=4, n_orb=4)     # N = 32: every index set is everything
    lam, V = np.linalg.eigh(synth.to_dense(m))
    mu = 0.5 * (lam[m.n_occ - 1] + lam[m.n_occ])
    P, plan = _check(m, mu, prec, tol)
    assert np.all(plan.info()["n"] == m.n_orb) and np.all(plan.info()["npad"] == 32)
    Pex = V[:, :m.n_occ] @ V[:, :m.n_occ].T
    Pd = synth.to_dense(synth.BlockSparse(**{**m.__dict__, "vals": P}))
    assert np.max(np.abs(Pd - Pex)) < tol


def _two_atoms(b0, b1, seed):
    rng = np.random.default_rng(seed)
    blk = 0.3 * rng.standard_normal((b0, b1))
    onsite = np.concatenate([np.where(np.arange(b) < b // 2, -3.0, 3.0) + 0.3 * rng.standard_normal(b)
                             for b in (b0, b1)])
    return synth.from_pairs([b0, b1], [(0, 1)], [blk], onsite, n_occ=b0 // 2 + b1 // 2)


@pytest.mark.parametrize("b1,pad_to", [(32, 32), (32, 64), (33, 32), (33, 64)])
@pytest.mark.parametrize("prec,tol", PRECS)
def test_tile_boundaries(b1, pad_to, prec, tol, dev):
    m = _two_atoms(32, b1, seed=b1 + pad_to)
    P, plan = _check(m, 0.0, prec, tol, pad_to=pad_to)
    info = plan.info()
    n = 32 + b1
    assert np.all(info["n"] == n)
    assert np.all(info["npad"] == -(-n // pad_to) * pad_to)


@pytest.mark.parametrize("prec,refine", [("f64", 0), ("f32", 0), ("bf16x3", 0), ("bf16x3", 2)])
def test_converged_at_start(prec, refine, dev):
    """T_i = diag(+-2) (no couplings): c = 2 and X_0 = T / c is already a sign
    matrix, exactly in every precision, so the iteration stops after the first
    square with no update (the final X is X_0 itself: stored as T for the
    float32 and 16-bit schedules and rescaled on read-out), or, with
    refinement steps, after exactly those."""
    onsite = np.array([2.5, -1.5, -1.5, 2.5, -1.5, 2.5, 2.5, -1.5, -1.5, -1.5, 2.5, 2.5])
    m = synth.from_pairs([4, 4, 4], [], [], onsite, n_occ=6)
    P, E, Ne, st, plan = run_fixed_mu(m, 0.5, prec, pad_to=32, refine_steps=refine)
    Po = om.density_matrix(m, 0.5)
    assert np.max(np.abs(P - Po)) < 1e-14
    assert np.all(st["scale"] == 2.0)
    assert np.all(st["iters"] == refine) and np.all(st["status"] == (2 if refine else 1))


def test_nonfinite_h_is_reported(dev):
    import torch
    m = synth.config1()
    vals = m.vals.copy()
    vals[17] = np.nan
    plan = sm.Plan(m, 32)
    H = torch.from_numpy(vals).cuda()
    o = sm.default_opts("f64")
    work = sm.Workspace(plan, sm.storage_prec(o), H.device)
    sm.build_submatrices(plan, 0, H, 0.0, o, work.ws, work.stats)
    with pytest.raises(sm.SmError, match="NaN"):
        sm.submatrix_sign(plan, 0, work.ws, o, work.stats)
    # the flag is cleared by the next build: a clean H runs through
    H.copy_(torch.from_numpy(m.vals))
    sm.build_submatrices(plan, 0, H, 0.0, o, work.ws, work.stats)
    sm.submatrix_sign(plan, 0, work.ws, o, work.stats)
    torch.cuda.synchronize()
    assert np.all(work.stats_host()["status"] >= 1)


def _near_sign_chain(seed=7):
    """Four atoms of two orbitals at about -4 and +4, nearest neighbours
    coupled by 0.03-sized blocks: every submatrix is within a few percent of
    a signed identity once scaled by its spectral radius (||X_0^2 - I||_F
    0.02-0.07), while c_G exceeds that radius by the couplings' absolute row
    sums (c_G / rho 1.004-1.024)."""
    rng = np.random.default_rng(seed)
    onsite = np.tile([-4.0, 4.0], 4) + 0.001 * rng.standard_normal(8)
    pairs = [(0, 1), (1, 2), (2, 3)]
    blocks = [0.03 * rng.standard_normal((2, 2)) for _ in pairs]
    return synth.from_pairs([2, 2, 2, 2], pairs, blocks, onsite, n_occ=4)


@pytest.mark.parametrize("prec,tol", PRECS)
def test_first_square_bound_when_the_first_square_has_converged(prec, tol, dev):
    """Power scale within 0.1 % of rho with accel 1: the first square runs
    unscaled (c_G / c > 1) and its residual is already below switch_tol, so
    for split bf16 the first update is a refinement step (two updates in all,
    none in the main phase); the bound it was scaled for lies between
    rho(T) / c and c_G / c, and P matches the oracle."""
    m = _near_sign_chain()
    view = om.BlockView(m)
    o = sm.default_opts(prec, scaling=sm.SM_SCALE_POWER, power_steps=30, scale_margin=1e-3, accel=1,
                        lbound=0.9, retry=0)
    P, E, Ne, st, plan = run_fixed_mu(m, 0.0, opts=o, pad_to=32)
    rho = np.array([np.max(np.abs(np.linalg.eigvalsh(om.submatrix(view, i, 0.0)))) for i in range(m.n_atoms)])
    top0 = st["gersh"] / st["scale"]
    top1 = st["top1"].astype(np.float64)
    print(f"{prec}: c_G/c {top0.round(4)}, top1 {top1.round(4)}, updates {st['iters']}")
    assert np.all(top0 > 1.002)
    assert np.all(top1 >= (rho / st["scale"]) * (1 - 1e-6)) and np.all(top1 <= top0 * (1 + 1e-6))
    assert np.all(st["status"] >= 1)
    if prec == "bf16x3":
        assert np.all(st["iters_low"] == 0) and np.all(st["iters"] == 2)
    Po = om.density_matrix(m, 0.0)
    assert float(np.max(np.abs(P - Po))) < tol
