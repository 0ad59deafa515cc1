"""The non-orthogonal basis (S != I) on the GPU through the C ABI, against the
oracle (oracle/overlap.py): the inverse square roots of the overlap
submatrices (Eq. 12), and P of Eq. 14 on the submatrix pairs with tr(PH) and
tr(PS)."""
import numpy as np
import pytest
import scipy.linalg

import synth
from oracle import overlap as ov
from oracle import submatrix as om
from paper_2205_14741_amd import smsign as sm
from gpu_helpers import h_dev, run_fixed_mu, rel

pytestmark = pytest.mark.gpu


def _pencil_gap_mu(m, s):
    lam = scipy.linalg.eigh(synth.to_dense(m), synth.to_dense(s), eigvals_only=True)
    return 0.5 * (lam[m.n_occ - 1] + lam[m.n_occ])


def _workspaces(plan, dev):
    import torch
    o = sm.default_opts("f64", retry=0)
    w = sm.Workspace(plan, sm.SM_F64, dev)
    aux = torch.empty_like(w.ws)
    return o, w, aux


def _run(m, s, mu, pad_to=64, max_chunk_elems=0):
    import torch
    plan = sm.Plan(m, pad_to, max_chunk_elems)
    H, S = h_dev(m), h_dev(s)
    o, w, aux = _workspaces(plan, H.device)
    E, Ne = sm.sm_density_matrix_overlap(plan, H, S, mu, o, w.ws, aux, w.P, w.stats)
    torch.cuda.synchronize()
    return w.P.cpu().numpy(), E, Ne, w.stats_host(), plan


@pytest.mark.parametrize("make", [synth.config1, lambda: synth.water_system(16, 1.5, 3)],
                         ids=["config1", "water16"])
def test_inverse_square_roots(make, dev):
    """Z_i in the auxiliary workspace equals T_i(S)^(-1/2) of the oracle
    (eigendecomposition), to 1e-12, for every submatrix."""
    import torch
    m = make()
    s = synth.overlap_for(m, 1)
    plan = sm.Plan(m, 64)
    S = h_dev(s)
    o, w, aux = _workspaces(plan, S.device)
    steps, r = sm.sm_overlap_inv_sqrt(plan, 0, S, aux, w.ws)
    torch.cuda.synchronize()
    print(f"{steps} steps, residual {r:.2e}")
    assert r < 1e-12 and steps < 20
    reg, off = plan.ws_layout(sm.SM_F64)
    info = plan.info()
    mats = aux.cpu().numpy()[reg[0]:reg[1]].view(np.float64)
    vs = om.BlockView(s)
    worst = 0.0
    for g in range(m.n_atoms):
        i = int(info["order"][g])
        npad, n = int(info["npad"][i]), int(info["n"][i])
        Z = mats[off[g]: off[g] + npad * npad].reshape(npad, npad).T
        Zo = ov.inv_sqrt_eigh(ov.overlap_submatrix(vs, i))
        worst = max(worst, float(np.abs(Z[:n, :n] - Zo).max()))
        assert np.array_equal(Z[n:, n:], np.eye(npad - n))
    print(f"max |Z - T(S)^-1/2| {worst:.2e}")
    assert worst < 1e-12


@pytest.mark.parametrize("make,pad_to", [(synth.config1, 64), (synth.config1, 32),
                                         (lambda: synth.water_system(16, 1.5, 3), 64)],
                         ids=["config1-64", "config1-32", "water16"])
def test_density_matrix_overlap(make, pad_to, dev):
    """P of Eq. 14 (S != I) against the oracle's generalized eigendecomposition
    of every submatrix pair: max |dP| < 1e-9, tr(PH) and tr(PS) to 1e-11."""
    m = make()
    s = synth.overlap_for(m, 1)
    mu = _pencil_gap_mu(m, s)
    P, E, Ne, st, plan = _run(m, s, mu, pad_to)
    Po = ov.density_matrix_overlap(m, s, mu)
    Eo, Neo = ov.traces_overlap(m, s, Po)
    dP = float(np.max(np.abs(P - Po)))
    print(f"max|dP| {dP:.2e}, E {E:.12f} ({Eo:.12f}), Ne {Ne:.10f} ({Neo:.10f}), iters "
          f"{st['iters'].min()}-{st['iters'].max()}")
    assert dP < 1e-9
    assert rel(E, Eo) < 1e-11 and abs(Ne - Neo) < 1e-9
    assert np.all(st["status"] == 1)


def test_overlap_chunked(dev):
    """Several chunks (the auxiliary workspace is rebuilt per chunk) give the
    single-chunk result."""
    m = synth.water_system(16, 1.5, 3)
    s = synth.overlap_for(m, 1)
    mu = _pencil_gap_mu(m, s)
    P1, E1, Ne1, _, p1 = _run(m, s, mu)
    P2, E2, Ne2, _, p2 = _run(m, s, mu, max_chunk_elems=3 * 320 * 320 * 8)
    assert p2.n_chunks > 2
    assert float(np.max(np.abs(P1 - P2))) < 1e-12 and abs(E1 - E2) < 1e-10 * abs(E1)


def test_fully_coupled_overlap_is_exact(dev):
    """Every submatrix is the whole pencil: P is the exact generalized
    projector, P S P = P, tr(PS) = n_occ."""
    m = synth.fully_coupled_lattice(0)
    s = synth.overlap_for(m, 2)
    mu = _pencil_gap_mu(m, s)
    P, E, Ne, st, _ = _run(m, s, mu)
    Hd, Sd = synth.to_dense(m), synth.to_dense(s)
    Pd = synth.to_dense(m.with_vals(P))
    Pf = ov.full_P_overlap(Hd, Sd, m.n_occ)
    assert float(np.max(np.abs(Pd - Pf))) < 1e-10
    assert float(np.max(np.abs(Pd @ Sd @ Pd - Pd))) < 1e-10
    assert abs(Ne - m.n_occ) < 1e-9


def test_identity_overlap_matches_orthogonal_path(dev):
    """S = I: Z_i = I and K_i = T_i - mu I, so P equals the S = I path's."""
    m = synth.config1(0)
    s = synth.overlap_for(m, 1, strength=0.0)
    mu = _pencil_gap_mu(m, s)
    P, E, Ne, _, _ = _run(m, s, mu)
    P0, E0, Ne0, _, _ = run_fixed_mu(m, mu, "f64", pad_to=64)
    assert float(np.max(np.abs(P - P0))) < 1e-12
    assert rel(E, E0) < 1e-13


def test_overlap_rejects_unsupported_schedules(dev):
    m = synth.config1()
    s = synth.overlap_for(m, 1)
    plan = sm.Plan(m, 64)
    H, S = h_dev(m), h_dev(s)
    o, w, aux = _workspaces(plan, H.device)
    for bad in (sm.default_opts("f64"),                       # retry on
                sm.default_opts("f64", retry=0, scaling=sm.SM_SCALE_LEARNED),
                sm.default_opts("f32", retry=0)):
        with pytest.raises(sm.SmError):
            sm.sm_density_matrix_overlap(plan, H, S, 0.0, bad, w.ws, aux, w.P, w.stats)
    with pytest.raises(sm.SmError):   # K needs this chunk's Z first
        sm.build_submatrices_overlap(plan, 0, H, 0.0, o, w.ws, aux, w.stats)


def test_overlap_scaled_first_step_from_the_square(dev):
    """The non-orthogonal path with a power scale and scaled Newton-Schulz
    (accel 1): the first step of every K_i = Z_i T_i(H) Z_i takes its scale
    from the first square's column-sum bound (stats.top1 between 1 and
    c_G / c), and P still matches the oracle to 1e-9."""
    import torch
    m = synth.water_system(16, 1.5, 3)
    s = synth.overlap_for(m, 1)
    mu = _pencil_gap_mu(m, s)
    plan = sm.Plan(m, 64)
    H, S = h_dev(m), h_dev(s)
    _, w, aux = _workspaces(plan, H.device)
    o = sm.default_opts("f64", retry=0, scaling=sm.SM_SCALE_POWER, power_steps=20, scale_margin=0.02,
                        accel=1, lbound=0.01)
    E, Ne = sm.sm_density_matrix_overlap(plan, H, S, mu, o, w.ws, aux, w.P, w.stats)
    torch.cuda.synchronize()
    P, st = w.P.cpu().numpy(), w.stats_host()
    top0 = st["gersh"] / st["scale"]
    bounded = top0 > 1.0 + 1e-9
    print(f"{int(bounded.sum())} of {m.n_atoms} with c_G/c > 1: top {top0[bounded].mean():.2f} -> "
          f"{st['top1'][bounded].mean():.2f}; updates {st['iters'].mean():.2f}")
    assert bounded.sum() > m.n_atoms // 2
    assert np.all(st["top1"][bounded] >= 1.0) and np.all(st["top1"][bounded] <= top0[bounded] * (1 + 1e-6))
    assert np.all(st["status"] == 1)
    Po = ov.density_matrix_overlap(m, s, mu)
    Eo, Neo = ov.traces_overlap(m, s, Po)
    assert float(np.max(np.abs(P - Po))) < 1e-9
    assert rel(E, Eo) < 1e-11 and abs(Ne - Neo) < 1e-9
