"""Scaled Newton-Schulz (opts.accel) on the GPU.

* the lower bound on the smallest |eigenvalue| of X_0 that a plain run
  derives from its residuals (stats.lb_est) is a true lower bound: checked
  against the oracle's eigenvalues of every submatrix;
* with that bound as l_0 the scaled iteration needs fewer updates and gives
  the same P (float64: to 1e-10 of the plain run; split bf16: within the
  precision target of the oracle);
* a badly wrong l_0 (too large or too small) only costs iterations;
* learned: the scaling network's second output trained on lb_est of earlier
  trajectory steps supplies l_0 on later steps;
* the float64 commutator probe ||X T v - T X v|| / (c ||v||) against a CPU
  recomputation from the final X and the oracle's T.
"""
import numpy as np
import pytest

import synth
from oracle import submatrix as om
from paper_2205_14741_amd import smsign as sm
from gpu_helpers import gap_mu, rel, run_fixed_mu

pytestmark = pytest.mark.gpu


def _system():
    m = synth.water_system(24, 1.4, 5)
    return m, gap_mu(m)


def test_lb_est_is_a_lower_bound(dev):
    m, mu = _system()
    P, E, Ne, st, plan = run_fixed_mu(m, mu, "f64", pad_to=32)
    view = om.BlockView(m)
    have = 0
    for i in range(m.n_atoms):
        if st["lb_est"][i] <= 0:
            continue
        have += 1
        lam = np.linalg.eigvalsh(om.submatrix(view, i, mu))
        x_min = np.min(np.abs(lam)) / st["scale"][i]
        assert st["lb_est"][i] <= x_min * (1 + 1e-6), (i, st["lb_est"][i], x_min)
        assert st["lb_est"][i] > 0.3 * x_min        # and not a trivial one
    assert have == m.n_atoms


@pytest.mark.parametrize("prec,pad,dp_max", [("f64", 32, None), ("bf16x3", 64, 1e-4)])
def test_scaled_ns_fewer_iterations_same_p(prec, pad, dp_max, dev):
    m, mu = _system()
    P0, E0, N0, st0, plan = run_fixed_mu(m, mu, prec, pad_to=pad)
    # a plain float64 run supplies the bounds (relative to c_G)
    _, _, _, stf, _ = run_fixed_mu(m, mu, "f64", pad_to=32)
    lrel = float(np.min(stf["lb_est"] * stf["scale"] / stf["gersh"]))
    P1, E1, N1, st1, _ = run_fixed_mu(m, mu, prec, plan=plan, accel=1, lbound=lrel)
    print(f"{prec}: iterations plain {st0['iters'].mean():.2f} scaled {st1['iters'].mean():.2f} "
          f"(l_0 {lrel:.4f}), max|P1-P0| {np.max(np.abs(P1 - P0)):.2e}")
    assert np.all(st1["status"] >= 1)
    assert st1["iters"].mean() < st0["iters"].mean() - 2.0
    assert np.all(st1["lb0"] > 0)
    if prec == "f64":
        assert np.max(np.abs(P1 - P0)) < 1e-10 and rel(E1, E0) < 1e-12
    else:
        Po = om.density_matrix(m, mu)
        assert np.max(np.abs(P1 - Po)) < dp_max
        Eo, _ = om.energy_trace(m, Po)
        assert rel(E1, Eo) < 1e-5


@pytest.mark.parametrize("factor", [1e-3, 20.0])
def test_scaled_ns_wrong_bound_is_safe(factor, dev):
    """l_0 far too small (the scale then stays near its cap) or far too large
    (eigenvalues below l_0 grow no slower than in the plain iteration): every
    submatrix still converges to the same P."""
    m, mu = _system()
    P0, E0, N0, st0, plan = run_fixed_mu(m, mu, "f64", pad_to=32)
    _, _, _, stf, _ = run_fixed_mu(m, mu, "f64", plan=plan)
    lrel = float(np.median(stf["lb_est"] * stf["scale"] / stf["gersh"]))
    P1, E1, N1, st1, _ = run_fixed_mu(m, mu, "f64", plan=plan, accel=1, lbound=min(lrel * factor, 1.0))
    print(f"l_0 x {factor}: iterations {st1['iters'].mean():.2f} (plain {st0['iters'].mean():.2f})")
    assert np.all(st1["status"] == 1)
    assert np.max(np.abs(P1 - P0)) < 1e-10
    assert st1["iters"].max() <= st0["iters"].max() + 3


def test_learned_lower_bound_on_trajectory(dev):
    """Both outputs of the scaling network trained on plain runs of steps 0-2
    (power-iteration bounds and lb_est); on steps 5-6 the learned scale plus
    scaled Newton-Schulz from the learned l_0 needs fewer updates than the
    learned scale alone, with P unchanged to 1e-9."""
    import torch
    mu = -2.85
    feats, ys = [], []
    for t in (0, 1, 2):
        m = synth.config5_step(t, n_mol=32, cutoff=1.5)
        o = sm.default_opts("f64", scaling=sm.SM_SCALE_POWER, power_steps=40, scale_margin=0.02)
        _, _, _, st, _ = run_fixed_mu(m, mu, "f64", opts=o, pad_to=32)
        ok = st["lb_est"] > 0
        feats.append(st["feat"][ok])
        ys.append(np.stack([np.log(st["rho_est"] / st["gersh"]),
                            np.log(st["lb_est"] * st["scale"] / st["gersh"])], 1)[ok])
    X = torch.from_numpy(np.concatenate(feats).astype(np.float32)).cuda()
    Y = torch.from_numpy(np.concatenate(ys).astype(np.float32)).cuda()
    net = sm.Mlp(seed=3)
    hist = sm.sm_mlp_train(net, X, Y, X.shape[0], epochs=300, batch=128, lr=2e-3)
    assert hist[-1] < 0.1 * hist[0]
    for t in (5, 6):
        m = synth.config5_step(t, n_mol=32, cutoff=1.5)
        plan = sm.Plan(m, 32)
        sm.sm_plan_set_mlp(plan, net)
        kw = dict(scaling=sm.SM_SCALE_LEARNED, power_steps=4, scale_margin=0.05)
        Pl, El, _, stl, _ = run_fixed_mu(m, mu, "f64", plan=plan, **kw)
        Pa, Ea, _, sta, _ = run_fixed_mu(m, mu, "f64", plan=plan, accel=1, **kw)
        Pg, Eg, _, stg, _ = run_fixed_mu(m, mu, "f64", plan=plan)
        print(f"step {t}: iterations Gershgorin {stg['iters'].mean():.2f}, learned scale "
              f"{stl['iters'].mean():.2f}, + learned l_0 {sta['iters'].mean():.2f}")
        assert np.mean(sta["scale_src"] == 2) > 0.7
        assert sta["iters"].mean() < stl["iters"].mean() - 1.0
        assert np.max(np.abs(Pa - Pg)) < 1e-9 and rel(Ea, Eg) < 1e-12


def _probe_vec(q, n):
    """The fixed +-1 probe vector q of the float64 checks (a counter hash of
    (q, row); the same definition as the device's)."""
    r = np.arange(n, dtype=np.uint64)
    M = np.uint64(0xFFFFFFFF)
    h = (r * np.uint64(0x9E3779B1) + np.uint64(q) * np.uint64(0x85EBCA77) + np.uint64(0x165667B1)) & M
    h ^= h >> np.uint64(15)
    h = (h * np.uint64(0x2C1B3C6D)) & M
    h ^= h >> np.uint64(12)
    h = (h * np.uint64(0x297A2D39)) & M
    h ^= h >> np.uint64(15)
    return np.where(h & np.uint64(1), 1.0, -1.0)


def test_commutator_probe(dev):
    """res_comm = max_v ||X T v - T X v|| / (c ||v||): recomputed on the CPU
    from the final float32 X in the workspace and the oracle's T; ordered by
    precision (float64 << split bf16 << bf16) like the subspace error."""
    import torch
    m, mu = _system()
    plan = sm.Plan(m, 64)
    H = torch.from_numpy(m.vals).cuda()
    o = sm.default_opts("f32", comm_probes=2)
    work = sm.Workspace(plan, sm.storage_prec(o), H.device)
    sm.build_submatrices(plan, 0, H, mu, o, work.ws, work.stats)
    sm.submatrix_sign(plan, 0, work.ws, o, work.stats)
    sm.sm_comm_probe(plan, 0, H, mu, o, work.ws, work.stats)
    torch.cuda.synchronize()
    st = work.stats_host()
    reg, off = plan.ws_layout(sm.SM_F32)
    mats = work.ws.cpu().numpy()[reg[0]:reg[1]].view(np.float32)
    info = plan.info()
    view = om.BlockView(m)
    for g in (0, 17, 40):
        i = info["order"][g]
        npad, n = info["npad"][i], info["n"][i]
        nn = npad * npad
        b = int(st["iters"][i]) & 1
        X = mats[off[g] + b * nn: off[g] + (b + 1) * nn].reshape(npad, npad).T[:n, :n].astype(np.float64)
        T = om.submatrix(view, i, mu)
        worst = 0.0
        for q in range(2):
            v = _probe_vec(100 + q, n)
            worst = max(worst, np.linalg.norm(X @ (T @ v) - T @ (X @ v)) / np.sqrt(n))
        ref = worst / st["scale"][i]
        assert abs(st["res_comm"][i] - ref) <= 1e-6 * ref + 1e-12, (i, st["res_comm"][i], ref)
    vals = {}
    for prec in ("f64", "bf16x3", "bf16"):
        P, E, Ne, st2, _ = run_fixed_mu(m, mu, prec, pad_to=64, comm_probes=2)
        vals[prec] = float(st2["res_comm"].max())
    print("max res_comm:", vals, "f32:", float(st["res_comm"].max()))
    assert vals["f64"] < 1e-12 < vals["bf16x3"] < 1e-4 < vals["bf16"]
    assert np.all(st["res_comm"] > 0)


FIRST_SQUARE = [("f64", 1e-9), ("f32", 1e-5), ("bf16x3", 1e-4), ("f16", 5e-3), ("bf16", 5e-2)]


@pytest.mark.parametrize("prec,dp_max", FIRST_SQUARE, ids=[c[0] for c in FIRST_SQUARE])
def test_first_square_bounds_the_first_step(prec, dp_max, dev):
    """Power scale (c near rho(T), far below c_G) with accel 1: the first
    square runs unscaled and the largest column sum of |X_0^2| bounds the top
    of the spectrum of X_0 the first update is scaled for (stats.top1).  That
    bound is rigorous (never below rho(T) / c from the oracle's eigenvalues of
    every submatrix), at most c_G / c and well below it; the run needs fewer
    updates than accel 2 (the first step scaled for c_G / c) and its P matches
    the oracle within the schedule's bar (bf16, whose main phase ends at its
    precision floor, needs no more updates); a graph replay gives the eager P.
    Cutoff 2.5 (submatrices up to 552 rows): c_G / c near 5, where the
    tighter first step saves an update."""
    m = synth.water_system(24, 2.5, 5)
    mu = gap_mu(m)
    view = om.BlockView(m)
    rho, lrel = np.empty(m.n_atoms), np.inf
    for i in range(m.n_atoms):
        T = om.submatrix(view, i, mu)
        lam = np.abs(np.linalg.eigvalsh(T))
        rho[i] = lam.max()
        lrel = min(lrel, lam.min() / om.gershgorin_bound(T))
    plan = sm.Plan(m, 64)
    kw = dict(scaling=sm.SM_SCALE_POWER, power_steps=20, scale_margin=0.02, lbound=0.8 * lrel, retry=0)
    P1, E1, _, st1, _ = run_fixed_mu(m, mu, prec, plan=plan, accel=1, **kw)
    P2, E2, _, st2, _ = run_fixed_mu(m, mu, prec, plan=plan, accel=2, **kw)
    top0 = st1["gersh"] / st1["scale"]
    top1 = st1["top1"].astype(np.float64)
    print(f"{prec}: top c_G/c {top0.mean():.2f} -> {top1.mean():.2f} (rho/c {np.mean(rho / st1['scale']):.3f}); "
          f"updates {st2['iters'].mean():.2f} -> {st1['iters'].mean():.2f}")
    assert np.all(top0 > 1.5) and np.all(st2["top1"] == 0)
    assert np.all(top1 >= (rho / st1["scale"]) * (1 - 1e-6))
    assert np.all(top1 <= top0 * (1 + 1e-6)) and top1.mean() < 0.7 * top0.mean()
    assert np.all(st1["status"] >= 1) and np.all(st2["status"] >= 1)
    if prec == "bf16":   # its main phase ends at the bf16 floor (stagnation), not by convergence
        assert st1["iters"].sum() <= st2["iters"].sum()
    else:
        assert st1["iters"].sum() < st2["iters"].sum()
    Po = om.density_matrix(m, mu)
    Eo, _ = om.energy_trace(m, Po)
    assert float(np.max(np.abs(P1 - Po))) < dp_max
    if prec in ("f64", "bf16x3"):
        assert rel(E1, Eo) < (1e-11 if prec == "f64" else 1e-5)
        Pg, Eg, _, _, _ = run_fixed_mu(m, mu, prec, plan=plan, accel=1, graph_iters=3, **kw)
        assert np.array_equal(Pg, P1) and Eg == E1
