"""The batching, precision and learned-scaling forms of the path on the GPU.

* graph replay == eager launches, bitwise, over repeated calls;
* several independent systems in one batch (block-diagonal union, one plan,
  one set of launches) == each system on its own;
* large uneven water submatrices through a chunked workspace, P columns
  checked against the oracle on sampled atoms;
* a trajectory: the scaling network trained on the bounds of early steps cuts
  iterations on later steps with P unchanged.
"""
import numpy as np
import pytest

import synth
from oracle import submatrix as om
from paper_2205_14741_amd import smsign as sm
from gpu_helpers import gap_mu, h_dev, rel, run_fixed_mu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["f64", "bf16x3"])
def test_graph_replay_equals_eager(prec, dev):
    m = synth.water_system(24, 1.4, 5)
    mu = gap_mu(m)
    pad = 32 if prec == "f64" else 64
    P0, E0, N0, st0, plan = run_fixed_mu(m, mu, prec, pad_to=pad)
    for G in (1, 3, 4):
        for rep in range(3):   # repeated replays of the cached graph
            P, E, Ne, st, _ = run_fixed_mu(m, mu, prec, plan=plan, graph_iters=G)
            np.testing.assert_array_equal(P, P0)
            assert E == E0 and Ne == N0
            np.testing.assert_array_equal(st["iters"], st0["iters"])


def test_batch_of_systems_equals_separate(dev):
    """Four independent water systems of different sizes and cutoffs in one
    plan (uneven submatrices, one launch per GEMM phase for all of them)."""
    import torch
    parts = [synth.water_system(nm, rc, [7, k]) for k, (nm, rc) in
             enumerate(((8, 1.2), (12, 1.3), (16, 1.4), (24, 1.45)))]
    u = synth.union(parts)
    mu = -2.7   # inside every part's gap (between -4.4 and -1.04)
    o = sm.default_opts("bf16x3", graph_iters=4)
    Pu, Eu, Nu, stu, plan = run_fixed_mu(u, mu, "bf16x3", opts=o)
    info = plan.info()
    assert info["n"].max() > 2 * info["n"].min()
    off = 0
    Es = []
    for part in parts:
        P, E, Ne, st, _ = run_fixed_mu(part, mu, "bf16x3", opts=o)
        np.testing.assert_array_equal(Pu[off:off + P.shape[0]], P)
        off += P.shape[0]
        Es.append(E)
    assert abs(Eu - sum(Es)) < 1e-9 * abs(Eu)
    assert off == Pu.shape[0]


@pytest.mark.parametrize("prec,dp_max", [("f32", 1e-5), ("bf16x3", 1e-4)])
def test_large_water_chunked_sampled(prec, dp_max, dev):
    """Water-like system with submatrices of n ~ 1000-1300 processed through a
    workspace of a few chunks; sampled P columns against the oracle."""
    m = synth.water_system(128, 2.2, 11)
    mu = -2.95  # gap of this system: [-4.23, -1.68]
    plan = sm.Plan(m, 64, max_chunk_elems=3 * 1344 * 1344 * 40)
    assert plan.n_chunks >= 3
    P, E, Ne, st, _ = run_fixed_mu(m, mu, prec, plan=plan, graph_iters=4)
    info = plan.info()
    assert info["n"].min() > 700
    atoms = [0, 1, 2, 77, 200, 383]
    Po = om.density_matrix(m, mu, atoms=atoms)
    mask = ~np.isnan(Po)
    dP = np.max(np.abs(P[mask] - Po[mask]))
    print(f"{prec}: n {info['n'].min()}-{info['n'].max()}, chunks {plan.n_chunks}, "
          f"max|dP| on {len(atoms)} sampled atoms {dP:.2e}, iters {st['iters'].min()}-{st['iters'].max()}")
    assert dP < dp_max
    assert np.all(st["status"] >= 1)


MU5 = -2.85   # gap of the 32-molecule walk at step 0: [-4.44, -1.27]


def test_trajectory_learned_scaling(dev):
    """Train on the power-iteration bounds of steps 0-2 of a random walk,
    apply to steps 5 and 6: most predictions accepted, fewer iterations than
    Gershgorin scaling, P within 1e-9 of the float64 Gershgorin run."""
    import torch
    steps_train, steps_test = (0, 1, 2), (5, 6)
    feats, ys = [], []
    for t in steps_train:
        m = synth.config5_step(t, n_mol=32, cutoff=1.5)
        o = sm.default_opts("f64", scaling=sm.SM_SCALE_POWER, power_steps=40, scale_margin=0.02)
        _, _, _, st, _ = run_fixed_mu(m, MU5, "f64", opts=o, pad_to=32)
        feats.append(st["feat"])
        ys.append(np.stack([np.log(st["rho_est"] / st["gersh"]),
                            np.log(st["lb_est"] * st["scale"] / st["gersh"])], 1))
    X = torch.from_numpy(np.concatenate(feats).astype(np.float32)).cuda()
    Y = torch.from_numpy(np.concatenate(ys).astype(np.float32)).cuda()
    net = sm.Mlp(seed=2)
    hist = sm.sm_mlp_train(net, X, Y, X.shape[0], epochs=300, batch=128, lr=2e-3)
    assert hist[-1] < 0.1 * hist[0]
    for t in steps_test:
        m = synth.config5_step(t, n_mol=32, cutoff=1.5)
        plan = sm.Plan(m, 32)
        sm.sm_plan_set_mlp(plan, net)
        ol = sm.default_opts("f64", scaling=sm.SM_SCALE_LEARNED, power_steps=4, scale_margin=0.05)
        Pl, El, _, stl, _ = run_fixed_mu(m, MU5, "f64", opts=ol, plan=plan)
        Pg, Eg, _, stg, _ = run_fixed_mu(m, MU5, "f64", plan=plan)
        acc = np.mean(stl["scale_src"] == 2)
        print(f"step {t}: accepted {acc:.2f}, iters learned {stl['iters'].mean():.2f} "
              f"vs Gershgorin {stg['iters'].mean():.2f}")
        assert acc > 0.7
        assert stl["iters"].mean() < stg["iters"].mean() - 1.0
        assert np.max(np.abs(Pl - Pg)) < 1e-9 and rel(El, Eg) < 1e-12
