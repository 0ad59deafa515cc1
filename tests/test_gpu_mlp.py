"""The scaling network on the GPU against the float64 numpy oracle: inference,
full-batch gradients (relative 1e-4), one Adam step, and training progress;
then learned scaling inside the method: guard, fallback, and unchanged P."""
import numpy as np
import pytest

import synth
from oracle import mlp as omlp
from oracle import submatrix as om
from paper_2205_14741_amd import smsign as sm
from gpu_helpers import gap_mu, h_dev, rel

pytestmark = pytest.mark.gpu


def _data(seed, n):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(n, 16)).astype(np.float32)
    T = np.stack([np.tanh(X[:, 0]) - 0.3 * X[:, 1], 0.2 * X[:, 2] * X[:, 3]], 1).astype(np.float32)
    return X, T


def _dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def test_inference_matches_oracle(dev):
    X, _ = _data(0, 1000)
    net = sm.Mlp(seed=3)
    th = omlp.init_params(7).astype(np.float32)
    norm = np.concatenate([X.mean(0), X.std(0)]).astype(np.float32)
    net.set_weights(th, norm)
    Y = sm.sm_mlp_infer(net, _dev(X), len(X)).cpu().numpy()
    xn = (X.astype(np.float64) - norm[:16]) / norm[16:]
    Yo, _ = omlp.forward(th.astype(np.float64), xn)
    np.testing.assert_allclose(Y, Yo, rtol=1e-4, atol=1e-5)


@pytest.mark.parametrize("n", [1, 37, 1000])
def test_gradient_matches_oracle(n, dev):
    X, T = _data(1, n)
    net = sm.Mlp(seed=3)
    th = omlp.init_params(2).astype(np.float32)
    net.set_weights(th, np.concatenate([np.zeros(16), np.ones(16)]).astype(np.float32))
    loss, g = sm.sm_mlp_loss_grad(net, _dev(X), _dev(T), n)
    lo, go = omlp.grad(th.astype(np.float64), X.astype(np.float64), T.astype(np.float64))
    assert rel(loss, lo) < 1e-5
    scale = np.abs(go).max()
    np.testing.assert_allclose(g, go, rtol=1e-4, atol=1e-5 * scale)


def test_one_adam_step_matches_oracle(dev):
    n = 64
    X, T = _data(2, n)
    net = sm.Mlp(seed=3)
    th = omlp.init_params(4).astype(np.float32)
    norm = np.concatenate([np.zeros(16), np.ones(16)]).astype(np.float32)
    net.set_weights(th, norm)
    sm.sm_mlp_train(net, _dev(X), _dev(T), n, epochs=1, batch=n, lr=1e-3, fit_norm=False, shuffle_seed=0)
    th1, _ = net.get_weights()
    _, go = omlp.grad(th.astype(np.float64), X.astype(np.float64), T.astype(np.float64))
    tho, _, _ = omlp.adam_step(th.astype(np.float64), go, np.zeros_like(go), np.zeros_like(go), 1, 1e-3)
    # first step moves by -lr sign(g) except where g is ~0: compare where |g| is not tiny
    big = np.abs(go) > 1e-3 * np.abs(go).max()
    np.testing.assert_allclose(th1[big], tho[big], atol=1e-6)


def test_training_reduces_loss_and_is_deterministic(dev):
    n = 4000
    X, T = _data(5, n)
    Xd, Td = _dev(X), _dev(T)
    hists = []
    for _ in range(2):
        net = sm.Mlp(seed=11)
        hists.append(sm.sm_mlp_train(net, Xd, Td, n, epochs=40, batch=512, lr=3e-3, shuffle_seed=9))
    np.testing.assert_array_equal(hists[0], hists[1])
    assert hists[0][-1] < 0.1 * hists[0][0]


def test_learned_scaling_guard_and_fallback(dev):
    """A network that predicts log(rho/c_G) well is accepted and cuts
    iterations; a corrupted one is rejected by the guard (Gershgorin
    fallback); P agrees with the oracle either way."""
    import torch
    m = synth.water_system(24, 1.4, 5)
    mu = gap_mu(m)
    plan = sm.Plan(m, 64)
    H = h_dev(m)
    base = sm.default_opts("f64")
    work = sm.Workspace(plan, sm.SM_F64, H.device)
    # labels the method generates: long power iteration
    o_pow = sm.default_opts("f64", scaling=sm.SM_SCALE_POWER, power_steps=40, scale_margin=0.02)
    sm.sm_density_matrix(plan, H, mu, o_pow, work.ws, work.P, work.stats)
    st = work.stats_host()
    feats = np.ascontiguousarray(st["feat"], dtype=np.float32)
    y = np.stack([np.log(st["rho_est"] / st["gersh"]), np.zeros(len(st))], 1).astype(np.float32)
    net = sm.Mlp(seed=1)
    sm.sm_mlp_train(net, _dev(feats), _dev(y), len(y), epochs=400, batch=len(y), lr=3e-3)
    sm.sm_plan_set_mlp(plan, net)
    o_l = sm.default_opts("f64", scaling=sm.SM_SCALE_LEARNED, power_steps=4, scale_margin=0.05)
    E_l, _ = sm.sm_density_matrix(plan, H, mu, o_l, work.ws, work.P, work.stats)
    st_l = work.stats_host()
    P_l = work.P.cpu().numpy()
    E_g, _ = sm.sm_density_matrix(plan, H, mu, base, work.ws, work.P, work.stats)
    st_g = work.stats_host()
    accepted = np.mean(st_l["scale_src"] == 2)
    print(f"accepted {accepted:.2f}, iters learned {st_l['iters'].mean():.2f} vs gershgorin {st_g['iters'].mean():.2f}")
    assert accepted > 0.8
    assert st_l["iters"].mean() < st_g["iters"].mean() - 1.0
    Po = om.density_matrix(m, mu)
    assert np.nanmax(np.abs(P_l - Po)) < 1e-9 and rel(E_l, E_g) < 1e-11
    # corrupted network: predicts tiny scales -> rejected everywhere
    p, q = net.get_weights()
    p[-2:] = -20.0
    net.set_weights(p, q)
    sm.sm_density_matrix(plan, H, mu, o_l, work.ws, work.P, work.stats)
    st_c = work.stats_host()
    assert np.all(st_c["scale_src"] == 3)
    np.testing.assert_array_equal(st_c["scale"], st_g["scale"])
    assert np.nanmax(np.abs(work.P.cpu().numpy() - Po)) < 1e-9


def test_scaling_pairs_from_records(dev):
    """The training pairs the library builds from the records of an explicit
    pass (power scale, plain Newton-Schulz) are the records with both bounds,
    in record order: features copied, targets log(rho_est / c_G) and
    log(lb_est c / c_G) (float32 of the float64 values)."""
    import torch
    m = synth.water_system(16, 1.5, 3)
    lam = np.linalg.eigvalsh(synth.to_dense(m))
    mu = 0.5 * (lam[m.n_occ - 1] + lam[m.n_occ])
    o = sm.default_opts("f64", scaling=sm.SM_SCALE_POWER, power_steps=40, scale_margin=0.02)
    plan = sm.Plan(m, 64)
    H = torch.from_numpy(m.vals).to(dev)
    work = sm.Workspace(plan, sm.storage_prec(o), dev)
    sm.sm_density_matrix(plan, H, mu, o, work.ws, work.P, work.stats)
    st = work.stats_host()
    X, T = sm.sm_scaling_pairs(work.stats, m.n_atoms)
    ok = (st["rho_est"] > 0) & (st["lb_est"] > 0) & (st["gersh"] > 0)
    assert ok.sum() > m.n_atoms // 2 and X.shape[0] == ok.sum()
    np.testing.assert_array_equal(X.cpu().numpy(), st["feat"][ok])
    want = np.stack([np.log(st["rho_est"] / st["gersh"]), np.log(st["lb_est"] * st["scale"] / st["gersh"])], 1)[ok]
    np.testing.assert_allclose(T.cpu().numpy(), want, rtol=1e-6, atol=1e-6)
