"""The processing order from atom positions and the GEMM variants per chunk
size class, on the GPU through the C ABI: the order changes which workgroup
computes what, never a result; the autotuner's choice reaches exactly the
chunks of the tuned chunk's size class."""
import numpy as np
import pytest

import synth
from paper_2205_14741_amd import smsign as sm
from gpu_helpers import gap_mu, h_dev, run_fixed_mu

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("prec", ["f64", "bf16x3"])
def test_positions_order_changes_no_result(prec, dev):
    """Index order against Morton order of the atom centres (and size buckets):
    P, tr(PH) and tr P are bitwise the same, every submatrix's iteration count
    too (each submatrix's arithmetic does not depend on where it is processed;
    the reductions run in atom order)."""
    m = synth.water_system(32, 1.5, 1)
    mu = gap_mu(m)
    budget = 3 * 320 * 320 * 12
    runs = []
    for bucket in (None, 0, 128):
        plan = sm.Plan(m, 64, budget)
        if bucket is not None:
            plan.set_positions(m.positions, bucket_rows=bucket)
        P, E, Ne, st, _ = run_fixed_mu(m, mu, prec, plan=plan)
        runs.append((P, E, Ne, st["iters"].copy(), plan.info()["order"], plan.n_chunks))
    assert runs[0][5] > 2
    assert not np.array_equal(runs[0][4], runs[1][4])
    for P, E, Ne, it, _, _ in runs[1:]:
        assert np.array_equal(P, runs[0][0])
        assert E == runs[0][1] and Ne == runs[0][2]
        assert np.array_equal(it, runs[0][3])


def test_autotune_sets_its_size_class_only(dev):
    """A batch of two water-like systems in separate chunks of two size
    classes: tuning a chunk of the first class (here restricted to variant 4)
    changes that class's variant and the plan-wide one, not the other class's;
    sm_plan_tuning's set reaches every class; the results stay within the
    split-bf16 accuracy of the float64 path."""
    import torch
    a, b = synth.water_system(16, 1.5, 3), synth.water_system(24, 2.6, 4)
    u = synth.union([a, b])
    probe = sm.Plan(u, 64)
    need = int(np.sum(3 * probe.info()["npad"][:a.n_atoms].astype(np.int64) ** 2))
    plan = sm.Plan(u, 64, need)            # the first system fills chunk 0 exactly
    cls0, v0 = plan.chunk_variants(0)
    cls1, v1 = plan.chunk_variants(1)
    assert cls0 != cls1
    H = h_dev(u)
    mu = gap_mu(u)
    o = sm.default_opts("bf16x3")
    w = sm.Workspace(plan, sm.storage_prec(o), H.device)
    best, times = sm.sm_autotune(plan, 0, H, mu, o, w.ws, w.stats, repeats=1, variants=(4,))
    torch.cuda.synchronize()
    assert best == 4
    # the float32 refinement keeps its own choice (slab products, see the header)
    assert plan.chunk_variants(0)[1][sm.SM_BF16X3] == 4 and plan.chunk_variants(0)[1][sm.SM_F32] == v0[sm.SM_F32]
    assert plan.chunk_variants(1)[1] == v1
    assert int(sm.sm_plan_tuning(plan)[sm.SM_BF16X3]) == 4
    E, Ne = sm.sm_density_matrix(plan, H, mu, o, w.ws, w.P, w.stats)
    torch.cuda.synchronize()
    P = w.P.cpu().numpy()
    P64, E64, _, _, _ = run_fixed_mu(u, mu, "f64", pad_to=64)
    assert float(np.max(np.abs(P - P64))) < 1e-4 and abs(E - E64) < 1e-5 * abs(E64)
    table = [1, 1, 2, 2, 2]
    sm.sm_plan_tuning(plan, table)
    for c in range(plan.n_chunks):
        assert plan.chunk_variants(c)[1] == table


def test_synchronized_rounds_on_two_streams_at_once(dev):
    """Two plans, each with its own workspace (and so its own round counters
    of the synchronized 256-wide kernel), run their sign passes at the same
    time from two host threads on two streams: both results equal the ones
    each gives alone, bit for bit (the round barriers order only time)."""
    import threading
    import torch
    m = synth.water_system(48, 2.2, 5)       # n_pad up to 1024: the 256-wide tiles
    mu = gap_mu(m)
    o = sm.default_opts("bf16x3", variant=8)
    H = h_dev(m)
    runs = []
    for _ in range(2):
        plan = sm.Plan(m, 64)
        w = sm.Workspace(plan, sm.storage_prec(o), H.device)
        runs.append((plan, w, torch.cuda.Stream()))
    torch.cuda.synchronize()   # H's upload (current stream) before the other streams read it
    alone = []
    for plan, w, st in runs:
        sm.sm_density_matrix(plan, H, mu, o, w.ws, w.P, w.stats, stream=st)
        torch.cuda.synchronize()
        alone.append(w.P.cpu().numpy().copy())
    errors = []

    def work(plan, w, st):
        try:
            for _ in range(2):
                sm.sm_density_matrix(plan, H, mu, o, w.ws, w.P, w.stats, stream=st)
        except Exception as e:   # reported below
            errors.append(e)

    ts = [threading.Thread(target=work, args=r) for r in runs]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    torch.cuda.synchronize()
    assert not errors, errors
    for (plan, w, st), P0 in zip(runs, alone):
        assert np.array_equal(w.P.cpu().numpy(), P0)
