"""Helpers for the GPU tests: run the HIP path through the C ABI on seeded
systems and compare with the oracle."""
import numpy as np

from paper_2205_14741_amd import smsign as sm


def h_dev(m, device="cuda:0"):
    import torch
    return torch.from_numpy(np.ascontiguousarray(m.vals)).to(device)


def run_fixed_mu(m, mu, prec="f64", pad_to=64, max_chunk_elems=0, opts=None, plan=None, **kw):
    import torch
    plan = plan or sm.Plan(m, pad_to, max_chunk_elems)
    o = opts or sm.default_opts(prec, **kw)
    H = h_dev(m)
    work = sm.Workspace(plan, sm.storage_prec(o), H.device)
    E, Ne = sm.sm_density_matrix(plan, H, mu, o, work.ws, work.P, work.stats)
    torch.cuda.synchronize()
    return work.P.cpu().numpy(), E, Ne, work.stats_host(), plan


def gap_mu(m):
    from synth import to_dense
    lam = np.linalg.eigvalsh(to_dense(m))
    return 0.5 * (lam[m.n_occ - 1] + lam[m.n_occ])


def rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)
