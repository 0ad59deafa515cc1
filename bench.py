#!/usr/bin/env python3
"""Throughput of the submatrix-method density matrix on one MI355X.

One step = one pass of the whole hot path over the synthetic system: the
chemical potential by bisection on tr P (each midpoint a full gather, scaling,
batched Newton-Schulz sign and electron count on the GPU), P assembled at the
accepted mu, then tr(PH) and tr P in float64.  The symbolic plan (once per
sparsity pattern) and the input generation are outside the timed region; H is
resident in HBM when timing starts.

Workload (default): 10x10x10 lattice, 3% vacancies, jitter N(0, 0.05),
6 orbitals per atom (N = 5802, 967 submatrices of n = 192..276), cutoff 2.2,
mu by bisection to half filling.  Each precision schedule is timed; the plain
float64 path is the reference for the error of the others, and the headline
value is the fastest schedule within 1e-5 relative energy and 1e-4 max |dP| of
it.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

MODES = {"f64": "f64", "f32": "f32", "bf16x3": "bf16x3", "f16": "f16", "bf16": "bf16"}
DT_NAME = {0: "f64", 1: "f32", 2: "bf16", 3: "f16", 4: "bf16x3"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--modes", default="f64,f32,bf16x3")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="target CPU time of the oracle baseline sample (0 = skip)")
    ap.add_argument("--no-profile", action="store_true", help="skip the per-kernel event timing")
    return ap.parse_args()


def cpu_baseline(m, mu, target_s):
    """The oracle as it stands, on a bounded sample of the same workload:
    the submatrix P columns of the first k atoms, k sized to ~target_s."""
    from oracle import submatrix as om
    from threadpoolctl import threadpool_info
    view = om.BlockView(m)
    t0 = time.perf_counter()
    om.density_matrix(view, mu, atoms=range(32))
    per = (time.perf_counter() - t0) / 32
    k = int(min(m.n_atoms, max(64, target_s / max(per, 1e-6))))
    t0 = time.perf_counter()
    om.density_matrix(view, mu, atoms=range(k))
    dt = time.perf_counter() - t0
    threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
    return {"value": k / dt, "unit": "submatrices/s", "cores": int(threads), "kind": "oracle",
            "sample": f"float64 eigendecomposition oracle, P columns of the first {k} of "
                      f"{m.n_atoms} submatrices at the benchmark's mu ({dt:.1f} s)"}


def main():
    a = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if a.gpus != 1 or world != 1:
        print("bench.py: this build runs on one GPU only (the submatrix path shards by atom "
              "domains; the multi-GPU exchange is not built). Use --gpus 1.", file=sys.stderr)
        sys.exit(2)
    import torch
    import synth
    from paper_2205_14741_amd import smsign as sm
    from paper_2205_14741_amd import metrics

    dev = torch.device("cuda:0")
    m = synth.config2(a.seed)
    # float64 / float32 schedules pad submatrices to 32, the bf16-family ones to 64
    plans = {32: sm.Plan(m, 32), 64: sm.Plan(m, 64)}
    H = torch.from_numpy(m.vals).to(dev)
    torch.cuda.synchronize()

    modes = [x for x in a.modes.split(",") if x]
    if "f64" not in modes:
        modes = ["f64"] + modes
    res = {}
    ref_P = ref_E = None
    for mode in modes:
        o = sm.default_opts(MODES[mode])
        plan = plans[32 if mode in ("f64", "f32") else 64]
        info = plan.info()
        n, npad = info["n"], info["npad"]
        work = sm.Workspace(plan, sm.storage_prec(o), dev)
        # the autotuner picks the GEMM kernel variant for this schedule (untimed)
        lo, hi = sm.sm_gershgorin_bracket(plan, H)
        best, tune_ms = sm.sm_autotune(plan, 0, H, 0.5 * (lo + hi), o, work.ws, work.stats, repeats=2)

        def step():
            mu, k, _ = sm.sm_find_mu(plan, H, m.n_occ, o, work.ws, work.stats, P=work.P)
            E, Ne = sm.energy_trace(plan, H, work.P)
            return mu, k, E, Ne

        for _ in range(a.warmup):
            step()
        prof = not a.no_profile
        if prof:
            sm.sm_profile_read(plan)
            sm.sm_profile_enable(plan, True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(a.steps):
            mu, k, E, Ne = step()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        if prof:
            sm.sm_profile_enable(plan, False)
            launches, ms = sm.sm_profile_read(plan)
        st = work.stats_host()
        fl = metrics.flops_by_class(st, n, npad, o)
        useful = sum(v[0] for v in fl.values())
        P = work.P.cpu().numpy()
        r = {"ms_per_step": dt / a.steps * 1e3, "pad_to": 32 if mode in ("f64", "f32") else 64, "mu": mu, "bisection_passes": k, "E": E, "Ne": Ne,
             "iters": [int(st["iters"].min()), int(st["iters"].max())],
             "iters_mean": float(st["iters"].mean()),
             "submatrices_per_s": m.n_atoms * a.steps / dt,
             "useful_tflops": useful * k * a.steps / dt / 1e12,
             "status_ok": bool(np.all(st["status"] >= 1)),
             "probe_max": float(st["res_probe"].max()),
             "gemm_variant": int(best), "autotune_sign_ms": [float(x) for x in tune_ms]}
        if prof:
            # dominant GEMM class of this schedule: most kernel time
            cls = int(np.argmax(ms))
            key = (cls // 2, cls % 2)
            fu, fi = fl.get(key, (0.0, 0.0))
            passes = k * a.steps
            avg_ms = ms[cls] / max(launches[cls], 1)
            per_launch = fu * passes / max(launches[cls], 1)
            r["kernel"] = {"name": f"ns_gemm_kernel<{DT_NAME[key[0]]},{'square' if key[1] == 0 else 'update'}>",
                           "launches": int(launches[cls]), "avg_ms": avg_ms,
                           "useful_flops_per_launch": per_launch,
                           "issued_flops_per_launch": fi * passes / max(launches[cls], 1),
                           "achieved_tflops": per_launch / (avg_ms * 1e-3) / 1e12,
                           "gemm_ms_total_per_step": float(ms.sum()) / a.steps,
                           "peak_tflops": metrics.PEAK_TFLOPS[key[0]]}
        if mode == "f64":
            ref_P, ref_E = P, E
            r["rel_dE_vs_f64"] = 0.0
            r["max_dP_vs_f64"] = 0.0
        else:
            r["rel_dE_vs_f64"] = abs(E - ref_E) / abs(ref_E)
            r["max_dP_vs_f64"] = float(np.max(np.abs(P - ref_P)))
        r["meets_target"] = r["rel_dE_vs_f64"] <= 1e-5 and r["max_dP_vs_f64"] <= 1e-4 and r["status_ok"]
        res[mode] = r
        print(f"# {mode}: {r['ms_per_step']:.2f} ms/step, {r['submatrices_per_s']:.0f} subm/s, "
              f"{r['useful_tflops']:.2f} TF/s useful, iters {r['iters']}, dE {r['rel_dE_vs_f64']:.2e}, "
              f"dP {r['max_dP_vs_f64']:.2e}, variant {best} (tune ms {' / '.join(f'{x:.2f}' for x in tune_ms)})"
              + (f", {r['kernel']['name']} {r['kernel']['achieved_tflops']:.2f} TF/s" if prof else ""),
              file=sys.stderr, flush=True)
        del work

    ok = [k for k in res if res[k]["meets_target"]]
    head = max(ok, key=lambda k: res[k]["submatrices_per_s"]) if ok else "f64"
    h = res[head]
    out = {
        "metric": "submatrix-sign TFLOP/s & submatrices/s vs FP64 plain at 1e-5 rel energy",
        "value": h["submatrices_per_s"],
        "unit": "submatrices/s",
        "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": h["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DT_NAME[sm.default_opts(MODES[head]).phase1] + ("+f32" if head in ("bf16x3", "f16", "bf16") else ""),
        "data": "synthetic",
        "config": {"workload": "lattice1000: 10x10x10 lattice, 3% vacancies, jitter 0.05, 6 orbitals "
                               "(N=5802), cutoff 2.2, 967 submatrices n=192..276, mu by bisection",
                   "n_sub": m.n_atoms, "N": m.n_orb, "mode": head, "seed": a.seed},
        "useful_tflops": h["useful_tflops"],
        "speedup_vs_fp64_plain": res["f64"]["ms_per_step"] / h["ms_per_step"],
        "modes": res,
    }
    if "kernel" in h:
        kk = h["kernel"]
        out["roofline"] = {"bound": "mfma", "achieved": kk["achieved_tflops"], "peak": kk["peak_tflops"],
                           "unit": "TFLOP/s", "frac": kk["achieved_tflops"] / kk["peak_tflops"],
                           "traffic": None, "kernel": kk["name"]}
    if a.cpu_seconds > 0:
        out["cpu_baseline"] = cpu_baseline(m, res["f64"]["mu"], a.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
