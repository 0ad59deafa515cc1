"""Flop accounting of the Newton-Schulz passes from the per-submatrix records.

A pass over submatrix i of size n (padded to np) runs, per precision phase,
some squares (A = X^2, Y = 3I - A) and updates (X' = 1/2 X Y).  Every product
is symmetric, so the kernels compute the tiles on and below the diagonal only:

    useful flops of one product  = n^2 (n + 1)       (n(n+1)/2 entries x 2n)
    issued MFMA flops            = (32 x 32 wave blocks computed) * 2 * 32 * 32 * np
                                   (the blocks on or below the diagonal inside n_pad)

With a refinement phase of r steps (status 2) the counts are
    main precision:   squares = iters_low + 1, updates = iters_low (+ 1)
    refinement:       squares = r - 1,         updates = r (- 1)
and without one (status 0 / 1): squares = iters + 1, updates = iters.  The
(+ 1 / - 1): after a 16-bit main phase the first refinement update multiplies
the main phase's operand copies and runs on the main-precision kernel.
"""
from __future__ import annotations

import numpy as np

PEAK_TFLOPS = {0: 78.6, 1: 157.3, 2: 2500.0, 3: 2500.0, 4: 2500.0}   # MI355X dense matrix peaks


def product_counts(stats: np.ndarray, opts) -> dict:
    """{(precision, kind): per-submatrix product counts}; kind 0 square, 1 update."""
    iters = stats["iters"].astype(np.int64)
    low = stats["iters_low"].astype(np.int64)
    r = int(opts.refine_steps)
    refined = (stats["status"] == 2)
    out = {}
    first_on_main = np.where(refined & (int(opts.phase1) >= 2), 1, 0)
    main_sq = np.where(refined, low + 1, iters + 1)
    main_up = np.where(refined, low, iters) + first_on_main
    out[(int(opts.phase1), 0)] = main_sq
    out[(int(opts.phase1), 1)] = main_up
    if r > 0:
        ref_all = np.where(refined, iters - low, 0)
        ref_up = ref_all - first_on_main
        ref_sq = np.where(refined, np.maximum(ref_all - 1, 0), 0)
        key_sq = (int(opts.refine), 0)
        key_up = (int(opts.refine), 1)
        out[key_sq] = out.get(key_sq, 0) + ref_sq
        out[key_up] = out.get(key_up, 0) + ref_up
    return out


def flops_by_class(stats: np.ndarray, n: np.ndarray, npad: np.ndarray, opts):
    """{(precision, kind): (useful flops, issued MFMA flops)} of one pass."""
    n = n.astype(np.float64)
    useful_one = n * n * (n + 1.0)
    issued_one = wave_blocks(npad) * 2.0 * 32 * 32 * npad.astype(np.float64)
    res = {}
    for key, cnt in product_counts(stats, opts).items():
        cnt = np.asarray(cnt, dtype=np.float64)
        res[key] = (float((cnt * useful_one).sum()), float((cnt * issued_one).sum()))
    return res


def wave_blocks(npad: np.ndarray) -> np.ndarray:
    """32 x 32 wave blocks computed per product by the 64-tile kernels: the
    blocks on or below the diagonal inside n_pad (tiles with bi >= bj; a
    diagonal tile skips its block above the diagonal, an edge tile the blocks
    past n_pad), i.e. nb (nb + 1) / 2 with nb = n_pad / 32."""
    nb = np.asarray(npad, dtype=np.int64) // 32
    return (nb * (nb + 1) // 2).astype(np.float64)


def useful_flops(stats, n, npad, opts) -> float:
    return sum(v[0] for v in flops_by_class(stats, n, npad, opts).values())


# Matrix-core products one product of the schedule costs: the split-bfloat16
# form computes hi*hi + hi*lo + lo*hi, three bfloat16 products per product.
MFMA_PRODUCTS = {0: 1, 1: 1, 2: 1, 3: 1, 4: 3}


def gemm_kernel_symbol(mode: int, which: int, variant: int, pad_to: int) -> str:
    """Demangled name prefix (as profilers print it) of the GEMM kernel that
    runs for (precision, square/update, kernel variant) on a plan with the
    given padding; mirrors the variant fallback of the launcher."""
    v = variant
    if v >= 3 and (mode == 0 or pad_to < 64):
        v = 1
    if mode >= 2 and pad_to < 64:   # 16-bit products on a plan padded to 32
        v = 2
    if v >= 3:   # 128-wide tiles: <precision, kind, XCD-aware walk, prefetch depth>
        return f"sm::ns_gemm128_kernel<{mode}, {which}, {'false' if v == 4 else 'true'}, {6 if v == 5 else 1}>"
    kdiv = 2 if v == 2 else 1   # variant 2: half-depth LDS stages
    return f"sm::ns_gemm_kernel<{mode}, {which}, {kdiv}, {'true' if v >= 1 else 'false'}>"


# Bytes per stored element of a product's operands and result: float64 and
# float32 iterates, 16-bit copies for bf16 / f16, hi + lo copies for split bf16.
STORE_BYTES = {0: 8, 1: 4, 2: 2, 3: 2, 4: 4}
HBM_PEAK_GBS = 8000.0   # MI355X HBM3E


def bytes_by_class(stats: np.ndarray, n: np.ndarray, opts) -> dict:
    """{(precision, kind): algorithmic memory bytes of one pass}: a square
    reads X and writes Y, an update reads X and Y and writes X', each an
    n x n matrix in the storage of that precision's products."""
    n2 = n.astype(np.float64) ** 2
    res = {}
    for (prec, kind), cnt in product_counts(stats, opts).items():
        per = (2.0 if kind == 0 else 3.0) * STORE_BYTES[prec] * n2
        res[(prec, kind)] = float((np.asarray(cnt, dtype=np.float64) * per).sum())
    return res
