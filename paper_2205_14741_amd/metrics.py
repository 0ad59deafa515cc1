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

The last refinement update of a status-2 submatrix computes only the tile
columns that hold the atom's own b columns (the ones P takes), all tile rows
and no mirror, where that slab has fewer tiles than the triangle and the
update is not the one that runs on the main-precision kernel:

    useful flops of a slab update = 2 n^2 b            (n b entries x 2n)
    issued MFMA flops             = (n_pad / 32) * (32-wide columns of the wave
                                    blocks that hold atom columns) * 2 * 32 * 32 * np
                                    (wave blocks are half a tile wide: 32 or 64)

With two or more refinement steps the square before that update (a
refinement square) computes the same slab of Y, which is all the update
reads: counted the same way, with bytes s (n^2 + n b).
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


def effective_variant(mode: int, variant: int, pad_to: int) -> int:
    """The GEMM kernel variant the launcher runs for a precision: no 128-wide
    tiles in float64 or on a plan padded to 32, and 16-bit products on a plan
    padded to 32 take the half-depth-stage kernel."""
    v = variant
    if v >= 6 and mode < 2:      # 256-wide tiles: 16-bit operand copies only
        v = 5
    if v >= 3 and (mode == 0 or pad_to < 64):
        v = 1
    if mode >= 2 and pad_to < 64:
        v = 2
    return v


def tile_shift(mode: int, variant: int, pad_to: int) -> int:
    """log2 of the output tile width of that kernel (64, 128 or 256)."""
    v = effective_variant(mode, variant, pad_to)
    if v >= 6:
        return 8
    return 7 if v >= 3 and mode != 0 else 6


def slab_tiles(npad, loc, b, tshift):
    """Tiles of a last-update slab: every tile row times the tile columns
    that hold columns loc .. loc + b - 1."""
    npad, loc, b = (np.asarray(x, dtype=np.int64) for x in (npad, loc, b))
    T = (npad + (1 << tshift) - 1) >> tshift
    return T * (((loc + b - 1) >> tshift) - (loc >> tshift) + 1)


def slab_mask(stats: np.ndarray, npad, loc, b, opts, tshift_ref: int) -> np.ndarray:
    """Submatrices whose last refinement update ran as a column slab (the
    scheduler's rule: status 2, not the update that runs on the main-precision
    kernel, fewer slab tiles than triangle tiles)."""
    npad = np.asarray(npad, dtype=np.int64)
    first_on_main = int(opts.phase1) >= 2 and int(opts.refine_steps) == 1
    T = (npad + (1 << tshift_ref) - 1) >> tshift_ref
    fewer = slab_tiles(npad, loc, b, tshift_ref) < T * (T + 1) // 2
    return (stats["status"] == 2) & fewer & (not first_on_main) & (int(opts.refine_steps) > 0)


def slab_columns32(npad, loc, b, tshift):
    """32-wide columns of the wave blocks a slab computes: the wave blocks
    (half a tile wide) that hold any of columns loc .. loc + b - 1."""
    npad, loc, b = (np.asarray(x, dtype=np.int64) for x in (npad, loc, b))
    ws = tshift - 1                     # log2 of the wave-block width
    c0 = (loc >> ws) << ws
    c1 = np.minimum((((loc + b - 1) >> ws) + 1) << ws, npad)
    return (c1 - c0) // 32


def flops_by_class(stats: np.ndarray, n: np.ndarray, npad: np.ndarray, opts, slab=None):
    """{(precision, kind): (useful flops, issued MFMA flops)} of one pass.
    slab: (loc, b, tshift_ref) of the plan, to count last updates that ran as
    column slabs at their own cost (None: every update counted in full)."""
    nf = n.astype(np.float64)
    useful_one = nf * nf * (nf + 1.0)
    issued_one = wave_blocks(npad) * 2.0 * 32 * 32 * npad.astype(np.float64)
    res = {}
    for key, cnt in product_counts(stats, opts).items():
        cnt = np.asarray(cnt, dtype=np.float64)
        res[key] = [float((cnt * useful_one).sum()), float((cnt * issued_one).sum())]
    if slab is not None and int(opts.refine_steps) > 0:
        loc, b, tsh = slab
        msk = slab_mask(stats, npad, loc, b, opts, tsh)
        key = (int(opts.refine), 1)
        useful_slab = 2.0 * nf * nf * np.asarray(b, dtype=np.float64)
        issued_slab = ((npad // 32).astype(np.float64) * slab_columns32(npad, loc, b, tsh)
                       * 2.0 * 32 * 32 * npad.astype(np.float64))
        res[key][0] += float(((useful_slab - useful_one) * msk).sum())
        res[key][1] += float(((issued_slab - issued_one) * msk).sum())
        if int(opts.refine_steps) >= 2:   # the slab square before it
            key = (int(opts.refine), 0)
            res[key][0] += float(((useful_slab - useful_one) * msk).sum())
            res[key][1] += float(((issued_slab - issued_one) * msk).sum())
    return {k: tuple(v) for k, v in res.items()}


def wave_blocks(npad: np.ndarray) -> np.ndarray:
    """32 x 32 wave blocks computed per product by the 64-tile kernels: the
    blocks on or below the diagonal inside n_pad (tiles with bi >= bj; a
    diagonal tile skips its block above the diagonal, an edge tile the blocks
    past n_pad), i.e. nb (nb + 1) / 2 with nb = n_pad / 32."""
    nb = np.asarray(npad, dtype=np.int64) // 32
    return (nb * (nb + 1) // 2).astype(np.float64)


def useful_flops(stats, n, npad, opts, slab=None) -> float:
    return sum(v[0] for v in flops_by_class(stats, n, npad, opts, slab).values())


# Matrix-core products one product of the schedule costs: the split-bfloat16
# form computes hi*hi + hi*lo + lo*hi, three bfloat16 products per product.
MFMA_PRODUCTS = {0: 1, 1: 1, 2: 1, 3: 1, 4: 3}


def gemm_kernel_symbol(mode: int, which: int, variant: int, pad_to: int) -> str:
    """Demangled name prefix (as profilers print it) of the GEMM kernel that
    runs for (precision, square/update, kernel variant) on a plan with the
    given padding; mirrors the variant fallback of the launcher."""
    v = effective_variant(mode, variant, pad_to)
    if v == 8:   # 256-wide tiles, synchronized rounds
        return f"sm::ns_gemm256_sync_kernel<{mode}, {which}>"
    if v >= 6:   # 256-wide tiles, 512 threads: <precision, kind, stage depth, buffers>
        return f"sm::ns_gemm256_kernel<{mode}, {which}, {32 if v == 6 else 16}, {2 if v == 6 else 4}>"
    if v >= 3:   # 128-wide tiles: <precision, kind, XCD-aware walk, prefetch depth>
        return f"sm::ns_gemm128_kernel<{mode}, {which}, {'false' if v == 4 else 'true'}, {6 if v == 5 else 1}>"
    kdiv = 2 if v == 2 else 1   # variant 2: half-depth LDS stages
    return f"sm::ns_gemm_kernel<{mode}, {which}, {kdiv}, {'true' if v >= 1 else 'false'}>"


# Bytes per stored element of a product's operands and result: float64 and
# float32 iterates, 16-bit copies for bf16 / f16, hi + lo copies for split bf16.
STORE_BYTES = {0: 8, 1: 4, 2: 2, 3: 2, 4: 4}
HBM_PEAK_GBS = 8000.0   # MI355X HBM3E


def bytes_by_class(stats: np.ndarray, n: np.ndarray, opts, slab=None, npad=None) -> dict:
    """{(precision, kind): algorithmic memory bytes of one pass}: a square
    reads X and writes Y, an update reads X and Y and writes X', each an
    n x n matrix in the storage of that precision's products; a slab update
    (slab = (loc, b, tshift_ref), with npad) reads one whole operand and b
    rows of the other and writes b rows."""
    nf = n.astype(np.float64)
    n2 = nf ** 2
    res = {}
    for (prec, kind), cnt in product_counts(stats, opts).items():
        per = (2.0 if kind == 0 else 3.0) * STORE_BYTES[prec] * n2
        res[(prec, kind)] = float((np.asarray(cnt, dtype=np.float64) * per).sum())
    if slab is not None and int(opts.refine_steps) > 0:
        loc, b, tsh = slab
        msk = slab_mask(stats, npad, loc, b, opts, tsh)
        prec = int(opts.refine)
        bf = np.asarray(b, dtype=np.float64)
        diff = STORE_BYTES[prec] * ((n2 + 2.0 * nf * bf) - 3.0 * n2)
        res[(prec, 1)] += float((diff * msk).sum())
        if int(opts.refine_steps) >= 2:   # slab square: read X, write b columns
            diff = STORE_BYTES[prec] * ((n2 + nf * bf) - 2.0 * n2)
            res[(prec, 0)] += float((diff * msk).sum())
    return res
