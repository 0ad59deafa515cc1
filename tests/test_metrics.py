"""Host-side accounting used by the benchmark: wave blocks per product
against a brute-force count, product counts per precision phase, byte
counts, and the kernel names the launcher's variant fallback selects."""
import numpy as np

from paper_2205_14741_amd import metrics
from paper_2205_14741_amd import smsign as sm


def _brute_blocks(npad):
    T = (npad + 63) // 64
    c = 0
    for bi in range(T):
        for bj in range(bi + 1):
            for wm in range(2):
                for wn in range(2):
                    if bi * 64 + wm * 32 < npad and bj * 64 + wn * 32 < npad and not (bi == bj and wm < wn):
                        c += 1
    return c


def test_wave_blocks_brute_force():
    npads = np.arange(32, 1025, 32)
    assert np.array_equal(metrics.wave_blocks(npads), [_brute_blocks(int(x)) for x in npads])


def _stats(iters, low, status):
    st = np.zeros(len(iters), dtype=sm.STATS_DTYPE)
    st["iters"], st["iters_low"], st["status"] = iters, low, status
    return st


def test_product_counts_refined_and_plain():
    o = sm.default_opts("bf16x3")          # 2 float32 refinement steps
    st = _stats([12, 10], [10, 10], [2, 1])
    c = metrics.product_counts(st, o)
    # refined: 11 squares + 10 updates in bf16x3, 1 square + 2 updates in
    # f32, the first of which runs on the bf16x3 kernel (it multiplies the
    # main phase's copies); plain (status 1): 11 squares + 10 updates in bf16x3
    assert list(c[(sm.SM_BF16X3, 0)]) == [11, 11] and list(c[(sm.SM_BF16X3, 1)]) == [11, 10]
    assert list(c[(sm.SM_F32, 0)]) == [1, 0] and list(c[(sm.SM_F32, 1)]) == [1, 0]
    # float64 refined in float64: every product stays in float64
    o64 = sm.default_opts("f64", refine_steps=2, switch_tol=0.1)
    c64 = metrics.product_counts(st, o64)
    assert list(c64[(sm.SM_F64, 1)]) == [12, 10] and list(c64[(sm.SM_F64, 0)]) == [12, 11]


def test_bytes_by_class():
    o = sm.default_opts("f64")
    st = _stats([3], [3], [1])
    b = metrics.bytes_by_class(st, np.array([10]), o)
    assert b[(sm.SM_F64, 0)] == 4 * 2 * 8 * 100   # 4 squares: read X, write Y
    assert b[(sm.SM_F64, 1)] == 3 * 3 * 8 * 100   # 3 updates: read X, Y, write X'


def test_kernel_symbols_follow_launcher_fallback():
    assert metrics.gemm_kernel_symbol(4, 0, 1, 64) == "sm::ns_gemm_kernel<4, 0, 1, true>"
    assert metrics.gemm_kernel_symbol(4, 1, 2, 64) == "sm::ns_gemm_kernel<4, 1, 2, true>"
    assert metrics.gemm_kernel_symbol(4, 1, 3, 64) == "sm::ns_gemm128_kernel<4, 1, true, 1>"
    assert metrics.gemm_kernel_symbol(1, 0, 4, 64) == "sm::ns_gemm128_kernel<1, 0, false, 1>"
    assert metrics.gemm_kernel_symbol(4, 0, 5, 64) == "sm::ns_gemm128_kernel<4, 0, true, 6>"
    # 16-bit products on a plan padded to 32 run the half-depth-stage kernel
    assert metrics.gemm_kernel_symbol(4, 0, 3, 32) == "sm::ns_gemm_kernel<4, 0, 2, true>"
    # no 128-wide tiles in float64 or on a plan padded to 32
    assert metrics.gemm_kernel_symbol(0, 0, 3, 64) == "sm::ns_gemm_kernel<0, 0, 1, true>"
    assert metrics.gemm_kernel_symbol(1, 0, 3, 32) == "sm::ns_gemm_kernel<1, 0, 1, true>"
    assert metrics.gemm_kernel_symbol(0, 1, 0, 32) == "sm::ns_gemm_kernel<0, 1, 1, false>"
    # 256-wide tiles (16-bit copies only; float32 falls back to the ring kernel)
    assert metrics.gemm_kernel_symbol(4, 1, 6, 64) == "sm::ns_gemm256_kernel<4, 1, 32, 2>"
    assert metrics.gemm_kernel_symbol(3, 0, 7, 64) == "sm::ns_gemm256_kernel<3, 0, 16, 4>"
    assert metrics.gemm_kernel_symbol(4, 1, 8, 64) == "sm::ns_gemm256_sync_kernel<4, 1>"
    assert metrics.gemm_kernel_symbol(1, 1, 8, 64) == "sm::ns_gemm128_kernel<1, 1, true, 6>"
    assert metrics.gemm_kernel_symbol(4, 1, 8, 32) == "sm::ns_gemm_kernel<4, 1, 2, true>"


def _brute_slab(npad, loc, b, tsh):
    w = 1 << tsh
    T = (npad + w - 1) // w
    cols = {c // w for c in range(loc, loc + b)}
    return sum(1 for bi in range(T) for bj in range(T) if bj in cols)


def test_slab_tiles_brute_force():
    for npad in (64, 128, 192, 320, 576):
        for tsh in (6, 7):
            for loc in range(0, npad - 6, 13):
                for b in (1, 2, 6):
                    assert int(metrics.slab_tiles(npad, loc, b, tsh)) == _brute_slab(npad, loc, b, tsh)


def test_slab_accounting():
    # one refined submatrix, n = 200 padded to 256, the atom's 6 columns at
    # 61 .. 66 (two 64-wide tile columns: 8 slab tiles < 10 triangle tiles)
    n, npad, loc, b = np.array([200]), np.array([256]), np.array([61]), np.array([6])
    st = _stats([12], [10], [2])
    o = sm.default_opts("bf16x3")                   # 2 refinement steps
    assert metrics.slab_mask(st, npad, loc, b, o, 6).all()
    fl = metrics.flops_by_class(st, n, npad, o, (loc, b, 6))
    full = metrics.flops_by_class(st, n, npad, o)
    # the one float32 update (the second refinement update) is the slab
    assert fl[(sm.SM_F32, 1)][0] == 2.0 * 200 * 200 * 6
    # issued: 8 row blocks x 2 column blocks (the 32-wide wave blocks 32..63
    # and 64..95 that hold columns 61 .. 66)
    assert fl[(sm.SM_F32, 1)][1] == 8 * 2 * 2 * 32 * 32 * 256
    assert fl[(sm.SM_BF16X3, 1)] == full[(sm.SM_BF16X3, 1)]
    # the one float32 square (before the last update) is a slab too
    assert fl[(sm.SM_F32, 0)][0] == 2.0 * 200 * 200 * 6
    assert fl[(sm.SM_F32, 0)][1] == 8 * 2 * 2 * 32 * 32 * 256
    assert fl[(sm.SM_BF16X3, 0)] == full[(sm.SM_BF16X3, 0)]
    by = metrics.bytes_by_class(st, n, o, (loc, b, 6), npad)
    assert by[(sm.SM_F32, 1)] == 4 * (200 * 200 + 2 * 200 * 6)
    assert by[(sm.SM_F32, 0)] == 4 * (200 * 200 + 200 * 6)
    # a single refinement step runs on the main kernel in full: no slab
    o1 = sm.default_opts("bf16x3", refine_steps=1)
    assert not metrics.slab_mask(st, npad, loc, b, o1, 6).any()
    # 128-wide tiles: 2 tile rows x 1 tile column = 2 tiles < 3 triangle tiles
    assert metrics.slab_mask(st, npad, loc, b, o, 7).all()
    fl7 = metrics.flops_by_class(st, n, npad, o, (loc, b, 7))
    # 64-wide wave blocks 0..63 and 64..127: 4 columns of 32
    assert fl7[(sm.SM_F32, 1)][1] == 8 * 4 * 2 * 32 * 32 * 256
    # not converged (status 1): no refinement ran, nothing changes
    st1 = _stats([12], [12], [1])
    assert metrics.flops_by_class(st1, n, npad, o, (loc, b, 6)) == metrics.flops_by_class(st1, n, npad, o)
    # a slab with no fewer tiles than the triangle is not taken (npad 64)
    assert not metrics.slab_mask(st, np.array([64]), np.array([10]), b, o, 6).any()
    # float64 refined in float64: the last of the float64 updates and the
    # square before it are slabs (12 updates, 12 squares in all)
    o64 = sm.default_opts("f64", refine_steps=2, switch_tol=0.1)
    f64 = metrics.flops_by_class(st, n, npad, o64, (loc, b, 6))
    assert f64[(sm.SM_F64, 1)][0] == 11 * 200 * 200 * 201 + 2.0 * 200 * 200 * 6
    assert f64[(sm.SM_F64, 0)][0] == 11 * 200 * 200 * 201 + 2.0 * 200 * 200 * 6
    # one refinement step (float32 main phase): the square before the last
    # update decided the switch and stays full
    of1 = sm.default_opts("f32", refine_steps=1, switch_tol=0.1)
    f1 = metrics.flops_by_class(st, n, npad, of1, (loc, b, 6))
    f1full = metrics.flops_by_class(st, n, npad, of1)
    assert f1[(sm.SM_F32, 0)] == f1full[(sm.SM_F32, 0)]
    assert f1[(sm.SM_F32, 1)][0] == f1full[(sm.SM_F32, 1)][0] - 200 * 200 * 201 + 2.0 * 200 * 200 * 6
