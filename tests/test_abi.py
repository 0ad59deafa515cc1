"""Host-side checks of the C ABI (no GPU needed): the library loads and exports
every function the header declares, the symbolic plan matches the oracle's
index sets, chunking respects the budget, and bad input is rejected."""
import os
import re

import numpy as np
import pytest

import synth
from oracle import submatrix as om
from paper_2205_14741_amd import smsign as sm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if not fn.endswith(".h"):
            continue
        txt = open(os.path.join(ROOT, "include", fn)).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][\w\s\*]*?\b([A-Za-z_]\w*)\s*\(", txt, re.M):
            if m.group(1) not in ("if", "return", "sizeof"):
                names.add(m.group(1))
    return names


def test_library_exports_every_declared_symbol():
    lib = sm.lib()
    declared = _declared_functions()
    assert {"build_submatrices", "submatrix_sign", "assemble_P", "energy_trace"} <= declared
    for name in declared:
        assert hasattr(lib, name), name
    assert set(sm.EXPORTED) <= declared


@pytest.mark.parametrize("make", [synth.config1,
                                  lambda: synth.water_system(20, 1.3, 1),
                                  lambda: synth.lattice_system(4, 3, 1.6, 2, vacancy=0.1, jitter=0.05)])
def test_plan_matches_oracle_index_sets(make):
    m = make()
    p = sm.Plan(m, 64)
    info = p.info()
    view = om.BlockView(m)
    for i in range(m.n_atoms):
        atoms, idx, loc = om.submatrix_indices(view, i)
        assert info["n"][i] == idx.shape[0]
        assert info["loc"][i] == loc
        assert info["npad"][i] == -(-idx.shape[0] // 64) * 64
    n_sub, n_chunks, ws_bytes, nvals = p.sizes(sm.SM_F64)
    assert n_sub == m.n_atoms and n_chunks == 1 and nvals == m.vals.shape[0]
    reg, off = p.ws_layout(sm.SM_F64)
    assert np.all(np.diff(reg) >= 0) and reg[-1] == ws_bytes
    assert off[0] == 0 and np.all(np.diff(off) == 3 * info["npad"][:-1].astype(np.int64) ** 2)
    # float32 iterates plus their 16-bit operand copies take 8 bytes per element slot
    for code in (sm.SM_BF16, sm.SM_F16, sm.SM_BF16X3):
        assert p.sizes(code)[2] == ws_bytes
    assert p.sizes(sm.SM_F32)[2] < ws_bytes
    with pytest.raises(sm.SmError, match="storage"):
        p.sizes(7)


def test_workspace_too_small_for_schedule():
    """A float32-storage workspace is refused (before any launch) for a
    schedule whose products read operand copies."""
    import torch
    m = synth.config1()
    p = sm.Plan(m, 64)
    ws = torch.empty(p.sizes(sm.SM_F32)[2], dtype=torch.uint8)
    stats = torch.empty(1, dtype=torch.uint8)
    H = torch.zeros(m.vals.shape[0], dtype=torch.float64)
    with pytest.raises(sm.SmError, match="workspace"):
        sm.build_submatrices(p, 0, H, 0.0, sm.default_opts("bf16x3"), ws, stats)


def test_chunking_respects_budget():
    m = synth.config1()
    budget = 3 * 128 * 128 * 10   # ten submatrices of n_pad 128
    p = sm.Plan(m, 64, budget)
    info = p.info()
    n_chunks = p.n_chunks
    assert n_chunks == 7
    for c in range(n_chunks):
        sel = info["chunk"] == c
        assert 0 < sel.sum() <= 10
    assert sorted(info["order"]) == list(range(m.n_atoms))
    _, _, ws_small, _ = p.sizes(sm.SM_F32)
    _, _, ws_full, _ = sm.Plan(m, 64).sizes(sm.SM_F32)
    assert ws_small < ws_full


def test_positions_order():
    """Morton order of the atom centres: a permutation in which consecutive
    atoms are close (much closer than in the random sequential placement
    order), larger size buckets first, chunks contiguous in the new order;
    refused once the plan lives on a device (not testable here) or for a
    non-finite position."""
    m = synth.water_system(64, 1.5, 2)
    p = sm.Plan(m, 64, 3 * 256 * 256 * 8)
    p.set_positions(m.positions, bucket_rows=0)
    info = p.info()
    order = info["order"]
    assert sorted(order) == list(range(m.n_atoms))
    pos = m.positions

    def mean_step(o, lag=9):   # atoms three molecules apart in the order
        return float(np.mean(np.linalg.norm(pos[o[lag:]] - pos[o[:-lag]], axis=1)))

    assert mean_step(order) < 0.75 * mean_step(np.arange(m.n_atoms))
    ch = info["chunk"][order]
    assert np.all(np.diff(ch) >= 0) and np.all(np.diff(ch) <= 1)
    p.set_positions(m.positions, bucket_rows=64)
    info = p.info()
    assert np.all(np.diff(info["npad"][info["order"]] // 64) <= 0)
    bad = m.positions.copy()
    bad[3, 1] = np.nan
    with pytest.raises(sm.SmError):
        p.set_positions(bad)


def test_pad_128():
    m = synth.config1()
    info = sm.Plan(m, 128).info()
    assert np.all(info["npad"] == 128)


def _mutated(mut):
    m = synth.lattice_system(3, 2, 1.1, 0)
    cp, ri, po = m.col_ptr.copy(), m.row_idx.copy(), m.panel_off.copy()
    bs = m.block_size.copy()
    mut(bs, cp, ri, po)
    return synth.BlockSparse(bs, cp, ri, po, m.vals, m.positions, m.box, m.n_occ)


@pytest.mark.parametrize("mut,msg", [
    (lambda bs, cp, ri, po: ri.__setitem__(slice(0, 2), ri[0:2][::-1].copy()), "ascending"),
    (lambda bs, cp, ri, po: po.__setitem__(1, po[1] + 1), "panel_off"),
    (lambda bs, cp, ri, po: bs.__setitem__(0, 0), "block_size"),
])
def test_plan_rejects_bad_patterns(mut, msg):
    with pytest.raises(sm.SmError) as e:
        sm.Plan(_mutated(mut))
    assert e.value.code == sm.SM_ERR_ARG and msg in str(e.value)


def test_plan_rejects_missing_diagonal_and_asymmetry():
    # 2 atoms, column 0 stores only row 1 (no diagonal)
    bs = np.array([1, 1], np.int32)
    m = synth.BlockSparse(bs, np.array([0, 1, 3]), np.array([1, 0, 1], np.int32),
                          np.array([0, 1, 3]), np.zeros(3), np.zeros((2, 3)), None, 1)
    with pytest.raises(sm.SmError, match="diagonal"):
        sm.Plan(m)
    # column 0 stores rows {0, 1}, column 1 stores only {1}: not symmetric
    m = synth.BlockSparse(bs, np.array([0, 2, 3]), np.array([0, 1, 1], np.int32),
                          np.array([0, 2, 3]), np.zeros(3), np.zeros((2, 3)), None, 1)
    with pytest.raises(sm.SmError, match="symmetric"):
        sm.Plan(m)
    with pytest.raises(sm.SmError, match="pad_to"):
        sm.Plan(synth.config1(), 96)


def test_default_opts():
    o = sm.default_opts("f64")
    assert o.phase1 == sm.SM_F64 and o.refine_steps == 0 and o.tol == 1e-10
    o = sm.default_opts("bf16x3")
    assert o.phase1 == sm.SM_BF16X3 and o.refine == sm.SM_F32 and o.refine_steps == 2
    assert sm.storage_prec(o) == sm.SM_BF16X3
    assert sm.storage_prec(sm.default_opts("f32")) == sm.SM_F32
    with pytest.raises(sm.SmError):
        sm.default_opts(9)


def test_noalloc_bracket_rejects_plans_beyond_its_scratch():
    """More atoms than the fixed scratch holds: a clear error before any
    device work (this runs without a GPU)."""
    n = (1 << 19) + 1
    m = synth.from_pairs([1] * n, [], [], np.zeros(n), n_occ=0)
    plan = sm.Plan(m, 32)
    rc = sm.lib().sm_gershgorin_bracket_noalloc(plan.handle, 8, 8, None)
    assert rc == -1
    assert b"exceed the fixed scratch" in sm.lib().sm_last_error()


def test_default_gemm_variants():
    """Before tuning, a plan holds size-based GEMM variants: 64-wide XCD-aware
    tiles for float64 and small submatrices, 256-wide (16-bit) and 128-wide
    ring (float32) tiles for large ones padded to 64, half-depth stages for
    16-bit products padded to 32; the library reports 9 variants."""
    import synth
    from paper_2205_14741_amd import smsign as sm
    assert sm.lib().sm_gemm_variants() == 9
    small = synth.config1()
    assert list(sm.sm_plan_tuning(sm.Plan(small, 64))) == [1, 1, 1, 1, 1]
    assert list(sm.sm_plan_tuning(sm.Plan(small, 32))) == [1, 1, 2, 2, 2]
    big = synth.water_system(64, 1.95, 2)          # n_pad up to 896
    assert list(sm.sm_plan_tuning(sm.Plan(big, 64))) == [1, 5, 8, 8, 8]
