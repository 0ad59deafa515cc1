"""The allocation-free bracket (sm_gershgorin_bracket_noalloc) against the
allocating one (sm_gershgorin_bracket), through the C ABI: the same kernels on
the library's fixed device scratch, so the two results agree bitwise.  Two
calls in a row, the second on a smaller system, so the second reads only what
it wrote itself."""
import numpy as np
import pytest

import synth
from paper_2205_14741_amd import smsign as sm
from gpu_helpers import h_dev

pytestmark = pytest.mark.gpu


def test_noalloc_bracket_matches_allocating_one(dev):
    import torch
    out = torch.full((2,), float("nan"), dtype=torch.float64, device=dev)
    for m in (synth.config2(), synth.config1()):   # 967 atoms, then 64
        plan = sm.Plan(m, 32)
        H = h_dev(m)
        lo, hi = sm.sm_gershgorin_bracket(plan, H)      # allocating form (uploads the plan)
        out.fill_(float("nan"))
        sm.sm_gershgorin_bracket_noalloc(plan, H, out)
        torch.cuda.synchronize()
        got = out.cpu().numpy()
        print(f"{m.name}: [{lo}, {hi}] vs {got.tolist()}")
        assert got[0] == lo and got[1] == hi


def test_noalloc_bracket_needs_device_tables(dev):
    import torch
    m = synth.config1()
    plan = sm.Plan(m, 32)
    out = torch.zeros(2, dtype=torch.float64, device=dev)
    with pytest.raises(sm.SmError, match="device tables"):
        sm.sm_gershgorin_bracket_noalloc(plan, h_dev(m), out)
