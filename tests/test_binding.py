"""Host-side argument checks of the Python binding (no GPU): the size check
of caller-owned patch pools against the context's field count."""
import types

import numpy as np
import pytest
import torch

from paper_1308_1464_amd import inputs
from paper_1308_1464_amd import manyclaw as mc
from paper_1308_1464_amd import patchset


def fake_ctx(solver, dtype, key):
    mc._CTX[key] = (solver, dtype)
    return types.SimpleNamespace(value=key)


def test_patch_pools_sized_for_the_solver():
    plist = inputs.patch_set(4, seed=2)
    hp, pool, offs = patchset.pack(plist)
    need3 = max(o + 3 * nx * ny for o, (nx, ny, _) in zip(offs, plist))
    try:
        sw = fake_ctx(mc.MC_SW_ROE, mc.MC_F64, 101)
        eu = fake_ctx(mc.MC_EULER_ROE, mc.MC_F64, 102)
        f32 = fake_ctx(mc.MC_SW_ROE, mc.MC_F32, 103)
        ok = torch.zeros(need3, dtype=torch.float64)
        mc._check_pools("f", sw, hp, len(plist), (ok, ok))           # exactly large enough
        with pytest.raises(mc.ManyclawError):                         # one element short
            mc._check_pools("f", sw, hp, len(plist), (ok, torch.zeros(need3 - 1, dtype=torch.float64)))
        with pytest.raises(mc.ManyclawError):                         # four fields needed
            mc._check_pools("f", eu, hp, len(plist), (ok, ok))
        mc._check_pools("f", f32, hp, len(plist), (torch.zeros(need3, dtype=torch.float32),) * 2)
        mc._check_pools("f", sw, hp, len(plist), (12345, 67890))      # raw addresses pass through
    finally:
        for k in (101, 102, 103):
            mc._CTX.pop(k, None)


def test_grid_buffers_sized_for_the_context():
    try:
        sw = fake_ctx(mc.MC_SW_ROE, mc.MC_F64, 201)
        mc._CTX[201] = (mc.MC_SW_ROE, mc.MC_F64, 10, 7)
        vc = fake_ctx(mc.MC_ACOUSTICS_VC, mc.MC_F32, 202)
        mc._CTX[202] = (mc.MC_ACOUSTICS_VC, mc.MC_F32, 10, 7)
        good = torch.zeros((3, 7, 10), dtype=torch.float64)
        short = torch.zeros((3, 7, 9), dtype=torch.float64)
        mc._check_grid("f", sw, mc.state(good, good).nbytes)
        with pytest.raises(mc.ManyclawError):
            mc._check_grid("f", sw, mc.state(good, short).nbytes)
        q32 = torch.zeros((3, 7, 10), dtype=torch.float32)
        mc._check_grid("f", vc, (mc._nbytes(q32),), torch.zeros((2, 7, 10), dtype=torch.float32))
        with pytest.raises(mc.ManyclawError):      # aux needs two fields
            mc._check_grid("f", vc, (mc._nbytes(q32),), torch.zeros((1, 7, 10), dtype=torch.float32))
        with pytest.raises(mc.ManyclawError):      # FP64 buffers hold twice the bytes, FP32 not enough
            mc._check_grid("f", sw, (mc._nbytes(torch.zeros((3, 7, 10), dtype=torch.float32)),))
        mc._check_grid("f", sw, (None, None))      # raw addresses pass through
    finally:
        for k in (201, 202):
            mc._CTX.pop(k, None)
