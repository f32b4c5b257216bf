"""The allocation-free batched-patch entry point (mc_step2d_patches_noalloc)
against the allocating one (mc_step2d_patches, eager) on the same batches:
two calls in a row on one context and stream, the second with a smaller
batch, each bitwise equal to its reference (same kernel and schedule); a
batch whose schedule exceeds the static device array is refused before any
launch."""
import numpy as np
import pytest

import gpu_util as gu
from paper_1308_1464_amd import inputs
from paper_1308_1464_amd import manyclaw as mc

pytestmark = pytest.mark.gpu
G = 9.81
FIELDS = ("nx", "ny", "offset", "t", "dt", "cfl", "smax", "status", "n_acc", "n_rej", "cur")


def _buffers(plist):
    hp, pool, _ = gu.pack_patches(plist)
    p0 = gu.dev(pool)
    return hp, p0, gu.torch().zeros_like(p0), gu.patches_to_dev(hp)


def _result(plist, bufs):
    hp, p0, p1, dp = bufs
    n = len(plist)
    out = gu.patches_from_dev(dp, n)
    a, b = gu.host(p0), gu.host(p1)
    return out, [gu.unpack_patch(a, b, out[k]) for k in range(n)]


def _same(ref, got):
    for k, (dr, dg) in enumerate(zip(ref[0], got[0])):
        for f in FIELDS:
            assert getattr(dr, f) == getattr(dg, f), (k, f, getattr(dr, f), getattr(dg, f))
        assert np.array_equal(ref[1][k], got[1][k]), k


def test_noalloc_matches_allocating_entry_point():
    big = inputs.patch_set(300, seed=21)
    small = inputs.patch_set(45, seed=22)
    prm = mc.params(g=G, cfl_target=0.9, cfl_max=1.0)
    with gu.context(mc.MC_SW_ROE, mc.MC_F64, prm, 1, 1, 1.0, 1.0) as h:
        refs = []
        for plist, nst in ((big, 8), (small, 5)):
            print(f"allocating entry point: {len(plist)} patches, {nst} steps", flush=True)
            bufs = _buffers(plist)
            mc.mc_step2d_patches(h, bufs[0], bufs[3], len(plist), bufs[1], bufs[2], nst, mc.MC_LIM_MC,
                                 False)
            refs.append(_result(plist, bufs))
        # two allocation-free calls in a row on the same stream, no wait
        # between them: the second (smaller) schedule is copied in after the
        # first call's kernel
        bb, bs = _buffers(big), _buffers(small)
        print("allocation-free entry point: 300 then 45 patches", flush=True)
        mc.mc_step2d_patches_noalloc(h, bb[0], bb[3], len(big), bb[1], bb[2], 8, mc.MC_LIM_MC)
        mc.mc_step2d_patches_noalloc(h, bs[0], bs[3], len(small), bs[1], bs[2], 5, mc.MC_LIM_MC)
        _same(refs[0], _result(big, bb))
        _same(refs[1], _result(small, bs))
        assert all(d.n_acc == 8 for d in refs[0][0]) and all(d.n_acc == 5 for d in refs[1][0])


def test_noalloc_refuses_a_schedule_beyond_its_array():
    """One 60-column patch of 1.44 million rows at 4 rows per chunk makes
    360,000 work items (12 bytes each), more than the 4 MiB array."""
    nx, ny = 60, 1_440_000
    hp = mc.patch_array([dict(nx=nx, ny=ny, offset=0, dx=1.0 / nx, dy=1.0 / ny, t=0.0, dt=-1.0,
                              cfl=0.0, smax=0.0, bc=mc.MC_BC_EXTRAP, status=0, n_acc=0, n_rej=0,
                              cur=0)])
    t = gu.torch()
    p0 = t.ones(3 * nx * ny, dtype=t.float32, device="cuda")
    p1 = t.zeros_like(p0)
    dp = gu.patches_to_dev(hp)
    with gu.context(mc.MC_SW_ROE, mc.MC_F32, mc.params(g=G), 1, 1, 1.0, 1.0) as h:
        mc.mc_patches_set_rows(h, hp, 1, [4, 4, 4, 4])
        with pytest.raises(mc.ManyclawError) as ei:
            mc.mc_step2d_patches_noalloc(h, hp, dp, 1, p0, p1, 1, mc.MC_LIM_MC)
        assert ei.value.code == mc.MC_ESCRATCH
    assert not t.any(p1).item()
