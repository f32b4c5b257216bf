"""Separate contexts used from separate host threads at the same time:
every thread's unsplit steps and patch batch give bitwise the results of the
same work run alone (the library's per-context tables are shared between
threads; the binding releases the interpreter lock during each call)."""
import threading

import numpy as np
import pytest

import gpu_util as gu
from paper_1308_1464_amd import inputs
from paper_1308_1464_amd import manyclaw as mc

pytestmark = pytest.mark.gpu
G = 9.81
NX, NY = 96, 80


def work(seed):
    """unsplit steps on a grid and one patch batch, on a context of its own"""
    t = gu.torch()
    q0 = inputs.sw_dam_break(NX, seed=seed, ny=NY)
    q0[1] = 0.2 * inputs.random_field((NY, NX), seed=seed + 1)
    ctx = mc.mc_ctx_create(mc.MC_SW_ROE, mc.MC_F64, mc.params(g=G), NX, NY, 1 / NX, 1 / NY)
    try:
        a = gu.dev(q0)
        b = t.empty_like(a)
        st = mc.state(a, b)
        for _ in range(10):
            mc.mc_step2d_unsplit(ctx, st, None, 4e-4, mc.MC_LIM_MC, 1)
        plist = inputs.patch_set(12, seed=seed)
        hp, pool, _ = gu.pack_patches(plist)
        p0 = gu.dev(pool)
        p1 = t.zeros_like(p0)
        dp = gu.patches_to_dev(hp)
        mc.mc_step2d_patches(ctx, hp, dp, len(plist), p0, p1, 4, mc.MC_LIM_MC, 0)
        t.cuda.synchronize()
        grid = gu.host(a if st.cur == 0 else b)
        desc = gu.patches_from_dev(dp, len(plist))
        pa, pb = gu.host(p0), gu.host(p1)
        patches = [gu.unpack_patch(pa, pb, desc[k]) for k in range(len(plist))]
    finally:
        mc.mc_ctx_destroy(ctx)
    return grid, patches


def test_contexts_in_threads():
    seeds = list(range(8))
    print("threads: sequential reference", flush=True)
    ref = {s: work(s) for s in seeds}
    out, errs = {}, []

    def body(s):
        try:
            out[s] = work(s)
        except Exception as e:  # reported below
            errs.append((s, repr(e)))

    print("threads: 8 threads at once", flush=True)
    th = [threading.Thread(target=body, args=(s,)) for s in seeds]
    for x in th:
        x.start()
    for x in th:
        x.join(timeout=120)
    assert not errs, errs
    assert all(not x.is_alive() for x in th)
    for s in seeds:
        np.testing.assert_array_equal(out[s][0], ref[s][0])
        for a, b in zip(out[s][1], ref[s][1]):
            np.testing.assert_array_equal(a, b)
