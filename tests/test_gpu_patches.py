"""GPU parity of the batched-patch step (mc_step2d_patches): every patch
against an independent oracle run of that patch under its own time-step
rule (same dt sequence, rejections included)."""
import numpy as np
import pytest

import gpu_util as gu
from paper_1308_1464_amd import inputs
from paper_1308_1464_amd import manyclaw as mc

pytestmark = pytest.mark.gpu
G = 9.81


def _run(plist, nsteps, use_graph=False, rows=None, tune=False, limiter=mc.MC_LIM_MC,
         bc=mc.MC_BC_EXTRAP, calls=1, solver=mc.MC_SW_ROE, constants=None):
    hp, pool, _ = gu.pack_patches(plist, bc=bc)
    n = len(plist)
    p0 = gu.dev(pool)
    p1 = gu.torch().zeros_like(p0)
    dp = gu.patches_to_dev(hp)
    prm = mc.params(cfl_target=0.9, cfl_max=1.0, **(constants or dict(g=G)))
    chosen = None
    with gu.context(solver, mc.MC_F64, prm, 1, 1, 1.0, 1.0) as h:
        if rows is not None:
            mc.mc_patches_set_rows(h, hp, n, rows)
        if tune:
            chosen = mc.mc_patches_tune(h, hp, n, limiter)
        for _ in range(calls):
            mc.mc_step2d_patches(h, hp, dp, n, p0, p1, nsteps, limiter, use_graph)
        gu.torch().cuda.synchronize()
        out = gu.patches_from_dev(dp, n)
    return out, gu.host(p0), gu.host(p1), chosen


def _oracle(orc, nx, ny, q, nsteps, bc, solver=None, constants=None):
    P = orc.params(**(constants or dict(g=G)))
    sid = orc.SW_ROE if solver is None else solver
    return orc.run2d(sid, P, q, 1.0 / nx, 1.0 / ny, orc.LIM_MC, bc, 0.9, 1.0, nsteps)


def _check(orc, plist, out, a, b, idx, nsteps, tol=1e-10, bc=1, solver=None, constants=None):
    for k in idx:
        nx, ny, q = plist[k]
        d = out[k]
        qo, dts, t, nrej, st = _oracle(orc, nx, ny, q, nsteps, bc, solver, constants)
        g = gu.unpack_patch(a, b, d, meqn=q.shape[0])
        assert d.n_acc == nsteps, (k, d.n_acc)
        assert d.n_rej == nrej, (k, d.n_rej, nrej)
        assert abs(d.t - t) <= 1e-12 * t, (k, d.t, t)
        err = gu.rel_inf(g, qo)
        assert np.all(err <= tol), (k, nx, ny, err)


def test_small_batch_matches_oracle(orc):
    plist = inputs.patch_set(40, seed=3)
    print("patches: 40 patches, 20 steps", flush=True)
    out, a, b, _ = _run(plist, 20)
    _check(orc, plist, out, a, b, range(40), 20)


def test_degenerate_patches(orc):
    shapes = [(1, 1), (1, 9), (9, 1), (16, 256), (256, 16), (60, 60), (61, 17), (125, 3)]
    plist = []
    for k, (nx, ny) in enumerate(shapes):
        q = inputs.sw_dam_break(max(nx, 2), ny=max(ny, 2), noise=1e-3, seed=k, h_in=3.0)
        q = q[:, :ny, :nx].copy()
        q[1] = 0.2 * inputs.random_field((ny, nx), seed=100 + k)
        plist.append((nx, ny, q))
    for bc, obc in ((mc.MC_BC_EXTRAP, 1), (mc.MC_BC_PERIODIC, 0)):
        print(f"degenerate patches bc={bc}", flush=True)
        out, a, b, _ = _run(plist, 6, bc=bc)
        _check(orc, plist, out, a, b, range(len(plist)), 6, bc=obc)


def test_rows_invariance_and_graph(orc):
    """Bitwise the same results for any rows-per-chunk choice, eager or
    graph-replayed, in one call or two consecutive calls."""
    plist = inputs.patch_set(60, seed=5)
    ref, a0, b0, _ = _run(plist, 10, rows=[16, 24, 32, 48])
    for rows, graph, calls, ns in (([8, 8, 8, 8], False, 1, 10), ([32, 64, 128, 256], True, 1, 10),
                                   ([12, 24, 96, 40], True, 2, 5)):
        out, a, b, _ = _run(plist, ns, use_graph=graph, rows=rows, calls=calls)
        for k in range(len(plist)):
            assert out[k].n_acc == ref[k].n_acc and out[k].t == ref[k].t
            assert np.array_equal(gu.unpack_patch(a, b, out[k]), gu.unpack_patch(a0, b0, ref[k])), k


def test_full_batch_2000_sampled(orc):
    """The batch configuration: 2,000 dam-break patches with sides
    log-uniform in [16, 256], 20 steps each under its own dt, one persistent
    graph-captured launch with autotuned rows; sampled patches (largest,
    smallest, widest, tallest, random) against independent oracle runs."""
    plist = inputs.patch_set(2000, seed=0)
    print("patches: 2000 patches, 20 steps, tuned, graph", flush=True)
    out, a, b, rows = _run(plist, 20, use_graph=True, tune=True)
    print("tuned rows", rows, flush=True)
    assert all(out[k].n_acc == 20 for k in range(2000))
    assert all(out[k].status == 0 for k in range(2000))
    cells = np.array([nx * ny for nx, ny, _ in plist])
    nxs = np.array([nx for nx, _, _ in plist])
    nys = np.array([ny for _, ny, _ in plist])
    idx = {int(np.argmax(cells)), int(np.argmin(cells)), int(np.argmax(nxs)), int(np.argmax(nys)),
           int(np.argmin(nxs)), int(np.argmin(nys))}
    idx |= set(int(x) for x in inputs.rng(7).choice(2000, 20, replace=False))
    _check(orc, plist, out, a, b, sorted(idx), 20)
    for k in range(0, 2000, 97):
        assert gu.unpack_patch(a, b, out[k])[0].min() > 0


def test_invalid_patch_arguments():
    plist = inputs.patch_set(3, seed=1)
    hp, pool, _ = gu.pack_patches(plist)
    p0 = gu.dev(pool)
    dp = gu.patches_to_dev(hp)
    with gu.context(mc.MC_SW_ROE, mc.MC_F64, mc.params(), 1, 1, 1.0, 1.0) as h:
        with pytest.raises(mc.ManyclawError):
            mc.mc_step2d_patches(h, hp, dp, 3, p0, p0, 2, mc.MC_LIM_MC)
        bad = gu.pack_patches(plist)[0]
        bad[1].nx = 0
        with pytest.raises(mc.ManyclawError):
            mc.mc_step2d_patches(h, bad, dp, 3, p0, gu.torch().zeros_like(p0), 2, mc.MC_LIM_MC)
    # pools sized for three fields under a four-field solver: refused by the
    # binding's size check before the library is called
    with gu.context(mc.MC_EULER_ROE, mc.MC_F64, mc.params(), 1, 1, 1.0, 1.0) as h:
        with pytest.raises(mc.ManyclawError):
            mc.mc_step2d_patches(h, hp, dp, 3, p0, gu.torch().zeros_like(p0), 2, mc.MC_LIM_MC)


OTHER = {"EULER_ROE": dict(gamma=1.4), "ACOUSTICS": dict(rho=1.3, K=0.8), "ADVECTION": dict(u=1.0, v=-0.6)}


def _other_patches(solver):
    shapes = [(16, 40), (61, 17), (100, 64), (33, 130), (1, 9), (130, 5)]
    plist = []
    for k, (nx, ny) in enumerate(shapes):
        if solver == "EULER_ROE":
            q, _ = inputs.euler_quadrants(max(nx, 2), seed=20 + k, ny=max(ny, 2))
        elif solver == "ACOUSTICS":
            q = inputs.acoustics_pulse(max(nx, 2), max(ny, 2))
            q[1] = 0.2 * inputs.random_field(q[0].shape, seed=30 + k)
        else:
            q = inputs.random_field((1, max(ny, 2), max(nx, 2)), seed=40 + k)
        plist.append((nx, ny, np.ascontiguousarray(q[:, :ny, :nx])))
    return plist


@pytest.mark.parametrize("solver", sorted(OTHER))
def test_other_solvers_match_oracle(orc, solver):
    """Euler, acoustics and advection patches: every patch against the
    oracle under its own time-step rule, both boundary rules"""
    plist = _other_patches(solver)
    for bc, obc in ((mc.MC_BC_EXTRAP, 1), (mc.MC_BC_PERIODIC, 0)):
        print(f"patches: {solver} {len(plist)} patches bc={bc}", flush=True)
        out, a, b, _ = _run(plist, 8, bc=bc, solver=getattr(mc, "MC_" + solver), constants=OTHER[solver])
        _check(orc, plist, out, a, b, range(len(plist)), 8, bc=obc, solver=getattr(orc, solver),
               constants=OTHER[solver])


def test_unsupported_solvers():
    """variable-coefficient acoustics (per-cell aux) and the learned solvers
    are refused"""
    plist = inputs.patch_set(3, seed=9)
    for solver, dt_ in ((mc.MC_ACOUSTICS_VC, mc.MC_F64), (mc.MC_SW_SURROGATE, mc.MC_F32)):
        hp, pool, _ = gu.pack_patches(plist, dtype=gu.npdt(dt_))
        p0 = gu.dev(pool, dtype=gu.npdt(dt_))
        p1 = gu.torch().zeros_like(p0)
        dp = gu.patches_to_dev(hp)
        with gu.context(solver, dt_, mc.params(), 1, 1, 1.0, 1.0) as h:
            with pytest.raises(mc.ManyclawError):
                mc.mc_step2d_patches(h, hp, dp, len(plist), p0, p1, 2, mc.MC_LIM_MC, 0)


_TUNE_CHILD = r"""
import json, sys
sys.path.insert(0, sys.argv[1])
import torch
from paper_1308_1464_amd import inputs, patchset
from paper_1308_1464_amd import manyclaw as mc
plist = inputs.patch_set(60, seed=9)
hp, _, _ = patchset.pack(plist)
h = mc.mc_ctx_create(mc.MC_SW_ROE, mc.MC_F64, mc.params(g=9.81), 1, 1, 1.0, 1.0)
rows = mc.mc_patches_tune(h, hp, len(plist), mc.MC_LIM_MC)
torch.cuda.synchronize()
mc.mc_ctx_destroy(h)
print(json.dumps(rows))
"""


def test_tune_cache_persists_across_processes(tmp_path):
    """MANYCLAW_TUNE_CACHE: a first process tunes and writes its choice; the
    entry is then edited to a choice the tuner would not make, and a second
    process tuning the same batch returns exactly the edited entry (a cache
    hit, nothing timed)."""
    import json
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    cache = tmp_path / "tune.json"
    env = dict(os.environ, MANYCLAW_TUNE_CACHE=str(cache))

    def child():
        print("tune child process", flush=True)
        r = subprocess.run([sys.executable, "-c", _TUNE_CHILD, root], env=env, capture_output=True,
                           text=True, timeout=240)
        assert r.returncode == 0, r.stderr[-2000:]
        return json.loads(r.stdout.strip().splitlines()[-1])

    first = child()
    entries = json.loads(cache.read_text())
    assert len(entries) == 1 and list(entries.values())[0] == first
    edited = [4 if first[0] != 4 else 5, 4096, 4, 4096]
    key = list(entries)[0]
    cache.write_text(json.dumps({key: edited}))
    assert child() == edited


_ROWS_CHILD = r"""
import json, sys
sys.path.insert(0, sys.argv[1])
import torch
from paper_1308_1464_amd import inputs
from paper_1308_1464_amd import manyclaw as mc
n = 96
q0 = inputs.sw_dam_break(n, seed=4)
a = torch.from_numpy(q0).cuda()
b = torch.empty_like(a)
h = mc.mc_ctx_create(mc.MC_SW_ROE, mc.MC_F64, mc.params(g=9.81), n, n, 1.0 / n, 1.0 / n)
rows = mc.mc_tune_rows(h, mc.state(a, b), None, 1e-4, mc.MC_LIM_MC, mc.MC_BC_EXTRAP)
torch.cuda.synchronize()
mc.mc_ctx_destroy(h)
print(json.dumps(rows))
"""


def test_rows_tuner_uses_the_cache(tmp_path):
    """mc_tune_rows with MANYCLAW_TUNE_CACHE: the first process stores its
    choice under a key of its own beside a patch entry, and a second process
    returns an edited entry unchanged (a cache hit)."""
    import json
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    cache = tmp_path / "tune.json"
    cache.write_text('{\n"patch-entry": [8, 16, 32, 64]\n}\n')
    env = dict(os.environ, MANYCLAW_TUNE_CACHE=str(cache))

    def child():
        print("rows tuner child process", flush=True)
        r = subprocess.run([sys.executable, "-c", _ROWS_CHILD, root], env=env, capture_output=True,
                           text=True, timeout=240)
        assert r.returncode == 0, r.stderr[-2000:]
        return json.loads(r.stdout.strip().splitlines()[-1])

    first = child()
    entries = json.loads(cache.read_text())
    assert entries["patch-entry"] == [8, 16, 32, 64]
    keys = [k for k in entries if k.startswith("rows-")]
    assert len(keys) == 1 and entries[keys[0]] == [first], entries
    edited = 24 if first != 24 else 40
    entries[keys[0]] = [edited]
    cache.write_text(json.dumps(entries))
    assert child() == edited
