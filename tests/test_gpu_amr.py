"""GPU tests of the two-level refinement coupling (mc_amr_*) against the
refinement oracle (oracle/amr.py) and the plain step.

Bars (the plain step's, SURVEY readings A15/A16):
  FP64   per field max |GPU - oracle| / max |oracle| <= 1e-12 after one
         coarse step and <= 1e-9 after ten, on the coarse grid and on
         every patch
  FP32   per field relative L1 <= 1e-5 against the FP64 oracle from the
         FP32-rounded start, after three coarse steps
  r = 1  the hierarchy reproduces the plain split step (mc_step2d) of the
         coarse grid to 1e-14 (the fix-up then trades a flux for the same
         flux computed from the other side: round-off only)
  conservation  periodic domain: the totals of the coarse grid (covered
         cells carry the average of their patch) stay constant to 1e-13
"""
import numpy as np
import pytest

from paper_1308_1464_amd import inputs
from paper_1308_1464_amd import manyclaw as mc

pytestmark = pytest.mark.gpu

G = 9.81


def _t():
    import torch
    return torch


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def A():
    from oracle import amr as A_
    return A_


@pytest.fixture(scope="module")
def O():
    import oracle as O_
    return O_


def dev(a):
    return _t().from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(x):
    _t().cuda.synchronize()
    return x.detach().cpu().numpy()


def fine_ic(nx, ny, r, seed):
    """dam break sampled on the fine level plus a smooth velocity field"""
    qf = inputs.sw_dam_break(nx * r, seed=seed, ny=ny * r)
    yy, xx = np.meshgrid((np.arange(ny * r) + 0.5) / (ny * r), (np.arange(nx * r) + 0.5) / (nx * r),
                         indexing="ij")
    qf[1] = qf[0] * 0.3 * np.sin(2 * np.pi * yy)
    qf[2] = qf[0] * 0.2 * np.cos(2 * np.pi * xx)
    return qf


def average(qf, r):
    m, NY, NX = qf.shape
    return qf.reshape(m, NY // r, r, NX // r, r).mean(axis=(2, 4))


class Run:
    """a GPU hierarchy and the oracle's, from the same start"""

    def __init__(self, A, nx, ny, r, boxes, bc, dtype=np.float64, seed=0, solver=None, qf=None, consts=None):
        self.A = A
        self.H = A.Hierarchy(nx, ny, 1.0 / nx, 1.0 / ny, r, boxes, bc)
        qf = fine_ic(nx, ny, r, seed) if qf is None else qf
        self.consts = dict(g=G) if consts is None else consts
        self.qc = average(qf, r).astype(dtype).astype(np.float64)
        self.fine = [f.astype(dtype).astype(np.float64) for f in A.restrict(self.H, qf)]
        self.dtype = dtype
        self.solver = mc.MC_SW_ROE if solver is None else solver
        dt_code = mc.MC_F64 if dtype == np.float64 else mc.MC_F32
        self.ctx = mc.mc_ctx_create(self.solver, dt_code, mc.params(**self.consts), nx, ny, 1.0 / nx, 1.0 / ny)
        self.amr = mc.mc_amr_create(self.ctx, r, boxes, bc)
        mc.mc_amr_set(self.amr, -1, dev(self.qc.astype(dtype)))
        for p, f in enumerate(self.fine):
            assert mc.mc_amr_dims(self.amr, p) == (f.shape[2], f.shape[1])
            mc.mc_amr_set(self.amr, p, dev(f.astype(dtype)))
        self.cfl = _t().zeros(16, dtype=_t().uint8, device="cuda")

    def gpu_state(self):
        t = _t()
        qc = t.empty((self.qc.shape[0], self.H.ny, self.H.nx), dtype=t.float64 if self.dtype == np.float64 else t.float32,
                     device="cuda")
        mc.mc_amr_get(self.amr, -1, qc)
        out = [host(qc).astype(np.float64)]
        for p, f in enumerate(self.fine):
            x = t.empty(f.shape, dtype=qc.dtype, device="cuda")
            mc.mc_amr_get(self.amr, p, x)
            out.append(host(x).astype(np.float64))
        return out

    def step(self, dt, limiter, oracle_solver):
        mc.mc_amr_step(self.amr, dt, limiter, self.cfl)
        self.qc, self.fine, smc, smf = self.A.step(self.H, self.qc, self.fine, dt, limiter, solver=oracle_solver,
                                                   P=self.A.params(**self.consts))
        return smc, smf

    def close(self):
        mc.mc_amr_destroy(self.amr)
        mc.mc_ctx_destroy(self.ctx)


def maxrel(a, b):
    return max(np.abs(a[m] - b[m]).max() / np.abs(b[m]).max() for m in range(a.shape[0]) if np.abs(b[m]).max() > 0)


CASES = [
    # (nx, ny, r, boxes, bc)
    (40, 36, 2, [(4, 5, 8, 6), (12, 5, 5, 9), (0, 20, 6, 7), (30, 28, 10, 8)], 0),
    (40, 36, 4, [(4, 5, 8, 6), (12, 5, 5, 9), (0, 20, 6, 7), (30, 28, 10, 8)], 1),
    (150, 90, 4, [(20, 10, 20, 18), (40, 10, 6, 30), (100, 60, 25, 20)], 0),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_fp64_matches_oracle(A, O, case):
    nx, ny, r, boxes, bc = CASES[case]
    say(f"case: AMR FP64 {nx}x{ny} r={r} {len(boxes)} patches bc={bc}")
    R = Run(A, nx, ny, r, boxes, bc, seed=case)
    P = O.params(g=G)
    sm, _ = O.max_speed(O.SW_ROE, P, average(fine_ic(nx, ny, r, case), r), 1 / nx, 1 / ny, bc)
    dt = 0.45 / sm
    for k in range(10):
        smc, smf = R.step(dt, mc.MC_LIM_MC, O.SW_ROE)
        gs = R.gpu_state()
        err = max([maxrel(gs[0], R.qc)] + [maxrel(g, f) for g, f in zip(gs[1:], R.fine)])
        c = mc.cfl_from_tensor(R.cfl)
        ref_sm = max(smc, smf / r)
        if k == 0 or k == 9:
            say(f"step {k + 1}: max rel err {err:.3e}; smax gpu {c.smax:.6f} oracle {ref_sm:.6f}")
        assert err <= (1e-12 if k == 0 else 1e-9)
        assert abs(c.smax - ref_sm) <= 1e-12 * ref_sm
    R.close()


def test_hlle_and_limiters(A, O):
    nx, ny, r, boxes, bc = CASES[0]
    for solver, osolver, lim in ((mc.MC_SW_HLLE, O.SW_HLLE, mc.MC_LIM_SUPERBEE),
                                 (mc.MC_SW_ROE, O.SW_ROE, mc.MC_LIM_MINMOD),
                                 (mc.MC_SW_ROE, O.SW_ROE, mc.MC_LIM_FIRST_ORDER)):
        say(f"case: AMR FP64 solver {solver} limiter {lim}")
        R = Run(A, nx, ny, r, boxes, bc, seed=7, solver=solver)
        for _ in range(2):
            R.step(0.002, lim, osolver)
        gs = R.gpu_state()
        err = max([maxrel(gs[0], R.qc)] + [maxrel(g, f) for g, f in zip(gs[1:], R.fine)])
        say("max rel err", err)
        assert err <= 1e-12
        R.close()


def test_fp32_matches_oracle(A, O):
    nx, ny, r, boxes, bc = CASES[1]
    say(f"case: AMR FP32 {nx}x{ny} r={r}")
    R = Run(A, nx, ny, r, boxes, bc, dtype=np.float32, seed=3)
    for _ in range(3):
        R.step(0.0015, mc.MC_LIM_MC, O.SW_ROE)
    gs = R.gpu_state()
    for g, o in zip(gs, [R.qc] + R.fine):
        for m in range(3):
            e = np.abs(g[m] - o[m]).sum() / max(np.abs(o[m]).sum(), 1e-300)
            assert e <= 1e-5, (m, e)
    R.close()


# patch widths 61 and 121 put a patch's last edge (i = nx) in lane 63 of a
# strip that is not the patch's last; only the strip holding the patch's
# last cell may write that edge's flux record
RATIO_ONE = {"mixed": (130, 70, [(10, 5, 30, 20), (40, 5, 12, 40), (90, 30, 40, 40)]),
             "width_1_mod_60": (250, 70, [(5, 5, 61, 20), (100, 10, 121, 30), (70, 40, 60, 25)])}


@pytest.mark.parametrize("layout", sorted(RATIO_ONE))
@pytest.mark.parametrize("bc", [0, 1])
def test_ratio_one_is_the_plain_step(O, bc, layout):
    t = _t()
    nx, ny, boxes = RATIO_ONE[layout]
    say(f"case: AMR r=1 against mc_step2d bc={bc} layout={layout}")
    q0 = fine_ic(nx, ny, 1, 11)
    dt = 0.8 / O.max_speed(O.SW_ROE, O.params(g=G), q0, 1 / nx, 1 / ny, bc)[0]
    ctx = mc.mc_ctx_create(mc.MC_SW_ROE, mc.MC_F64, mc.params(g=G), nx, ny, 1 / nx, 1 / ny)
    amr = mc.mc_amr_create(ctx, 1, boxes, bc)
    mc.mc_amr_set(amr, -1, dev(q0))
    for p, (i0, j0, w, h) in enumerate(boxes):
        mc.mc_amr_set(amr, p, dev(q0[:, j0:j0 + h, i0:i0 + w].copy()))
    a = dev(q0)
    b = t.empty_like(a)
    st = mc.state(a, b)
    for _ in range(5):
        mc.mc_amr_step(amr, dt, mc.MC_LIM_MC)
        mc.mc_step2d(ctx, st, None, dt, mc.MC_LIM_MC, bc)
    qp = host(a if st.cur == 0 else b)
    qa = t.empty_like(a)
    mc.mc_amr_get(amr, -1, qa)
    err = maxrel(host(qa), qp)
    say("max rel err against the plain step", err)
    assert err <= 1e-14
    mc.mc_amr_destroy(amr)
    mc.mc_ctx_destroy(ctx)


def test_conservation_periodic(A):
    nx, ny, r, boxes, _ = CASES[2]
    say("case: AMR conservation, periodic")
    R = Run(A, nx, ny, r, boxes, 0, seed=5)
    tot0 = R.gpu_state()[0].reshape(3, -1).sum(axis=1)
    scale = np.abs(R.gpu_state()[0]).reshape(3, -1).sum(axis=1)
    for _ in range(6):
        mc.mc_amr_step(R.amr, 0.001, mc.MC_LIM_MC)   # fine-level CFL about 0.7
    tot = R.gpu_state()[0].reshape(3, -1).sum(axis=1)
    drift = np.abs(tot - tot0) / scale
    say("relative drift of the totals", drift)
    assert drift.max() < 1e-13
    R.close()


def test_invalid_arguments():
    say("case: AMR invalid arguments")
    ctx = mc.mc_ctx_create(mc.MC_SW_ROE, mc.MC_F64, mc.params(), 16, 16, 0.1, 0.1)
    for boxes in ([(0, 0, 4, 4), (3, 3, 2, 2)], [(14, 0, 4, 4)], [(0, 0, 0, 3)]):
        with pytest.raises(mc.ManyclawError):
            mc.mc_amr_create(ctx, 2, boxes, 0)
    with pytest.raises(mc.ManyclawError):
        mc.mc_amr_create(ctx, 0, [(0, 0, 2, 2)], 0)
    amr = mc.mc_amr_create(ctx, 2, [(2, 2, 3, 3)], 1)
    with pytest.raises(mc.ManyclawError):
        mc.mc_amr_step(amr, -1.0, mc.MC_LIM_MC)
    with pytest.raises(mc.ManyclawError):
        mc.mc_amr_dims(amr, 1)
    # patch 0 holds 6 x 6 fine cells: a smaller buffer is refused by the binding
    with pytest.raises(mc.ManyclawError):
        mc.mc_amr_set(amr, 0, dev(np.zeros((3, 5, 6))))
    mc.mc_amr_set(amr, 0, dev(np.ones((3, 6, 6))))
    mc.mc_amr_destroy(amr)
    mc.mc_ctx_destroy(ctx)
    # variable-coefficient acoustics (no flux form) is refused
    ce = mc.mc_ctx_create(mc.MC_ACOUSTICS_VC, mc.MC_F64, mc.params(), 16, 16, 0.1, 0.1)
    with pytest.raises(mc.ManyclawError):
        mc.mc_amr_create(ce, 2, [(2, 2, 3, 3)], 1)
    mc.mc_ctx_destroy(ce)


@pytest.mark.parametrize("bc", [0, 1])
def test_no_patches_is_the_plain_step(bc):
    t = _t()
    nx, ny = 70, 50
    say(f"case: AMR without patches against mc_step2d bc={bc}")
    q0 = fine_ic(nx, ny, 1, 13)
    ctx = mc.mc_ctx_create(mc.MC_SW_ROE, mc.MC_F64, mc.params(g=G), nx, ny, 1 / nx, 1 / ny)
    amr = mc.mc_amr_create(ctx, 2, [], bc)
    mc.mc_amr_set(amr, -1, dev(q0))
    a = dev(q0)
    b = t.empty_like(a)
    st = mc.state(a, b)
    for _ in range(3):
        mc.mc_amr_step(amr, 0.002, mc.MC_LIM_MC)
        mc.mc_step2d(ctx, st, None, 0.002, mc.MC_LIM_MC, bc)
    qa = t.empty_like(a)
    mc.mc_amr_get(amr, -1, qa)
    # the same walker arithmetic: bit for bit
    np.testing.assert_array_equal(host(qa), host(a if st.cur == 0 else b))
    mc.mc_amr_destroy(amr)
    mc.mc_ctx_destroy(ctx)


OTHERS = {"EULER_ROE": dict(gamma=1.4), "ACOUSTICS": dict(rho=1.3, K=0.8), "ADVECTION": dict(u=0.9, v=-0.6)}


def other_ic(solver, NX, NY, seed):
    """fine-level data [m][NY][NX]: Euler four quadrants, an acoustic pulse
    with a random velocity, a random advected field"""
    if solver == "EULER_ROE":
        q, _ = inputs.euler_quadrants(NX, seed=seed, ny=NY)
        return q
    if solver == "ACOUSTICS":
        q = inputs.acoustics_pulse(NX, NY, width=60.0)
        q[1] = 0.2 * inputs.random_field((NY, NX), seed=seed)
        return q
    return 1.0 + inputs.random_field((1, NY, NX), seed=seed)


@pytest.mark.parametrize("solver", sorted(OTHERS))
@pytest.mark.parametrize("bc", [0, 1])
def test_other_solvers_match_oracle(A, O, solver, bc):
    nx, ny, r, boxes, _ = CASES[0]
    say(f"case: AMR FP64 {solver} {nx}x{ny} r={r} bc={bc}")
    qf = other_ic(solver, nx * r, ny * r, 3)
    sid, P = getattr(O, solver), O.params(**OTHERS[solver])
    R = Run(A, nx, ny, r, boxes, bc, solver=getattr(mc, "MC_" + solver), qf=qf, consts=OTHERS[solver])
    sm, _ = O.max_speed(sid, P, average(qf, r), 1 / nx, 1 / ny, bc)
    dt = 0.45 / sm
    for k in range(5):
        R.step(dt, mc.MC_LIM_MC, sid)
        gs = R.gpu_state()
        err = max([maxrel(gs[0], R.qc)] + [maxrel(g, f) for g, f in zip(gs[1:], R.fine)])
        if k in (0, 4):
            say(f"step {k + 1}: max rel err {err:.3e}")
        assert err <= (1e-12 if k == 0 else 1e-9)
    R.close()


def test_euler_fp32_matches_oracle(A, O):
    nx, ny, r, boxes, _ = CASES[1]
    say(f"case: AMR FP32 EULER_ROE {nx}x{ny} r={r}")
    qf = other_ic("EULER_ROE", nx * r, ny * r, 4)
    P = O.params(gamma=1.4)
    R = Run(A, nx, ny, r, boxes, 1, dtype=np.float32, solver=mc.MC_EULER_ROE, qf=qf, consts=dict(gamma=1.4))
    dt = 0.45 / O.max_speed(O.EULER_ROE, P, average(qf, r), 1 / nx, 1 / ny, 1)[0]
    for _ in range(3):
        R.step(dt, mc.MC_LIM_MC, O.EULER_ROE)
    gs = R.gpu_state()
    for g, o in zip(gs, [R.qc] + R.fine):
        for m in range(4):
            e = np.abs(g[m] - o[m]).sum() / max(np.abs(o[m]).sum(), 1e-300)
            assert e <= 1e-5, (m, e)
    R.close()


@pytest.mark.parametrize("solver", sorted(OTHERS))
def test_other_solvers_ratio_one_is_the_plain_step(O, solver):
    t = _t()
    nx, ny, boxes = RATIO_ONE["mixed"]
    q0 = other_ic(solver, nx, ny, 9)
    say(f"case: AMR r=1 {solver} against mc_step2d")
    sid, P = getattr(O, solver), O.params(**OTHERS[solver])
    dt = 0.8 / O.max_speed(sid, P, q0, 1 / nx, 1 / ny, 1)[0]
    ctx = mc.mc_ctx_create(getattr(mc, "MC_" + solver), mc.MC_F64, mc.params(**OTHERS[solver]), nx, ny,
                           1 / nx, 1 / ny)
    amr = mc.mc_amr_create(ctx, 1, boxes, 1)
    mc.mc_amr_set(amr, -1, dev(q0))
    for p, (i0, j0, w, h) in enumerate(boxes):
        mc.mc_amr_set(amr, p, dev(q0[:, j0:j0 + h, i0:i0 + w].copy()))
    a = dev(q0)
    b = t.empty_like(a)
    st = mc.state(a, b)
    for _ in range(4):
        mc.mc_amr_step(amr, dt, mc.MC_LIM_MC)
        mc.mc_step2d(ctx, st, None, dt, mc.MC_LIM_MC, 1)
    qp = host(a if st.cur == 0 else b)
    qa = t.empty_like(a)
    mc.mc_amr_get(amr, -1, qa)
    err = maxrel(host(qa), qp)
    say("max rel err against the plain step", err)
    assert err <= 1e-14
    mc.mc_amr_destroy(amr)
    mc.mc_ctx_destroy(ctx)
