"""GPU tests of the unsplit step with transverse solves (mc_step2d_unsplit)
against the unsplit oracle (oracle/unsplit.py).

Bars (the plain step's, readings A15/A16): FP64 per field max |GPU -
oracle| / max |oracle| <= 1e-12 after one step and <= 1e-9 after ten; FP32
relative L1 <= 1e-5 after three steps from the FP32-rounded start; smax to
1e-12.
"""
import numpy as np
import pytest

from paper_1308_1464_amd import inputs
from paper_1308_1464_amd import manyclaw as mc

pytestmark = pytest.mark.gpu


def _t():
    import torch
    return torch


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def U():
    from oracle import unsplit as U_
    return U_


@pytest.fixture(scope="module")
def O():
    import oracle as O_
    return O_


def dev(a, dtype):
    return _t().from_numpy(np.ascontiguousarray(a)).to("cuda", dtype)


def host(x):
    _t().cuda.synchronize()
    return x.detach().cpu().numpy().astype(np.float64)


def medium(name, nx, ny):
    """aux (rho, c): the four-block layered medium, or a medium with an
    independent random (rho, c) in every cell"""
    if name == "vc":
        return np.ascontiguousarray(inputs.layered_medium(nx, ny))
    return np.stack([inputs.random_field((ny, nx), seed=31, lo=0.5, hi=3.0),
                     inputs.random_field((ny, nx), seed=32, lo=0.4, hi=1.5)])


def problem(name, nx, ny):
    if name in ("vc", "vc_rand"):
        q = inputs.acoustics_pulse(nx, ny)
        q[1] = 0.2 * inputs.random_field((ny, nx), seed=33)
        q[2] = -0.1 * inputs.random_field((ny, nx), seed=34)
        return "ACOUSTICS_VC", dict(), np.ascontiguousarray(q)
    if name in ("sw", "hlle"):
        q = inputs.sw_dam_break(nx, seed=1, ny=ny)
        q[1] = 0.3 * q[0] * inputs.random_field((ny, nx), seed=2)
        q[2] = -0.2 * q[0] * inputs.random_field((ny, nx), seed=3)
        return ("SW_ROE" if name == "sw" else "SW_HLLE"), dict(g=9.81), q
    if name == "euler":
        q, _ = inputs.euler_quadrants(nx, seed=6, ny=ny)
        return "EULER_ROE", dict(gamma=1.4), q
    if name == "acoustics":
        q = inputs.acoustics_pulse(max(nx, ny))[:, :ny, :nx]
        q[1] = 0.2 * inputs.random_field((ny, nx), seed=4)
        return "ACOUSTICS", dict(rho=1.3, K=0.8), np.ascontiguousarray(q)
    u, v = {"adv_pp": (1.0, 0.5), "adv_pm": (0.8, -0.6), "adv_mm": (-0.7, -0.9)}[name]
    q = inputs.random_field((1, ny, nx), seed=5)
    return "ADVECTION", dict(u=u, v=v), q


def maxrel(a, b):
    return max(np.abs(a[m] - b[m]).max() / np.abs(b[m]).max() for m in range(a.shape[0])
               if np.abs(b[m]).max() > 0)


@pytest.mark.parametrize("name,bc", [("sw", 0), ("sw", 1), ("hlle", 0), ("hlle", 1), ("euler", 1), ("euler", 0),
                                     ("acoustics", 0),
                                     ("vc", 0), ("vc", 1), ("vc_rand", 1),
                                     ("adv_pp", 0), ("adv_pm", 1), ("adv_mm", 0)])
def test_fp64_matches_oracle(U, O, name, bc):
    t = _t()
    nx, ny = 150, 130
    solver, prm, q0 = problem(name, nx, ny)
    aux = medium(name, nx, ny) if solver == "ACOUSTICS_VC" else None
    say(f"case: unsplit FP64 {name} {nx}x{ny} bc={bc}")
    P = O.params(**prm)
    sid = getattr(O, solver)
    sm0, _ = O.max_speed(sid, P, q0, 1 / nx, 1 / ny, bc, aux=aux)
    dt = 0.7 / sm0
    ctx = mc.mc_ctx_create(getattr(mc, "MC_" + solver), mc.MC_F64, mc.params(**prm), nx, ny, 1 / nx, 1 / ny)
    a = dev(q0, t.float64)
    b = t.empty_like(a)
    au = dev(aux, t.float64) if aux is not None else None
    st = mc.state(a, b)
    cfl = t.zeros(16, dtype=t.uint8, device="cuda")
    q = q0
    for k in range(10):
        mc.mc_step2d_unsplit(ctx, st, au, dt, mc.MC_LIM_MC, bc, cfl)
        q, sm = U.unsplit_step(sid, P, q, 1 / nx, 1 / ny, dt, O.LIM_MC, bc, aux=aux)
        g = host(a if st.cur == 0 else b)
        err = maxrel(g, q)
        c = mc.cfl_from_tensor(cfl)
        if k in (0, 9):
            say(f"step {k + 1}: max rel err {err:.3e}; smax gpu {c.smax:.6f} oracle {sm:.6f}")
        assert err <= (1e-12 if k == 0 else 1e-9)
        assert abs(c.smax - sm) <= 1e-12 * sm
    mc.mc_ctx_destroy(ctx)


@pytest.mark.parametrize("lim", ["LIM_NONE", "LIM_MINMOD", "LIM_SUPERBEE", "LIM_VANLEER", "LIM_FIRST_ORDER"])
def test_limiters(U, O, lim):
    t = _t()
    nx, ny = 70, 66
    solver, prm, q0 = problem("sw", nx, ny)
    say(f"case: unsplit FP64 sw {lim}")
    P = O.params(**prm)
    dt = 0.5 / O.max_speed(O.SW_ROE, P, q0, 1 / nx, 1 / ny, 1)[0]
    ctx = mc.mc_ctx_create(mc.MC_SW_ROE, mc.MC_F64, mc.params(**prm), nx, ny, 1 / nx, 1 / ny)
    a = dev(q0, t.float64)
    b = t.empty_like(a)
    st = mc.state(a, b)
    mc.mc_step2d_unsplit(ctx, st, None, dt, getattr(mc, "MC_" + lim), 1)
    q, _ = U.unsplit_step(O.SW_ROE, P, q0, 1 / nx, 1 / ny, dt, getattr(O, lim), 1)
    err = maxrel(host(b), q)
    say("max rel err", err)
    assert err <= 1e-12
    mc.mc_ctx_destroy(ctx)


@pytest.mark.parametrize("name", ["sw", "hlle", "acoustics", "euler", "vc_rand"])
def test_fp32_matches_oracle(U, O, name):
    t = _t()
    nx, ny = 97, 83
    solver, prm, q0 = problem(name, nx, ny)
    q0 = q0.astype(np.float32).astype(np.float64)
    aux = None
    if solver == "ACOUSTICS_VC":
        aux = medium(name, nx, ny).astype(np.float32).astype(np.float64)
    say(f"case: unsplit FP32 {name}")
    P = O.params(**prm)
    sid = getattr(O, solver)
    dt = 0.7 / O.max_speed(sid, P, q0, 1 / nx, 1 / ny, 0, aux=aux)[0]
    ctx = mc.mc_ctx_create(getattr(mc, "MC_" + solver), mc.MC_F32, mc.params(**prm), nx, ny, 1 / nx, 1 / ny)
    a = dev(q0, t.float32)
    b = t.empty_like(a)
    au = dev(aux, t.float32) if aux is not None else None
    st = mc.state(a, b)
    q = q0
    for _ in range(3):
        mc.mc_step2d_unsplit(ctx, st, au, dt, mc.MC_LIM_MC, 0)
        q, _ = U.unsplit_step(sid, P, q, 1 / nx, 1 / ny, dt, O.LIM_MC, 0, aux=aux)
    g = host(a if st.cur == 0 else b)
    for m in range(q.shape[0]):
        e = np.abs(g[m] - q[m]).sum() / np.abs(q[m]).sum()
        say("field", m, "rel L1", e)
        assert e <= 1e-5
    mc.mc_ctx_destroy(ctx)


def test_unsupported_solvers():
    t = _t()
    say("case: unsplit with a learned solver; VC acoustics without aux")
    # MC_ACOUSTICS_VC is supported but needs its (rho, c) fields
    for s, dt_, meqn in ((mc.MC_SW_SURROGATE, mc.MC_F32, 3), (mc.MC_ACOUSTICS_VC, mc.MC_F64, 3)):
        ctx = mc.mc_ctx_create(s, dt_, mc.params(), 8, 8, 0.1, 0.1)
        a = t.ones((meqn, 8, 8), dtype=t.float64 if dt_ == mc.MC_F64 else t.float32, device="cuda")
        b = t.ones_like(a)
        with pytest.raises(mc.ManyclawError):
            mc.mc_step2d_unsplit(ctx, mc.state(a, b), None, 1e-3, mc.MC_LIM_MC, 1)
        mc.mc_ctx_destroy(ctx)


@pytest.mark.parametrize("nx,ny", [(1, 1), (1, 7), (3, 2), (5, 61)])
def test_tiny_grids(U, O, nx, ny):
    t = _t()
    say(f"case: unsplit FP64 tiny grid {nx}x{ny}")
    q0 = np.stack([1.0 + 0.1 * inputs.random_field((ny, nx), seed=21),
                   0.1 * inputs.random_field((ny, nx), seed=22), 0.1 * inputs.random_field((ny, nx), seed=23)])
    P = O.params(g=9.81)
    ctx = mc.mc_ctx_create(mc.MC_SW_ROE, mc.MC_F64, mc.params(g=9.81), nx, ny, 0.1, 0.1)
    for bc in (0, 1):
        a = dev(q0, t.float64)
        b = t.empty_like(a)
        st = mc.state(a, b)
        mc.mc_step2d_unsplit(ctx, st, None, 0.005, mc.MC_LIM_MC, bc)
        q, _ = U.unsplit_step(O.SW_ROE, P, q0, 0.1, 0.1, 0.005, O.LIM_MC, bc)
        assert maxrel(host(b), q) <= 1e-13
    mc.mc_ctx_destroy(ctx)
    # variable-coefficient acoustics on the same tiny grids
    aux = medium("vc_rand", nx, ny)
    ctx = mc.mc_ctx_create(mc.MC_ACOUSTICS_VC, mc.MC_F64, mc.params(), nx, ny, 0.1, 0.1)
    for bc in (0, 1):
        a = dev(q0, t.float64)
        b = t.empty_like(a)
        st = mc.state(a, b)
        mc.mc_step2d_unsplit(ctx, st, dev(aux, t.float64), 0.02, mc.MC_LIM_MC, bc)
        q, _ = U.unsplit_step(O.ACOUSTICS_VC, O.params(), q0, 0.1, 0.1, 0.02, O.LIM_MC, bc, aux=aux)
        assert maxrel(host(b), q) <= 1e-13
    mc.mc_ctx_destroy(ctx)


@pytest.mark.parametrize("solver", ["SW_ROE", "SW_HLLE"])
def test_dry_block(U, O, solver):
    """a dry block (h = 0): its edges carry nothing and have no transverse
    part; the result is finite, matches the oracle and flags the step"""
    t = _t()
    nx, ny = 70, 52
    q0 = np.stack([1.0 + 0.2 * inputs.random_field((ny, nx), seed=61),
                   0.2 * inputs.random_field((ny, nx), seed=62), 0.2 * inputs.random_field((ny, nx), seed=63)])
    q0[:, 20:30, 15:40] = 0.0
    say(f"case: unsplit FP64 {solver} dry block")
    P = O.params(g=9.81)
    sid = getattr(O, solver)
    ctx = mc.mc_ctx_create(getattr(mc, "MC_" + solver), mc.MC_F64, mc.params(g=9.81), nx, ny, 1 / nx, 1 / ny)
    for bc in (0, 1):
        a = dev(q0, t.float64)
        b = t.empty_like(a)
        st = mc.state(a, b)
        mc.mc_step2d_unsplit(ctx, st, None, 0.002, mc.MC_LIM_MC, bc)
        q, _ = U.unsplit_step(sid, P, q0, 1 / nx, 1 / ny, 0.002, O.LIM_MC, bc)
        g = host(b)
        assert np.isfinite(g).all()
        err = maxrel(g, q)
        say("bc", bc, "max rel err", err)
        assert err <= 1e-12
        assert mc.mc_status_get(ctx) & mc.MC_ST_NONPHYS
    mc.mc_ctx_destroy(ctx)


@pytest.mark.parametrize("name,nx,ny", [("sw", 60, 9), ("sw", 61, 9), ("sw", 120, 5), ("sw", 121, 33),
                                        ("vc_rand", 61, 40), ("euler", 120, 24)])
def test_strip_edge_widths(U, O, name, nx, ny):
    """Widths at and one past whole multiples of the kernel's 60 output
    columns, both boundary rules: the last output lane of one strip meets the
    next strip's halo, and a transverse part enters the cell of a
    neighbouring strip."""
    t = _t()
    solver, prm, q0 = problem(name, nx, ny)
    aux = medium(name, nx, ny) if solver == "ACOUSTICS_VC" else None
    P = O.params(**prm)
    sid = getattr(O, solver)
    ctx = mc.mc_ctx_create(getattr(mc, "MC_" + solver), mc.MC_F64, mc.params(**prm), nx, ny, 1 / nx, 1 / ny)
    au = dev(aux, t.float64) if aux is not None else None
    try:
        for bc in (0, 1):
            say(f"case: unsplit FP64 {name} {nx}x{ny} bc={bc} (strip-edge width)")
            sm0, _ = O.max_speed(sid, P, q0, 1 / nx, 1 / ny, bc, aux=aux)
            dt = 0.6 / sm0
            a = dev(q0, t.float64)
            b = t.empty_like(a)
            st = mc.state(a, b)
            q = q0
            for _ in range(2):
                mc.mc_step2d_unsplit(ctx, st, au, dt, mc.MC_LIM_MC, bc)
                q, _ = U.unsplit_step(sid, P, q, 1 / nx, 1 / ny, dt, O.LIM_MC, bc, aux=aux)
            assert maxrel(host(a if st.cur == 0 else b), q) <= 1e-12
    finally:
        mc.mc_ctx_destroy(ctx)
