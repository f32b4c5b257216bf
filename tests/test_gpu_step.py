"""GPU parity of the fused split step (mc_step2d / mc_run2d) against the
oracle: element by element at sizes the oracle finishes in seconds, tile
and halo invariance, the CFL reduction, the device time-step rule, and
sampled windows at the full 4096 x 4096 size."""
import ctypes

import numpy as np
import pytest

import gpu_util as gu
from paper_1308_1464_amd import inputs
from paper_1308_1464_amd import manyclaw as mc

pytestmark = pytest.mark.gpu

G = 9.81
TOL1, TOL100 = 1e-12, 1e-9   # FP64, per-field max norm, after 1 and 100 steps
TOL32 = 1e-5                 # FP32 vs FP64 oracle, per-field relative L1


def _oracle_steps(orc, sid, P, q, dx, dy, dts, lim, bc, aux=None, nthreads=8):
    sm = []
    for dt in dts:
        q, s, _ = orc.step2d(sid, P, q, dx, dy, dt, lim, bc, aux=aux, nthreads=nthreads)
        sm.append(s)
    return q, sm


def test_acoustics_pulse_128(orc):
    """Constant acoustics, 128 x 128, periodic, MC, CFL 0.9 (dt = 0.9/128):
    1 step within 1e-12 and 100 steps within 1e-9 of the oracle."""
    n = 128
    print("acoustics 128x128 FP64 periodic MC", flush=True)
    q0 = inputs.acoustics_pulse(n)
    prm = mc.params(rho=1.0, K=1.0)
    P = orc.params(rho=1.0, K=1.0)
    dt = 0.9 / 128
    g1, sm1, st = gu.run_steps(mc.MC_ACOUSTICS, mc.MC_F64, prm, q0, 1 / n, 1 / n, [dt],
                               mc.MC_LIM_MC, mc.MC_BC_PERIODIC)
    o1, osm = _oracle_steps(orc, orc.ACOUSTICS, P, q0, 1 / n, 1 / n, [dt], orc.LIM_MC, orc.BC_PERIODIC)
    assert np.all(gu.rel_inf(g1, o1) <= TOL1), gu.rel_inf(g1, o1)
    assert sm1[0] == 128.0 and osm[0] == 128.0
    g100, _, _ = gu.run_steps(mc.MC_ACOUSTICS, mc.MC_F64, prm, q0, 1 / n, 1 / n, [dt] * 100,
                              mc.MC_LIM_MC, mc.MC_BC_PERIODIC)
    o100, _ = _oracle_steps(orc, orc.ACOUSTICS, P, q0, 1 / n, 1 / n, [dt] * 100, orc.LIM_MC,
                            orc.BC_PERIODIC)
    assert np.all(gu.rel_inf(g100, o100) <= TOL100), gu.rel_inf(g100, o100)


@pytest.mark.parametrize("nx,ny", [(512, 512), (127, 93)])
def test_sw_fp64_parity(orc, nx, ny):
    """Shallow-water dam break with noise, Roe + HH, MC, extrapolation:
    1 and 100 steps (oracle dt sequence) against the oracle."""
    print(f"sw fp64 {nx}x{ny}", flush=True)
    q0 = inputs.sw_dam_break(nx, ny=ny, seed=1)
    prm = mc.params(g=G)
    P = orc.params(g=G)
    dx, dy = 1 / nx, 1 / ny
    _, dts, _, _, _ = orc.run2d(orc.SW_ROE, P, q0, dx, dy, orc.LIM_MC, orc.BC_EXTRAP, 0.9, 1.0,
                                100, nthreads=8)
    g1, sm, st = gu.run_steps(mc.MC_SW_ROE, mc.MC_F64, prm, q0, dx, dy, dts[:1], mc.MC_LIM_MC,
                              mc.MC_BC_EXTRAP)
    o1, osm = _oracle_steps(orc, orc.SW_ROE, P, q0, dx, dy, dts[:1], orc.LIM_MC, orc.BC_EXTRAP)
    assert np.all(gu.rel_inf(g1, o1) <= TOL1), gu.rel_inf(g1, o1)
    assert abs(sm[0] - osm[0]) <= 1e-14 * osm[0]
    assert st == 0
    g100, sm, _ = gu.run_steps(mc.MC_SW_ROE, mc.MC_F64, prm, q0, dx, dy, dts, mc.MC_LIM_MC,
                               mc.MC_BC_EXTRAP)
    o100, osm = _oracle_steps(orc, orc.SW_ROE, P, q0, dx, dy, dts, orc.LIM_MC, orc.BC_EXTRAP)
    assert np.all(gu.rel_inf(g100, o100) <= TOL100), gu.rel_inf(g100, o100)
    assert np.max(np.abs(np.array(sm) - np.array(osm)) / np.array(osm)) < 1e-11


def test_sw_fp32_parity(orc):
    """FP32 state and arithmetic vs the FP64 oracle started from the
    FP32-rounded initial state, 50 steps, same dt sequence."""
    n = 512
    print("sw fp32 512x512 50 steps", flush=True)
    q0 = inputs.sw_dam_break(n, seed=2).astype(np.float32).astype(np.float64)
    prm = mc.params(g=G)
    P = orc.params(g=G)
    _, dts, _, _, _ = orc.run2d(orc.SW_ROE, P, q0, 1 / n, 1 / n, orc.LIM_MC, orc.BC_EXTRAP, 0.9,
                                1.0, 50, nthreads=8)
    g, _, _ = gu.run_steps(mc.MC_SW_ROE, mc.MC_F32, prm, q0, 1 / n, 1 / n, dts, mc.MC_LIM_MC,
                           mc.MC_BC_EXTRAP)
    o, _ = _oracle_steps(orc, orc.SW_ROE, P, q0, 1 / n, 1 / n, dts, orc.LIM_MC, orc.BC_EXTRAP)
    e = gu.rel_l1(g, o)
    print("fp32 L1", e, "inf", gu.rel_inf(g, o))
    assert np.all(e <= TOL32), e


@pytest.mark.parametrize("solver,lim,bc", [
    ("ADVECTION", "MC", "PERIODIC"), ("ADVECTION", "NONE", "EXTRAP"),
    ("ACOUSTICS", "SUPERBEE", "EXTRAP"), ("ACOUSTICS", "FIRST_ORDER", "PERIODIC"),
    ("SW_ROE", "MINMOD", "PERIODIC"), ("SW_ROE", "VANLEER", "EXTRAP"),
    ("SW_HLLE", "MC", "EXTRAP"), ("EULER_ROE", "MC", "PERIODIC"),
    ("ACOUSTICS_VC", "MC", "PERIODIC"),
])
def test_solvers_limiters_bcs_fp64(orc, solver, lim, bc):
    """Every solver, limiter and boundary rule: 10 steps on a ragged grid."""
    nx, ny = 133, 70
    print(f"{solver} {lim} {bc} {nx}x{ny}", flush=True)
    sid = getattr(mc, "MC_" + solver)
    osid = getattr(orc, solver)
    L, OL = getattr(mc, "MC_LIM_" + lim), getattr(orc, "LIM_" + lim)
    B, OB = getattr(mc, "MC_BC_" + bc), getattr(orc, "BC_" + bc)
    aux = None
    if solver == "ADVECTION":
        q0 = inputs.random_field((1, ny, nx), seed=3)
        q0[0, 20:40, 30:70] += 2.0
    elif solver.startswith("ACOUSTICS"):
        q0 = np.stack([inputs.acoustics_pulse(nx, ny=ny, width=80.0)[0],
                       0.1 * inputs.random_field((ny, nx), seed=4),
                       0.1 * inputs.random_field((ny, nx), seed=5)])
        if solver == "ACOUSTICS_VC":
            X, Y = inputs.centres(nx, ny)
            rho = np.where(X < 0.6, 1.0, 2.5)
            c = np.where(Y < 0.4, 1.0, 0.6)
            aux = np.stack([rho, c])
    elif solver == "EULER_ROE":
        q0, _ = inputs.euler_quadrants(nx, ny=ny, seed=1)
    else:
        q0 = inputs.sw_dam_break(nx, ny=ny, seed=6)
        q0[1] = 0.5 * inputs.random_field((ny, nx), seed=7)
    prm = mc.params(u=0.8, v=-0.6, rho=1.3, K=2.0, g=G)
    P = orc.params(u=0.8, v=-0.6, rho=1.3, K=2.0, g=G)
    _, dts, _, _, _ = orc.run2d(osid, P, q0, 1 / nx, 1 / ny, OL, OB, 0.8, 1.0, 10, aux=aux)
    g, sm, st = gu.run_steps(sid, mc.MC_F64, prm, q0, 1 / nx, 1 / ny, dts, L, B, aux=aux)
    o, osm = _oracle_steps(orc, osid, P, q0, 1 / nx, 1 / ny, dts, OL, OB, aux=aux)
    err = gu.rel_inf(g, o)
    tol = 1e-11 if solver != "EULER_ROE" else 1e-10
    assert np.all(err <= tol), err
    np.testing.assert_allclose(sm, osm, rtol=1e-13)


@pytest.mark.parametrize("nx,ny", [(1, 1), (1, 37), (61, 1), (60, 60), (61, 61), (121, 65),
                                   (2, 300)])
def test_ragged_and_degenerate_grids(orc, nx, ny):
    print(f"ragged {nx}x{ny}", flush=True)
    q0 = inputs.sw_dam_break(max(nx, 2), ny=max(ny, 2), seed=8)[:, :ny, :nx].copy()
    q0[1] = 0.3 * inputs.random_field((ny, nx), seed=9)
    q0[2] = -0.2 * inputs.random_field((ny, nx), seed=10)
    prm = mc.params(g=G)
    P = orc.params(g=G)
    for bc, obc in ((mc.MC_BC_PERIODIC, orc.BC_PERIODIC), (mc.MC_BC_EXTRAP, orc.BC_EXTRAP)):
        dts = [2e-3, 1.5e-3, 1e-3]
        g, sm, _ = gu.run_steps(mc.MC_SW_ROE, mc.MC_F64, prm, q0, 1 / nx, 1 / ny, dts,
                                mc.MC_LIM_MC, bc)
        o, osm = _oracle_steps(orc, orc.SW_ROE, P, q0, 1 / nx, 1 / ny, dts, orc.LIM_MC, obc)
        assert np.all(gu.rel_inf(g, o) <= 1e-12), (bc, gu.rel_inf(g, o))


def test_tile_shape_and_roll_invariance(orc):
    """Results are bitwise independent of the rows-per-item tiling and
    bitwise equivariant under periodic shifts across tile seams."""
    nx, ny = 250, 190
    q0 = inputs.sw_dam_break(nx, ny=ny, seed=11)
    q0[1] = 0.3 * inputs.random_field((ny, nx), seed=12)
    prm = mc.params(g=G)
    dts = [1e-3] * 3
    ref, _, _ = gu.run_steps(mc.MC_SW_ROE, mc.MC_F64, prm, q0, 1 / nx, 1 / ny, dts,
                             mc.MC_LIM_MC, mc.MC_BC_PERIODIC, rows=64)
    for rows in (8, 13, 32, 100, 512):
        g, _, _ = gu.run_steps(mc.MC_SW_ROE, mc.MC_F64, prm, q0, 1 / nx, 1 / ny, dts,
                               mc.MC_LIM_MC, mc.MC_BC_PERIODIC, rows=rows)
        assert np.array_equal(g, ref), rows
    for sx, sy in ((1, 0), (0, 1), (29, 17), (61, 64)):
        qs = np.roll(np.roll(q0, sx, axis=2), sy, axis=1)
        g, _, _ = gu.run_steps(mc.MC_SW_ROE, mc.MC_F64, prm, qs, 1 / nx, 1 / ny, dts,
                               mc.MC_LIM_MC, mc.MC_BC_PERIODIC)
        assert np.array_equal(g, np.roll(np.roll(ref, sx, axis=2), sy, axis=1)), (sx, sy)


@pytest.mark.parametrize("solver,dtype", [(mc.MC_SW_ROE, mc.MC_F64), (mc.MC_ADVECTION, mc.MC_F32),
                                          (mc.MC_ACOUSTICS_VC, mc.MC_F64)])
def test_tune_rows(solver, dtype):
    """mc_tune_rows writes the step of q[cur] into the other buffer and
    nothing else (cur unchanged), keeps one of its candidates, and the steps
    that follow are bitwise those of an untuned context."""
    nx, ny = 301, 203
    print(f"case: mc_tune_rows solver {solver} dtype {dtype} {nx}x{ny}", flush=True)
    T = gu.npdt(dtype)
    m, _, na = mc.mc_solver_dims(solver)
    q0 = inputs.random_field((m, ny, nx), seed=21) + (2.0 if solver == mc.MC_SW_ROE else 0.0)
    aux = None
    if na:
        aux = np.stack([1.0 + inputs.random_field((ny, nx), seed=22, lo=0.0, hi=1.0),
                        0.5 + inputs.random_field((ny, nx), seed=23, lo=0.0, hi=1.0)])
    prm = mc.params(g=G, rho=1.0, K=1.0, u=0.7, v=-0.4)
    dt = 2e-4
    ref, _, _ = gu.run_steps(solver, dtype, prm, q0, 1 / nx, 1 / ny, [dt] * 3, mc.MC_LIM_MC,
                             mc.MC_BC_EXTRAP, aux=aux)
    one, _, _ = gu.run_steps(solver, dtype, prm, q0, 1 / nx, 1 / ny, [dt], mc.MC_LIM_MC,
                             mc.MC_BC_EXTRAP, aux=aux)
    a = gu.dev(q0, T)
    b = gu.empty(q0.shape, T)
    auxd = gu.dev(aux, T) if aux is not None else None
    with gu.context(solver, dtype, prm, nx, ny, 1 / nx, 1 / ny) as h:
        st = mc.state(a, b)
        rows = mc.mc_tune_rows(h, st, auxd, dt, mc.MC_LIM_MC, mc.MC_BC_EXTRAP)
        assert rows in (0, 16, 24, 32, 40, 48, 64, 96, 128, 192), rows
        assert st.cur == 0
        np.testing.assert_array_equal(gu.host(a), q0.astype(T))
        np.testing.assert_array_equal(gu.host(b), one.astype(T))
        for _ in range(3):
            mc.mc_step2d(h, st, auxd, dt, mc.MC_LIM_MC, mc.MC_BC_EXTRAP)
        g = gu.host(a if st.cur == 0 else b)
    np.testing.assert_array_equal(g, ref.astype(T))


@pytest.mark.parametrize("solver,dtype", [(mc.MC_ADVECTION, mc.MC_F64), (mc.MC_ACOUSTICS, mc.MC_F32),
                                          (mc.MC_ACOUSTICS_VC, mc.MC_F64), (mc.MC_EULER_ROE, mc.MC_F32)])
def test_row_variants_bitwise(solver, dtype):
    """The rows of a work item's interior run a variant of the row body
    without row conditions (and, for the light walkers, with buffer stores);
    items of 8 rows use it for a few rows, items of 1024 for almost all, and
    the results must be bitwise those of every other tiling."""
    nx, ny = 187, 233
    print(f"case: row variants solver {solver} dtype {dtype} {nx}x{ny}", flush=True)
    m, _, na = mc.mc_solver_dims(solver)
    if solver == mc.MC_EULER_ROE:
        q0, _ = inputs.euler_quadrants(nx, ny=ny, seed=5)
        prm = mc.params(gamma=1.4)
        dt = 2e-4
    else:
        q0 = inputs.random_field((m, ny, nx), seed=31)
        prm = mc.params(rho=1.0, K=1.0, u=0.8, v=-0.6)
        dt = 5e-4
    aux = None
    if na:
        aux = np.stack([1.0 + inputs.random_field((ny, nx), seed=32, lo=0.0, hi=1.0),
                        0.5 + inputs.random_field((ny, nx), seed=33, lo=0.0, hi=1.0)])
    for bc in (mc.MC_BC_PERIODIC, mc.MC_BC_EXTRAP):
        ref = None
        for rows in (8, 9, 10, 11, 37, 1024):
            g, _, _ = gu.run_steps(solver, dtype, prm, q0, 1 / nx, 1 / ny, [dt] * 3, mc.MC_LIM_MC, bc,
                                   rows=rows, aux=aux)
            if ref is None:
                ref = g
            else:
                np.testing.assert_array_equal(g, ref, err_msg=f"bc {bc} rows {rows}")


def test_max_speed_and_clock_rule(orc):
    """mc_max_speed equals the oracle pre-pass; the device clock reproduces
    the oracle's dt sequence, rejections included, and its final state."""
    n = 200
    q0 = inputs.sw_dam_break(n, seed=13)
    P = orc.params(g=G)
    for cfl_t, cfl_m, nst in ((0.9, 1.0, 20), (0.999, 1.0, 8)):
        prm = mc.params(g=G, cfl_target=cfl_t, cfl_max=cfl_m)
        qo, dts, t, nrej, _ = orc.run2d(orc.SW_ROE, P, q0, 1 / n, 1 / n, orc.LIM_MC,
                                        orc.BC_EXTRAP, cfl_t, cfl_m, nst)
        sm0, _ = orc.max_speed(orc.SW_ROE, P, q0, 1 / n, 1 / n, orc.BC_EXTRAP)
        a = gu.dev(q0)
        b = gu.empty(q0.shape)
        out = gu.struct_buf(16)
        clk = gu.struct_buf(ctypes.sizeof(mc.mc_clock))
        with gu.context(mc.MC_SW_ROE, mc.MC_F64, prm, n, n, 1 / n, 1 / n) as h:
            mc.mc_max_speed(h, a, None, mc.MC_BC_EXTRAP, out)
            assert abs(mc.cfl_from_tensor(out).smax - sm0) <= 1e-15 * sm0
            mc.mc_clock_init(h, clk, a, None, mc.MC_BC_EXTRAP)
            c = mc.clock_from_tensor(clk)
            assert abs(c.dt - cfl_t / sm0) <= 1e-15 * c.dt and c.cur == 0
            ts, acc = [], 0
            for _ in range(nst + nrej + 5):  # bounded: every attempt ends
                if acc >= nst:
                    break
                mc.mc_run2d(h, a, b, None, clk, 1, mc.MC_LIM_MC, mc.MC_BC_EXTRAP)
                c = mc.clock_from_tensor(clk)
                if c.n_acc > acc:
                    acc = c.n_acc
                    ts.append(c.t)
            res = gu.host(a if c.cur == 0 else b)
        assert acc == nst and c.n_rej == nrej, (acc, c.n_rej, nrej)
        if cfl_t > 0.99:
            assert nrej >= 1
        np.testing.assert_allclose(np.diff([0.0] + ts), dts, rtol=1e-12)
        assert np.all(gu.rel_inf(res, qo) <= 1e-10)


def test_run2d_graph_matches_eager(orc):
    n = 300
    q0 = inputs.sw_dam_break(n, seed=14)
    prm = mc.params(g=G)
    outs = []
    for use_graph in (False, True, True):
        a = gu.dev(q0)
        b = gu.empty(q0.shape)
        clk = gu.struct_buf(ctypes.sizeof(mc.mc_clock))
        with gu.context(mc.MC_SW_ROE, mc.MC_F64, prm, n, n, 1 / n, 1 / n) as h:
            mc.mc_clock_init(h, clk, a, None, mc.MC_BC_EXTRAP)
            for _ in range(3):  # replays with eager work and syncs in between
                mc.mc_run2d(h, a, b, None, clk, 5, mc.MC_LIM_MC, mc.MC_BC_EXTRAP, use_graph)
                gu.torch().cuda.synchronize()
            c = mc.clock_from_tensor(clk)
            outs.append((gu.host(a if c.cur == 0 else b), c.t, c.n_acc, c.n_rej))
    for o in outs:
        assert o[2] + o[3] == 15 and o[2] >= 13
    for o in outs[1:]:
        assert np.array_equal(o[0], outs[0][0]) and o[1:] == outs[0][1:]


def test_invalid_arguments_rejected():
    prm = mc.params()
    with gu.context(mc.MC_SW_ROE, mc.MC_F64, prm, 8, 8, 0.1, 0.1) as h:
        a = gu.empty((3, 8, 8))
        with pytest.raises(mc.ManyclawError):
            mc.mc_step2d(h, mc.state(a, a), None, 0.1, mc.MC_LIM_MC, mc.MC_BC_EXTRAP)
        with pytest.raises(mc.ManyclawError):
            mc.mc_step2d(h, mc.state(a, gu.empty((3, 8, 8))), None, -1.0, mc.MC_LIM_MC, 0)
        with pytest.raises(mc.ManyclawError):
            mc.mc_step2d(h, mc.state(a, gu.empty((3, 8, 8))), None, 0.1, 9, 0)
        with pytest.raises(mc.ManyclawError):
            mc.mc_step2d(h, mc.state(a, gu.empty((3, 8, 8))), None, 0.1, 4, 5)
        with pytest.raises(mc.ManyclawError):
            mc.mc_ctx_set_tile(h, 3)


def _window_oracle(orc, P, q, win, halo, dts, dx, dy):
    """Oracle values of the cells in win = (j0, j1, i0, i1) after len(dts)
    steps, computed on a sub-block padded by `halo` cells (clipped at the
    domain edge, where the oracle applies the same boundary rule)."""
    j0, j1, i0, i1 = win
    ny, nx = q.shape[1:]
    ja, jb = max(0, j0 - halo), min(ny, j1 + halo)
    ia, ib = max(0, i0 - halo), min(nx, i1 + halo)
    sub = q[:, ja:jb, ia:ib].copy()
    for dt in dts:
        sub, _, _ = orc.step2d(orc.SW_ROE, P, sub, dx, dy, dt, orc.LIM_MC, orc.BC_EXTRAP,
                               nthreads=8)
    return sub[:, j0 - ja:j1 - ja, i0 - ia:i1 - ia]


@pytest.mark.parametrize("dtype", [mc.MC_F64, mc.MC_F32])
def test_full_size_4096_sampled(orc, dtype):
    """The benchmark configuration (4096 x 4096 dam break, 50 steps) in the
    benchmark's launch shape: windows at corners, edges, the dam rim and the
    interior checked against the oracle on padded sub-blocks (the update of a
    cell after n steps depends only on cells within 2n); whole-grid
    property: positivity."""
    n, nst = 4096, 50
    print(f"full size {n}x{n} dtype={dtype} {nst} steps", flush=True)
    T = gu.npdt(dtype)
    q0 = inputs.sw_dam_break(n, seed=0).astype(T).astype(np.float64)
    P = orc.params(g=G)
    sm0, _ = orc.max_speed(orc.SW_ROE, P, q0, 1 / n, 1 / n, orc.BC_EXTRAP, nthreads=8)
    dt = 0.9 / sm0 * 0.85  # fixed dt below the CFL bound for the whole run
    dts = [dt] * nst
    prm = mc.params(g=G)
    g, sm, st = gu.run_steps(mc.MC_SW_ROE, dtype, prm, q0, 1 / n, 1 / n, dts, mc.MC_LIM_MC,
                             mc.MC_BC_EXTRAP)
    assert st == 0 and np.all(np.array(sm) * dt <= 1.0)
    assert g[0].min() > 0
    wins = [(0, 24, 0, 24), (0, 20, 4070, 4096), (4080, 4096, 2000, 2030),
            (2040, 2070, 0, 16), (2048 - 1229 - 12, 2048 - 1229 + 12, 2040, 2060),
            (1500, 1530, 1700, 1730), (3000, 3016, 3100, 3140)]
    for w in wins:
        o = _window_oracle(orc, P, q0, w, 2 * nst + 2, dts, 1 / n, 1 / n)
        gw = g[:, w[0]:w[1], w[2]:w[3]].astype(np.float64)
        if dtype == mc.MC_F64:
            err = gu.rel_inf(gw, o)
            assert np.all(err <= TOL100), (w, err)
        else:
            err = np.abs(gw - o).sum(axis=(1, 2)) / _l1_scales(o)
            assert np.all(err <= TOL32), (w, err)


def _l1_scales(o):
    """Per-field L1 scales of the FP32 comparisons: the depth's own L1 norm,
    and for the momenta the L1 norm of h sqrt(g h), the momentum a wave
    carries (a window's own momentum can sit at the level of the initial
    noise, far below the scale the arithmetic works at)."""
    h = np.abs(o[0])
    mom = (h * np.sqrt(G * h)).sum()
    return np.array([h.sum(), mom, mom])


@pytest.mark.parametrize("dtype", [mc.MC_F64, mc.MC_F32])
def test_full_size_4096_device_clock(orc, dtype):
    """The benchmark's own run: the 4096 x 4096 dam break, 50 steps at CFL 0.9
    under the device time-step rule (mc_clock_init, then mc_run2d replayed
    from a graph), against the oracle's full grid after its own 50 steps of
    the same rule, as many attempts as the oracle made (it rejects one step
    as the dam breaks).  The dt sequence (through the accepted count,
    rejections and the final time) and every cell are compared: FP64 per field in the
    max norm, FP32 (from the rounded initial state) per field in L1."""
    import os
    n, nst = 4096, 50
    print(f"full size {n}x{n} device clock dtype={dtype} {nst} steps", flush=True)
    T = gu.npdt(dtype)
    q0 = inputs.sw_dam_break(n, seed=0).astype(T).astype(np.float64)
    P = orc.params(g=G)
    nth = max(1, min(16, os.cpu_count() or 1))
    qo, dts, to, nrej, _ = orc.run2d(orc.SW_ROE, P, q0, 1 / n, 1 / n, orc.LIM_MC, orc.BC_EXTRAP,
                                     0.9, 1.0, nst, nthreads=nth)
    print(f"oracle done: t = {to!r}, rejected {nrej}", flush=True)
    prm = mc.params(g=G, cfl_target=0.9, cfl_max=1.0)
    a = gu.dev(q0, T)
    b = gu.empty(q0.shape, T)
    clk = gu.struct_buf(ctypes.sizeof(mc.mc_clock))
    with gu.context(mc.MC_SW_ROE, dtype, prm, n, n, 1 / n, 1 / n) as h:
        mc.mc_clock_init(h, clk, a, None, mc.MC_BC_EXTRAP)
        # the oracle's attempts: its accepted steps and its rejections
        mc.mc_run2d(h, a, b, None, clk, nst + nrej, mc.MC_LIM_MC, mc.MC_BC_EXTRAP, use_graph=True)
        c = mc.clock_from_tensor(clk)
        res = gu.host(a if c.cur == 0 else b).astype(np.float64)
        assert mc.mc_status_get(h) == 0
    assert c.n_rej == nrej and c.n_acc == nst, (nrej, c.n_rej, c.n_acc)
    if dtype == mc.MC_F64:
        assert abs(c.t - to) <= 1e-12 * to, (c.t, to)
        err = gu.rel_inf(res, qo)
        assert np.all(err <= TOL100), err
    else:
        assert abs(c.t - to) <= 1e-5 * to, (c.t, to)
        err = np.abs(res - qo).sum(axis=(1, 2)) / _l1_scales(qo)
        assert np.all(err <= TOL32), err
    print(f"max error per field {err}", flush=True)


def test_copy_probe():
    t = gu.torch()
    n = (1 << 20) + 48
    src = t.arange(n // 8, dtype=t.float64, device="cuda")
    dst = t.zeros_like(src)
    with gu.context(mc.MC_SW_ROE, mc.MC_F64, mc.params(), 8, 8, 1.0, 1.0) as h:
        mc.mc_copy_probe(h, dst, src, n)
        assert t.equal(gu.torch().as_tensor(gu.host(dst)), gu.torch().as_tensor(gu.host(src)))
        with pytest.raises(mc.ManyclawError):
            mc.mc_copy_probe(h, dst, src, 17)


@pytest.mark.parametrize("solver", ["ADVECTION", "ACOUSTICS", "ACOUSTICS_VC"])
@pytest.mark.parametrize("bc", ["PERIODIC", "EXTRAP"])
def test_linear_kernels_fp64_fp32(orc, solver, bc):
    """The paper's linear kernels (advection, constant- and variable-
    coefficient acoustics; the last in the four-block layered medium) on a
    256 x 192 grid, MC limiter, the oracle's CFL 0.9 dt sequence: FP64 after
    1 and 100 steps within 1e-12 and 1e-9, FP32 after 30 steps within
    relative L1 1e-5 of the oracle started from the rounded inputs."""
    nx, ny = 256, 192
    print(f"{solver} {bc} {nx}x{ny} fp64 + fp32", flush=True)
    sid, osid = getattr(mc, "MC_" + solver), getattr(orc, solver)
    B, OB = getattr(mc, "MC_BC_" + bc), getattr(orc, "BC_" + bc)
    pulse = inputs.acoustics_pulse(nx, ny=ny)
    if solver == "ADVECTION":
        q0 = pulse[:1].copy()
    else:
        q0 = pulse.copy()
        q0[1] = 0.05 * inputs.random_field((ny, nx), seed=11)
    aux = inputs.layered_medium(nx, ny=ny) if solver == "ACOUSTICS_VC" else None
    prm = mc.params(u=1.0, v=0.5, rho=1.0, K=1.0)
    P = orc.params(u=1.0, v=0.5, rho=1.0, K=1.0)
    dx, dy = 1 / nx, 1 / ny
    _, dts, _, _, _ = orc.run2d(osid, P, q0, dx, dy, orc.LIM_MC, OB, 0.9, 1.0, 100, aux=aux,
                                nthreads=8)
    g1, _, _ = gu.run_steps(sid, mc.MC_F64, prm, q0, dx, dy, dts[:1], mc.MC_LIM_MC, B, aux=aux)
    o1, _ = _oracle_steps(orc, osid, P, q0, dx, dy, dts[:1], orc.LIM_MC, OB, aux=aux)
    assert np.all(gu.rel_inf(g1, o1) <= TOL1), gu.rel_inf(g1, o1)
    g, sm, _ = gu.run_steps(sid, mc.MC_F64, prm, q0, dx, dy, dts, mc.MC_LIM_MC, B, aux=aux)
    o, osm = _oracle_steps(orc, osid, P, q0, dx, dy, dts, orc.LIM_MC, OB, aux=aux)
    assert np.all(gu.rel_inf(g, o) <= TOL100), gu.rel_inf(g, o)
    np.testing.assert_allclose(sm, osm, rtol=1e-13)
    # FP32: the device state and aux are FP32, the oracle starts from their values
    q32 = q0.astype(np.float32).astype(np.float64)
    a32 = None if aux is None else aux.astype(np.float32).astype(np.float64)
    g, _, _ = gu.run_steps(sid, mc.MC_F32, prm, q32, dx, dy, dts[:30], mc.MC_LIM_MC, B, aux=a32)
    o, _ = _oracle_steps(orc, osid, P, q32, dx, dy, dts[:30], orc.LIM_MC, OB, aux=a32)
    e = gu.rel_l1(g, o)
    print("fp32 rel L1", e, flush=True)
    assert np.all(e <= TOL32), e
