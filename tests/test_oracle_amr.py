"""Pins of the two-level refinement oracle (oracle/amr.py) against results
fixed by the method and by the plain oracle, not by the module itself:

  r = 1            refined patches of ratio 1 reproduce the plain split step
                   of the uniform grid (the C oracle) with any patch layout:
                   ghost exchange, padded sweeps, refluxing and averaging
                   down must all reduce to the identity
  whole domain     one patch covering a periodic domain at r = 2 equals r
                   plain steps of dt / r on the fine grid (every ghost cell
                   comes from the patch itself), and the coarse grid is its
                   average
  conservation     periodic domain, r = 2 and 4, patches touching each other
                   and the domain edge: the total of every field is constant
                   to round-off; without refluxing it is not (the fix-up is
                   what makes the coupling conservative)
  lake at rest     h constant, u = v = 0 stays so at r = 2 (to 1e-14 at r = 4,
                   where 3 F is rounded in the flux sums)
  interpolation    linear coarse data is reproduced exactly at fine ghost
                   centres; the r x r interpolated values of a coarse cell
                   average to it (limited slopes are centred in the cell)
  linear field     advection of q = a + b x + c y: the fine level is exact
                   (space and time interpolation of ghost values), the coarse
                   level exact away from the patch and, on the ring around
                   it, equal to the closed-form flux mismatch of the split
                   step at two time-step sizes
  other solvers    Euler (four quadrants), acoustics (pulse) and advection:
                   r = 1 reproduces the plain step for both boundary rules;
                   periodic totals are conserved with the fix-up (and drift
                   without it) at r = 2 and 4; a uniform Euler stream stays
                   uniform
"""
import numpy as np
import pytest

import oracle as O
from oracle import amr as A
from paper_1308_1464_amd import inputs

G = 9.81


def dam(nx, ny, seed=0):
    return inputs.sw_dam_break(nx, seed=seed, ny=ny)


def fine_ic(H, seed=0, moving=True):
    """the dam break sampled on the fine level, plus a smooth velocity"""
    r = H.r
    qf = inputs.sw_dam_break(H.nx * r, seed=seed, ny=H.ny * r)
    if moving:
        yy, xx = np.meshgrid((np.arange(H.ny * r) + 0.5) / (H.ny * r),
                             (np.arange(H.nx * r) + 0.5) / (H.nx * r), indexing="ij")
        qf[1] = qf[0] * 0.3 * np.sin(2 * np.pi * yy)
        qf[2] = qf[0] * 0.2 * np.cos(2 * np.pi * xx)
    return qf


def average(qf, r):
    m, NY, NX = qf.shape
    return qf.reshape(m, NY // r, r, NX // r, r).mean(axis=(2, 4))


BOXES = [(3, 4, 6, 5), (9, 4, 4, 3), (20, 10, 4, 8), (0, 16, 3, 4)]


@pytest.mark.parametrize("bc", [O.BC_PERIODIC, O.BC_EXTRAP])
def test_ratio_one_is_the_plain_step(bc):
    nx, ny = 28, 24
    H = A.Hierarchy(nx, ny, 1.0 / nx, 1.0 / ny, 1, BOXES, bc)
    q0 = fine_ic(H, 1)
    fine = A.restrict(H, q0)
    qc = q0.copy()
    qp = q0.copy()
    P = O.params(g=G)
    sm, _ = O.max_speed(O.SW_ROE, P, q0, H.dx, H.dy, bc)
    dt = 0.8 / sm
    for _ in range(3):
        qc, fine, smc, smf = A.step(H, qc, fine, dt, O.LIM_MC)
        qp, smp, _ = O.step2d(O.SW_ROE, P, qp, H.dx, H.dy, dt, O.LIM_MC, bc)
    assert np.abs(qc - qp).max() <= 1e-13 * np.abs(qp).max()
    for p, f in enumerate(A.restrict(H, qp)):
        assert np.abs(fine[p] - f).max() <= 1e-13 * np.abs(qp).max()
    assert abs(smc - smp) <= 1e-14 * smp


def test_whole_domain_patch_is_the_fine_grid():
    nx, ny, r = 12, 10, 2
    H = A.Hierarchy(nx, ny, 1.0 / nx, 1.0 / ny, r, [(0, 0, nx, ny)], O.BC_PERIODIC)
    qf = fine_ic(H, 2)
    qc = average(qf, r)
    P = O.params(g=G)
    sm, _ = O.max_speed(O.SW_ROE, P, qf, H.dx / r, H.dy / r, O.BC_PERIODIC)
    dt = r * 0.7 / sm
    qc1, fine, _, smf = A.step(H, qc, A.restrict(H, qf), dt, O.LIM_MC)
    ref = qf
    for _ in range(r):
        ref, smr, _ = O.step2d(O.SW_ROE, P, ref, H.dx / r, H.dy / r, dt / r, O.LIM_MC, O.BC_PERIODIC)
    assert np.abs(fine[0] - ref).max() <= 1e-13 * np.abs(ref).max()
    np.testing.assert_allclose(qc1, average(fine[0], r), rtol=1e-14, atol=0)


@pytest.mark.parametrize("r", [2, 4])
def test_conservation_needs_the_fix_up(r):
    nx, ny = 24, 20
    boxes = [(2, 3, 5, 4), (7, 3, 3, 6), (0, 12, 4, 5), (15, 14, 9, 6)]
    H = A.Hierarchy(nx, ny, 1.0 / nx, 1.0 / ny, r, boxes, O.BC_PERIODIC)
    qf = fine_ic(H, 3)
    qc0 = average(qf, r)
    fine0 = A.restrict(H, qf)
    P = O.params(g=G)
    sm, _ = O.max_speed(O.SW_ROE, P, qf, H.dx / r, H.dy / r, O.BC_PERIODIC)
    dt = r * 0.5 / sm
    tot0 = A.total(H, qc0)
    scale = np.abs(qc0).reshape(3, -1).sum(axis=1) * H.dx * H.dy
    drift = {}
    for reflux in (True, False):
        qc, fine = qc0.copy(), [f.copy() for f in fine0]
        for _ in range(4):
            qc, fine, _, _ = A.step(H, qc, fine, dt, O.LIM_MC, reflux=reflux)
        drift[reflux] = np.abs(A.total(H, qc) - tot0) / scale
    assert drift[True].max() < 1e-13, drift
    assert drift[False].max() > 1e-7, drift


@pytest.mark.parametrize("r", [2, 4])
def test_lake_at_rest(r):
    nx, ny = 16, 16
    H = A.Hierarchy(nx, ny, 1.0 / nx, 1.0 / ny, r, [(2, 2, 5, 4), (7, 2, 3, 3), (10, 9, 6, 7)],
                    O.BC_EXTRAP)
    qc = np.zeros((3, ny, nx))
    qc[0] = 1.7
    fine = [np.zeros((3,) + H.fine_shape(p)) for p in range(3)]
    for f in fine:
        f[0] = 1.7
    qc1, f1, _, _ = A.step(H, qc, fine, 0.01, O.LIM_MC)
    tol = 0.0 if r == 2 else 1e-14
    assert np.abs(qc1 - qc).max() <= tol * 1.7
    for a, b in zip(f1, fine):
        assert np.abs(a - b).max() <= tol * 1.7


def test_interpolation_linear_and_conservative():
    nx, ny, r = 10, 8, 4
    H = A.Hierarchy(nx, ny, 1.0 / nx, 1.0 / ny, r, [(3, 3, 2, 2)], O.BC_EXTRAP)
    j, i = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    qc = np.stack([1.0 + 0.25 * i + 0.5 * j, -0.125 * i, 0.375 * j + 0.0 * i])
    Gp = A.pad(qc, O.BC_EXTRAP)
    # fine ghost centres of the patch, away from the domain edge
    I = np.arange(3 * r - 2, 5 * r + 2)
    J = np.full_like(I, 3 * r - 1)
    v = A._interp(H, Gp, I, J)
    x = (I + 0.5) / r - 0.5
    y = (J + 0.5) / r - 0.5
    np.testing.assert_allclose(v[0], 1.0 + 0.25 * x + 0.5 * y, rtol=0, atol=1e-15)
    np.testing.assert_allclose(v[1], -0.125 * x, rtol=0, atol=1e-15)
    # conservative: any data, the r x r values of one coarse cell average to it
    rnd = inputs.rng(5).normal(size=(3, ny, nx))
    Gp = A.pad(rnd, O.BC_PERIODIC)
    jj, ii = np.meshgrid(np.arange(4 * r, 5 * r), np.arange(6 * r, 7 * r), indexing="ij")
    v = A._interp(H, Gp, ii.ravel(), jj.ravel())
    np.testing.assert_allclose(v.mean(axis=1), rnd[:, 4, 6], rtol=1e-14, atol=1e-15)


def test_interfaces_cover_every_coarse_fine_edge():
    nx, ny = 12, 10
    boxes = [(0, 0, 3, 3), (3, 0, 2, 2), (8, 5, 4, 5)]
    for bc in (O.BC_PERIODIC, O.BC_EXTRAP):
        H = A.Hierarchy(nx, ny, 0.1, 0.1, 2, boxes, bc)
        n = 0
        for (i, j, ent) in H.interfaces():
            assert H.owner[j, i] < 0
            n += sum(e is not None for e in ent)
        # count the coarse-fine edges directly
        ref = 0
        for j in range(ny):
            for i in range(nx):
                for di, dj in ((1, 0), (0, 1)):
                    a, b = i + di, j + dj
                    if bc == O.BC_PERIODIC:
                        a, b = a % nx, b % ny
                    elif a >= nx or b >= ny:
                        continue
                    if (H.owner[j, i] >= 0) != (H.owner[b, a] >= 0):
                        ref += 1
        assert n == ref


def test_overlapping_patches_rejected():
    with pytest.raises(ValueError):
        A.Hierarchy(8, 8, 0.1, 0.1, 2, [(0, 0, 4, 4), (3, 3, 2, 2)], O.BC_EXTRAP)
    with pytest.raises(ValueError):
        A.Hierarchy(8, 8, 0.1, 0.1, 2, [(6, 0, 4, 4)], O.BC_EXTRAP)


OTHERS = {"EULER_ROE": dict(gamma=1.4), "ACOUSTICS": dict(rho=1.3, K=0.8), "ADVECTION": dict(u=0.9, v=-0.6)}


def other_ic(solver, NX, NY, seed):
    """fine-level data [m][NY][NX] for the other covered solvers"""
    if solver == "EULER_ROE":
        q, _ = inputs.euler_quadrants(NX, seed=seed, ny=NY)
        return q
    if solver == "ACOUSTICS":
        q = inputs.acoustics_pulse(NX, NY, width=60.0)
        q[1] = 0.2 * inputs.random_field((NY, NX), seed=seed)
        return q
    return 1.0 + inputs.random_field((1, NY, NX), seed=seed)


@pytest.mark.parametrize("solver", sorted(OTHERS))
@pytest.mark.parametrize("bc", [O.BC_PERIODIC, O.BC_EXTRAP])
def test_other_solvers_ratio_one(solver, bc):
    sid, P = getattr(O, solver), O.params(**OTHERS[solver])
    nx, ny = 28, 24
    H = A.Hierarchy(nx, ny, 1.0 / nx, 1.0 / ny, 1, BOXES, bc)
    q0 = other_ic(solver, nx, ny, 5)
    fine = A.restrict(H, q0)
    qc, qp = q0.copy(), q0.copy()
    sm, _ = O.max_speed(sid, P, q0, H.dx, H.dy, bc)
    dt = 0.8 / sm
    for _ in range(3):
        qc, fine, smc, _ = A.step(H, qc, fine, dt, O.LIM_MC, solver=sid, P=P)
        qp, smp, _ = O.step2d(sid, P, qp, H.dx, H.dy, dt, O.LIM_MC, bc)
    assert np.abs(qc - qp).max() <= 1e-13 * np.abs(qp).max()
    for p, f in enumerate(A.restrict(H, qp)):
        assert np.abs(fine[p] - f).max() <= 1e-13 * np.abs(qp).max()
    assert abs(smc - smp) <= 1e-14 * smp


@pytest.mark.parametrize("solver", sorted(OTHERS))
@pytest.mark.parametrize("r", [2, 4])
def test_other_solvers_conservation(solver, r):
    sid, P = getattr(O, solver), O.params(**OTHERS[solver])
    nx, ny = 24, 20
    boxes = [(2, 3, 5, 4), (7, 3, 3, 6), (0, 12, 4, 5), (15, 14, 9, 6)]
    H = A.Hierarchy(nx, ny, 1.0 / nx, 1.0 / ny, r, boxes, O.BC_PERIODIC)
    qf = other_ic(solver, nx * r, ny * r, 7)
    qc0 = average(qf, r)
    fine0 = A.restrict(H, qf)
    sm, _ = O.max_speed(sid, P, qf, H.dx / r, H.dy / r, O.BC_PERIODIC)
    dt = r * 0.5 / sm
    m = qf.shape[0]
    tot0 = A.total(H, qc0)
    scale = np.abs(qc0).reshape(m, -1).sum(axis=1) * H.dx * H.dy
    drift = {}
    for reflux in (True, False):
        qc, fine = qc0.copy(), [f.copy() for f in fine0]
        for _ in range(3):
            qc, fine, _, _ = A.step(H, qc, fine, dt, O.LIM_MC, solver=sid, P=P, reflux=reflux)
        # a field that starts at zero (acoustics: v) is measured against the others
        drift[reflux] = np.abs(A.total(H, qc) - tot0) / np.maximum(scale, 1e-3 * scale.max())
    assert drift[True].max() < 1e-13, drift
    assert drift[False].max() > 1e-9, drift


@pytest.mark.parametrize("r", [2, 4])
def test_euler_uniform_stream(r):
    P = O.params(gamma=1.4)
    nx, ny = 16, 16
    H = A.Hierarchy(nx, ny, 1.0 / nx, 1.0 / ny, r, [(2, 2, 5, 4), (7, 2, 3, 3), (10, 9, 6, 7)], O.BC_PERIODIC)
    state = np.array([1.2, 1.2 * 0.3, 1.2 * -0.2, 0.9 / 0.4 + 0.5 * 1.2 * (0.09 + 0.04)])
    qc = np.broadcast_to(state[:, None, None], (4, ny, nx)).copy()
    fine = [np.broadcast_to(state[:, None, None], (4,) + H.fine_shape(p)).copy() for p in range(3)]
    qc1, f1, _, _ = A.step(H, qc, fine, 0.01, O.LIM_MC, solver=O.EULER_ROE, P=P)
    tol = 1e-14
    assert np.abs(qc1 - qc).max() <= tol * np.abs(state).max()
    for a, b in zip(f1, fine):
        assert np.abs(a - b).max() <= tol * np.abs(state).max()


@pytest.mark.parametrize("r", [2, 4])
def test_linear_field_advected_exactly(r):
    """Constant-velocity advection of a linear field q = a + b x + c y.

    Fine level: exact to round-off.  Every part of the patch's sub-steps is
    exact on this data: the MC-limited split sweeps (theta = 1 gives the
    Lax-Wendroff correction), the limited linear interpolation of coarse data
    in space, and the linear interpolation of ghost values in time between
    the coarse states at t and t + dt (the solution is linear in t).  Ghost
    values frozen at time t, or a wrong space slope or time weight, leave an
    error of the size of the field's change over one fine step.

    Coarse level: exact away from the patch, and on the one-cell ring around
    it equal to a closed form.  In a split step the y-sweep reads the
    x-swept state: the coarse y-flux of an edge sees the x-shift u dt of a
    whole step, r fine y-fluxes see on average (r + 1)/(2r) of it; likewise
    a fine x-flux sees on average (r - 1)/(2r) of the y-shift v dt, the
    coarse x-flux none.  Refluxing puts those differences into the ring:
        below / above the patch   -/+ v b u dt (r - 1)/(2r) * dt/dy
        left / right of it        +/- u c v dt (r - 1)/(2r) * dt/dx
    and nothing into its corner cells.  The domain edge is far enough that
    its own boundary error cannot reach the checked cells in one step."""
    u, v = 0.9, -0.6
    P = O.params(u=u, v=v)
    n = 32
    i0, j0, w, h = 12, 11, 8, 9
    H = A.Hierarchy(n, n, 1.0 / n, 1.0 / n, r, [(i0, j0, w, h)], O.BC_EXTRAP)
    a, b, c = 1.5, 0.8, -0.45

    def field(N, t):
        x = (np.arange(N) + 0.5) / N
        X, Y = np.meshgrid(x, x)
        return (a + b * (X - u * t) + c * (Y - v * t))[None]

    qc = field(n, 0.0)
    fine = A.restrict(H, field(n * r, 0.0))
    dt = 0.4 / n / max(abs(u), abs(v))        # Courant number 0.4 on the coarse grid
    qc1, f1, _, _ = A.step(H, qc, fine, dt, O.LIM_MC, solver=O.ADVECTION, P=P)
    tol = 1e-13 * np.abs(qc).max()
    for got, want in zip(f1, A.restrict(H, field(n * r, dt))):
        assert np.abs(got - want).max() <= tol

    err = (qc1 - field(n, dt))[0]
    k = (r - 1) / (2.0 * r)
    ey = v * b * u * dt * k * (dt * n)
    ex = u * c * v * dt * k * (dt * n)
    want = np.zeros((n, n))
    want[j0 - 1, i0:i0 + w] = -ey
    want[j0 + h, i0:i0 + w] = ey
    want[j0:j0 + h, i0 - 1] = ex
    want[j0:j0 + h, i0 + w] = -ex
    inner = (slice(6, n - 6), slice(6, n - 6))
    assert abs(ey) > 1e-4 and abs(ex) > 1e-4
    assert np.abs(err[inner] - want[inner]).max() <= tol
