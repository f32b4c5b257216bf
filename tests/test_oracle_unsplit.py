"""Pins of the unsplit (transverse-propagation) oracle (oracle/unsplit.py)
against closed forms, the plain C oracle and invariants:

  donor cell     first-order advection, every sign pair of (u, v): the
                 unsplit step with transverse propagation equals the
                 product of the two one-dimensional upwind steps, i.e. the
                 C oracle's Godunov split step (LeVeque 2002, section 20.5)
  Fourier mode   advection, phi = 1, u, v > 0: a mode is multiplied by
                 1 - a(1 - e^-ix) - a(1 - a)(cos x - 1) - b(1 - e^-iy)
                 - b(1 - b)(cos y - 1) + a b (1 - e^-ix)(1 - e^-iy),
                 a = u dt/dx, b = v dt/dy
  y-invariant    data that do not vary in y: the y-edges carry nothing and
                 the transverse corrections cancel, so the step is the
                 C oracle's x-sweep (shallow water, acoustics)
  symmetry       transposing the data (momenta swapped) transposes the
                 result: the unsplit step treats x and y alike
  conservation   periodic shallow water, totals constant to round-off
  lake at rest   constant depth at rest stays so
  convergence    smooth acoustics pulse against the exact periodic solution,
                 order >= 1.8
"""
import numpy as np
import pytest

import exact
import oracle as O
from oracle import unsplit as U
from paper_1308_1464_amd import inputs

G = 9.81


@pytest.mark.parametrize("u,v", [(1.0, 0.5), (1.0, -0.5), (-0.7, 0.4), (-0.6, -0.9)])
def test_first_order_advection_is_donor_cell_product(u, v):
    nx, ny = 30, 26
    q = inputs.random_field((1, ny, nx), seed=3)
    P = O.params(u=u, v=v)
    dt = 0.9 / max(abs(u) * nx, abs(v) * ny)
    for bc in (O.BC_PERIODIC, O.BC_EXTRAP):
        a, sa = U.unsplit_step(O.ADVECTION, P, q, 1 / nx, 1 / ny, dt, O.LIM_FIRST_ORDER, bc)
        b, sb, _ = O.step2d(O.ADVECTION, P, q, 1 / nx, 1 / ny, dt, O.LIM_FIRST_ORDER, bc)
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-14)
        assert sa == sb


def test_fourier_mode_advection():
    nx, ny = 32, 24
    u, v = 1.0, 0.6
    dx, dy = 1.0 / nx, 1.0 / ny
    dt = 0.7 * min(dx / u, dy / v)
    a, b = u * dt / dx, v * dt / dy
    xi, eta = 2 * np.pi * 3 / nx, 2 * np.pi * 2 / ny
    I, J = np.meshgrid(np.arange(nx), np.arange(ny))
    mode = np.exp(1j * (xi * I + eta * J))
    c0 = 0.8 - 0.3j
    q = np.real(c0 * mode)[None]
    q1, _ = U.unsplit_step(O.ADVECTION, O.params(u=u, v=v), q, dx, dy, dt, O.LIM_NONE, O.BC_PERIODIC)
    ex, ey = 1 - np.exp(-1j * xi), 1 - np.exp(-1j * eta)
    g = 1 - a * ex - a * (1 - a) * (np.cos(xi) - 1) - b * ey - b * (1 - b) * (np.cos(eta) - 1) + a * b * ex * ey
    np.testing.assert_allclose(q1[0], np.real(g * c0 * mode), rtol=0, atol=1e-14)


@pytest.mark.parametrize("case", ["sw", "acoustics"])
def test_y_invariant_data_is_the_x_sweep(case):
    n = 36
    if case == "sw":
        solver, P = O.SW_ROE, O.params(g=G)
        row = inputs.sw_dam_break(n, seed=4)[:, n // 2:n // 2 + 1, :]
        q = np.repeat(row, n, axis=1)
        q[1] = 0.4 * q[0]
        q[2] = -0.2 * q[0]
    else:
        solver, P = O.ACOUSTICS, O.params(rho=1.0, K=1.0)
        q = np.repeat(inputs.acoustics_pulse(n)[:, n // 2:n // 2 + 1, :], n, axis=1)
        q[2] = 0.3 * q[0]
    dt = 0.1 / n
    for bc in (O.BC_PERIODIC, O.BC_EXTRAP):
        a, _ = U.unsplit_step(solver, P, q, 1 / n, 1 / n, dt, O.LIM_MC, bc)
        b, _, _ = O.step2d(solver, P, q, 1 / n, 1 / n, dt, O.LIM_MC, bc)
        np.testing.assert_allclose(a, b, rtol=0, atol=1e-14 * np.abs(b).max())


def test_transposition_symmetry():
    nx, ny = 28, 22
    q = inputs.sw_dam_break(nx, seed=5, ny=ny)
    q[1] = 0.3 * q[0] * inputs.random_field((ny, nx), seed=6)
    q[2] = 0.2 * q[0] * inputs.random_field((ny, nx), seed=7)
    P = O.params(g=G)
    dt = 0.002
    a, sa = U.unsplit_step(O.SW_ROE, P, q, 1 / nx, 1 / ny, dt, O.LIM_MC, O.BC_EXTRAP)
    qt = np.ascontiguousarray(np.stack([q[0].T, q[2].T, q[1].T]))
    b, sb = U.unsplit_step(O.SW_ROE, P, qt, 1 / ny, 1 / nx, dt, O.LIM_MC, O.BC_EXTRAP)
    bt = np.stack([b[0].T, b[2].T, b[1].T])
    np.testing.assert_allclose(a, bt, rtol=0, atol=1e-13 * np.abs(a).max())
    assert sa == pytest.approx(sb, rel=1e-15)


def test_conservation_and_lake_at_rest():
    n = 32
    q = inputs.sw_dam_break(n, seed=8)
    q[1] = 0.2 * q[0] * inputs.random_field((n, n), seed=9)
    P = O.params(g=G)
    s0 = q.reshape(3, -1).sum(axis=1)
    for _ in range(5):
        q, sm = U.unsplit_step(O.SW_ROE, P, q, 1 / n, 1 / n, 0.002, O.LIM_MC, O.BC_PERIODIC)
    s1 = q.reshape(3, -1).sum(axis=1)
    assert (np.abs(s1 - s0) / np.abs(q).reshape(3, -1).sum(axis=1)).max() < 1e-14
    lake = np.zeros((3, n, n))
    lake[0] = 1.3
    out, _ = U.unsplit_step(O.SW_ROE, P, lake, 1 / n, 1 / n, 0.01, O.LIM_MC, O.BC_EXTRAP)
    np.testing.assert_array_equal(out, lake)


def test_converges_at_second_order():
    P = O.params(rho=1.0, K=1.0)
    T = 0.15
    es = []
    for n in (32, 64, 128):
        q0 = inputs.acoustics_pulse(n, width=50.0)
        nst = int(np.ceil(T / (0.8 / n)))
        dt = T / nst
        a = q0
        for _ in range(nst):
            a, _ = U.unsplit_step(O.ACOUSTICS, P, a, 1.0 / n, 1.0 / n, dt, O.LIM_NONE, O.BC_PERIODIC)
        ref = exact.acoustics_spectral(q0[0], T, 1.0, 1.0)
        es.append(np.abs(a[0] - ref[0]).mean())
    order = np.log2(np.array(es[:-1]) / np.array(es[1:]))
    assert np.all(order >= 1.8), (es, order)


def test_unsupported_solver():
    with pytest.raises(ValueError):
        U.unsplit_step(O.EULER_ROE, O.params(), np.ones((4, 8, 8)), 0.1, 0.1, 0.01, O.LIM_MC, 0)
