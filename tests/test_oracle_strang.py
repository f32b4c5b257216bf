"""Pins of the Strang-splitting oracle (oracle/strang.py) against closed
forms and the plain C oracle:

  Fourier mode   phi = 1 acoustics: one Strang step multiplies a mode by
                 G_x(nu/2) G_y(nu) G_x(nu/2), the Lax-Wendroff matrices of
                 the three sweeps (the Godunov step gives G_y G_x)
  plain step     the module's x-then-y composition equals the C oracle's
                 mco_step2d (shallow water, Euler, variable-coefficient
                 acoustics with aux), which pins its sweep
  halving        data that do not vary in y: the y-sweep is an exact no-op,
                 so a Strang step equals two C-oracle steps of dt/2
  convergence    smooth acoustics pulse, phi = 1, against the exact periodic
                 solution: order >= 1.8 (on this problem the Godunov step's
                 splitting error is below the spatial error too, so the
                 order alone does not tell the two apart; the Fourier-mode
                 pin does)
  conservation   periodic shallow water: totals constant to round-off
"""
import numpy as np
import pytest

import exact
import oracle as O
from oracle import strang as St
from paper_1308_1464_amd import inputs

G = 9.81


def test_fourier_mode_amplification():
    rho, K = 1.0, 1.0
    nx, ny = 32, 24
    dx, dy = 1.0 / nx, 1.0 / ny
    dt = 0.8 * min(dx, dy)
    xi, eta = 2 * np.pi * 3 / nx, 2 * np.pi * 2 / ny
    P = O.params(rho=rho, K=K)
    v0 = np.array([0.4 - 0.3j, 0.6 + 0.1j, -0.2 + 0.5j])
    I, J = np.meshgrid(np.arange(nx), np.arange(ny))
    mode = np.exp(1j * (xi * I + eta * J))
    q = np.real(v0[:, None, None] * mode[None])
    q1, sm = St.strang_step(O.ACOUSTICS, P, q, dx, dy, dt, O.LIM_NONE, O.BC_PERIODIC)
    Gxh = exact.lw_matrix_factor(exact.acoustics_matrix_x(rho, K), 0.5 * dt / dx, xi)
    Gy = exact.lw_matrix_factor(exact.acoustics_matrix_y(rho, K), dt / dy, eta)
    ref = np.real((Gxh @ Gy @ Gxh @ v0)[:, None, None] * mode[None])
    np.testing.assert_allclose(q1, ref, rtol=0, atol=1e-13)
    assert sm == pytest.approx(max(0.5 / dx, 1.0 / dy), rel=1e-15)


@pytest.mark.parametrize("case", ["sw", "euler", "vc"])
@pytest.mark.parametrize("bc", [O.BC_PERIODIC, O.BC_EXTRAP])
def test_composition_matches_plain_step(case, bc):
    n = 24
    aux = None
    if case == "sw":
        solver, P = O.SW_ROE, O.params(g=G)
        q = inputs.sw_dam_break(n, seed=3)
        q[1] = 0.2 * q[0] * inputs.random_field((n, n), seed=4)
    elif case == "euler":
        solver, P = O.EULER_ROE, O.params(gamma=1.4)
        q, _ = inputs.euler_quadrants(n, seed=5)
    else:
        solver, P = O.ACOUSTICS_VC, O.params()
        q = inputs.acoustics_pulse(n)
        aux = inputs.layered_medium(n)
    dt = 0.3 / n
    a, sa = St.godunov_step(solver, P, q, 1.0 / n, 1.0 / n, dt, O.LIM_MC, bc, aux)
    b, sb, _ = O.step2d(solver, P, q, 1.0 / n, 1.0 / n, dt, O.LIM_MC, bc, aux=aux)
    np.testing.assert_array_equal(a, b)
    assert sa == sb


def test_y_invariant_data_is_two_half_steps():
    n = 40
    q = inputs.sw_dam_break(n, seed=6)
    q = np.repeat(q[:, :1, :], n, axis=1) * 0 + q[:, n // 2:n // 2 + 1, :]   # one row, repeated
    q[1] = 0.3 * q[0]
    q[2] = -0.1 * q[0]
    P = O.params(g=G)
    dt = 0.4 / n
    a, _ = St.strang_step(O.SW_ROE, P, q, 1.0 / n, 1.0 / n, dt, O.LIM_MC, O.BC_EXTRAP)
    b = q
    for _ in range(2):
        b, _, _ = O.step2d(O.SW_ROE, P, b, 1.0 / n, 1.0 / n, 0.5 * dt, O.LIM_MC, O.BC_EXTRAP)
    np.testing.assert_array_equal(a, b)


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
            a, _ = St.strang_step(O.ACOUSTICS, P, a, 1.0 / n, 1.0 / n, dt, O.LIM_NONE, O.BC_PERIODIC)
        ref = exact.acoustics_spectral(q0[0], T, 1.0, 1.0)
        es.append(np.abs(a[0] - ref[0]).mean())
    order_s = np.log2(np.array(es[:-1]) / np.array(es[1:]))
    assert np.all(order_s >= 1.8), (es, order_s)


def test_conservation_periodic():
    n = 32
    q = inputs.sw_dam_break(n, seed=8)
    q[1] = 0.2 * q[0] * inputs.random_field((n, n), seed=9)
    P = O.params(g=G)
    s0 = q.reshape(3, -1).sum(axis=1)
    for _ in range(6):
        q, _ = St.strang_step(O.SW_ROE, P, q, 1.0 / n, 1.0 / n, 0.4 / (n * 5.0), O.LIM_MC, O.BC_PERIODIC)
    s1 = q.reshape(3, -1).sum(axis=1)
    scale = np.abs(q).reshape(3, -1).sum(axis=1)
    assert (np.abs(s1 - s0) / scale).max() < 1e-14
