"""Pins of the oracle's Riemann solvers against mathematics, not against the
oracle itself: flux-difference (Roe) identities with independently written
physical fluxes, eigenvector relations, the exact acoustics middle state,
mirror symmetry and component permutation."""
import numpy as np
import pytest

import exact
from paper_1308_1464_amd import inputs

G = 9.81
GAMMA = 1.4


def rel(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


def _perm_xy(q):
    """swap the two velocity/momentum slots (1 <-> 2)"""
    r = q.copy()
    r[1], r[2] = q[2].copy(), q[1].copy()
    return r


# ------------------------------------------------------------ advection
def test_advection_wave_is_jump(orc):
    P = orc.params(u=0.7, v=-1.3)
    ql = inputs.random_field((1, 1000), seed=1)
    qr = inputs.random_field((1, 1000), seed=2)
    for ixy, a in ((1, 0.7), (2, -1.3)):
        W, s, am, ap, st = orc.rp2(orc.ADVECTION, P, ixy, ql, qr)
        assert st == 0
        np.testing.assert_array_equal(W[0], qr - ql)
        np.testing.assert_array_equal(s[0], np.full(1000, a))
        np.testing.assert_array_equal(am + ap, a * (qr - ql))
        assert np.all(am == (min(a, 0.0) * (qr - ql)))


# ------------------------------------------------------------ acoustics
@pytest.mark.parametrize("rho,K", [(1.0, 1.0), (2.5, 0.4)])
def test_acoustics_middle_state_and_eigen(orc, rho, K):
    P = orc.params(rho=rho, K=K)
    ql, qr = inputs.acoustics_random_states(20000, seed=3)
    W, s, am, ap, st = orc.rp2(orc.ACOUSTICS, P, 1, ql, qr)
    c = np.sqrt(K / rho)
    np.testing.assert_allclose(s[0], -c, rtol=0, atol=0)
    np.testing.assert_allclose(s[1], c, rtol=0, atol=0)
    # exact Riemann middle state is qL + W1
    pm, um = exact.acoustics_middle_state(ql[0], ql[1], qr[0], qr[1], rho, K)
    assert rel(ql[0] + W[0][0], pm) < 1e-13
    assert rel(ql[1] + W[0][1], um) < 1e-13
    # eigenvector relation A W_p = s_p W_p
    A = exact.acoustics_matrix_x(rho, K)
    for p in range(2):
        assert rel(A @ W[p], s[p] * W[p]) < 1e-13
    # sum of waves is the jump in (p, u); flux difference A dq
    dq = qr - ql
    assert rel((W[0] + W[1])[:2], dq[:2]) < 1e-13
    assert rel(am + ap, A @ dq) < 1e-13


def test_acoustics_y_is_permuted_x(orc):
    P = orc.params(rho=1.3, K=2.0)
    ql, qr = inputs.acoustics_random_states(5000, seed=4)
    Wx, sx, amx, apx, _ = orc.rp2(orc.ACOUSTICS, P, 1, ql, qr)
    Wy, sy, amy, apy, _ = orc.rp2(orc.ACOUSTICS, P, 2, _perm_xy(ql), _perm_xy(qr))
    np.testing.assert_array_equal(sx, sy)
    for p in range(2):
        np.testing.assert_array_equal(_perm_xy(Wx[p]), Wy[p])
    np.testing.assert_array_equal(_perm_xy(amx), amy)
    np.testing.assert_array_equal(_perm_xy(apx), apy)
    # y-direction eigen relation with the y matrix
    A = exact.acoustics_matrix_y(1.3, 2.0)
    for p in range(2):
        assert rel(A @ Wy[p], sy[p] * Wy[p]) < 1e-13


def test_acoustics_vc_reduces_and_interface(orc):
    rho, K = 1.7, 0.6
    c = np.sqrt(K / rho)
    P = orc.params(rho=rho, K=K)
    ql, qr = inputs.acoustics_random_states(4000, seed=5)
    aux_same = np.stack([np.stack([np.full(4000, rho), np.full(4000, c)])] * 2)
    W1, s1, am1, ap1, _ = orc.rp2(orc.ACOUSTICS_VC, P, 1, ql, qr, aux_same)
    W0, s0, am0, ap0, _ = orc.rp2(orc.ACOUSTICS, P, 1, ql, qr)
    assert rel(W1, W0) < 1e-14 and rel(am1, am0) < 1e-14 and rel(ap1, ap0) < 1e-14
    # different materials: left wave is an eigenvector of the left matrix,
    # right wave of the right matrix, and the waves sum to the jump
    g = inputs.rng(6)
    rl, rr = g.uniform(0.5, 3, 4000), g.uniform(0.5, 3, 4000)
    cl, cr = g.uniform(0.5, 3, 4000), g.uniform(0.5, 3, 4000)
    aux = np.stack([np.stack([rl, cl]), np.stack([rr, cr])])
    W, s, am, ap, _ = orc.rp2(orc.ACOUSTICS_VC, P, 1, ql, qr, aux)
    assert rel(W[0][:2] + W[1][:2], (qr - ql)[:2]) < 1e-13
    np.testing.assert_allclose(W[0][0], -rl * cl * W[0][1], rtol=1e-14, atol=1e-14)
    np.testing.assert_allclose(W[1][0], rr * cr * W[1][1], rtol=1e-14, atol=1e-14)
    np.testing.assert_array_equal(s[0], -cl)
    np.testing.assert_array_equal(s[1], cr)


# ------------------------------------------------------------ shallow water
def _sw_states(n=100000, seed=7):
    return inputs.sw_random_states(n, seed=seed, hlo=1e-2, hhi=10.0, ulim=5.0)


@pytest.mark.parametrize("solver", ["SW_ROE", "SW_HLLE"])
def test_sw_flux_difference_identity(orc, solver):
    sid = getattr(orc, solver)
    P = orc.params(g=G)
    ql, qr = _sw_states()
    W, s, am, ap, st = orc.rp2(sid, P, 1, ql, qr)
    df = exact.sw_flux_x(qr, G) - exact.sw_flux_x(ql, G)
    sw = sum(s[p] * W[p] for p in range(3))
    scale = np.max(np.abs(df), axis=0) + np.max(np.abs(sw), axis=0)
    # Roe identity: sum_p s_p W_p = f(qR) - f(qL); the fluctuations add up to it
    assert np.max(np.abs(sw - df) / scale) < 1e-12
    assert np.max(np.abs(am + ap - df) / scale) < 1e-12
    # waves add up to the jump
    dq = qr - ql
    assert np.max(np.abs(sum(W) - dq) / (np.max(np.abs(dq), axis=0) + 1e-300)) < 1e-12


def test_sw_roe_eigenstructure(orc):
    P = orc.params(g=G)
    ql, qr = _sw_states(20000, seed=8)
    W, s, am, ap, _ = orc.rp2(orc.SW_ROE, P, 1, ql, qr)
    hl, hr = ql[0], qr[0]
    ul, ur = ql[1] / hl, qr[1] / hr
    vl, vr = ql[2] / hl, qr[2] / hr
    # Roe speeds: u_hat -/+ sqrt(g (hL+hR)/2)
    uh = (np.sqrt(hl) * ul + np.sqrt(hr) * ur) / (np.sqrt(hl) + np.sqrt(hr))
    vh = (np.sqrt(hl) * vl + np.sqrt(hr) * vr) / (np.sqrt(hl) + np.sqrt(hr))
    ch = np.sqrt(G * 0.5 * (hl + hr))
    assert rel(s[0], uh - ch) < 1e-13 and rel(s[1], uh) < 1e-13 and rel(s[2], uh + ch) < 1e-13
    # eigenvectors of the Roe matrix: (1, u-c, v), (0, 0, 1), (1, u+c, v)
    assert rel(W[0][1], W[0][0] * (uh - ch)) < 1e-12
    assert rel(W[0][2], W[0][0] * vh) < 1e-12
    assert np.all(W[1][0] == 0) and np.all(W[1][1] == 0)
    assert rel(W[2][1], W[2][0] * (uh + ch)) < 1e-12


def test_sw_roe_no_fix_when_not_transonic(orc):
    """Away from transonic rarefactions the fluctuations are the plain
    upwind split sum_p min/max(s_p, 0) W_p."""
    P = orc.params(g=G)
    ql, qr = inputs.sw_random_states(20000, seed=9, hlo=1.0, hhi=2.0, ulim=0.5)
    W, s, am, ap, _ = orc.rp2(orc.SW_ROE, P, 1, ql, qr)
    am_ref = sum(np.minimum(s[p], 0) * W[p] for p in range(3))
    ap_ref = sum(np.maximum(s[p], 0) * W[p] for p in range(3))
    assert rel(am, am_ref) < 1e-12 and rel(ap, ap_ref) < 1e-12


def test_sw_mirror_swaps_fluctuations(orc):
    """x -> -x maps (qL, qR) to (M qR, M qL) with M = diag(1,-1,1); the
    left-going fluctuation of the mirrored problem is M times the right-going
    one of the original (holds with the entropy fix too)."""
    P = orc.params(g=G)
    ql, qr = _sw_states(50000, seed=10)
    M = np.array([1.0, -1.0, 1.0])[:, None]
    for sid in (orc.SW_ROE, orc.SW_HLLE):
        _, _, am, ap, _ = orc.rp2(sid, P, 1, ql, qr)
        _, _, am2, ap2, _ = orc.rp2(sid, P, 1, M * qr, M * ql)
        scale = np.max(np.abs(am) + np.abs(ap), axis=0) + 1e-300
        assert np.max(np.abs(am2 - M * ap) / scale) < 1e-12
        assert np.max(np.abs(ap2 - M * am) / scale) < 1e-12


def test_sw_transonic_fix_active_and_continuous(orc):
    """A transonic left-going rarefaction: the fix changes amdq from the
    plain split, keeps amdq + apdq, and is continuous across the sonic
    boundary (a tiny change of state changes the fluctuation a tiny amount)."""
    P = orc.params(g=G)
    hl, hr = 4.0, 1.0
    ul = np.linspace(-8.0, 8.0, 4001)
    ql = np.stack([np.full_like(ul, hl), hl * ul, np.zeros_like(ul)])
    qr = np.stack([np.full_like(ul, hr), hr * (ul + 3.0), np.zeros_like(ul)])
    W, s, am, ap, _ = orc.rp2(orc.SW_ROE, P, 1, ql, qr)
    am_plain = sum(np.minimum(s[p], 0) * W[p] for p in range(3))
    changed = np.max(np.abs(am - am_plain), axis=0) > 1e-9
    assert changed.any()
    # continuity in ul: neighbouring samples differ by O(step)
    jump = np.max(np.abs(np.diff(am, axis=1)))
    assert jump < 1.0
    df = exact.sw_flux_x(qr, G) - exact.sw_flux_x(ql, G)
    assert rel(am + ap, df) < 1e-12


def test_sw_zero_jump_gives_zero(orc):
    P = orc.params(g=G)
    ql, _ = _sw_states(1000, seed=11)
    W, s, am, ap, _ = orc.rp2(orc.SW_ROE, P, 1, ql, ql.copy())
    assert np.all(W == 0) and np.all(am == 0) and np.all(ap == 0)
    # HLLE forms q* = (sR q - sL q)/(sR - sL): zero up to rounding only
    W, s, am, ap, _ = orc.rp2(orc.SW_HLLE, P, 1, ql, ql.copy())
    assert np.max(np.abs(W) / np.max(np.abs(ql), axis=0)) < 1e-15


def test_sw_y_is_permuted_x(orc):
    P = orc.params(g=G)
    ql, qr = _sw_states(20000, seed=12)
    for sid in (orc.SW_ROE, orc.SW_HLLE):
        Wx, sx, amx, apx, _ = orc.rp2(sid, P, 1, ql, qr)
        Wy, sy, amy, apy, _ = orc.rp2(sid, P, 2, _perm_xy(ql), _perm_xy(qr))
        np.testing.assert_array_equal(sx, sy)
        for p in range(3):
            np.testing.assert_array_equal(_perm_xy(Wx[p]), Wy[p])
        np.testing.assert_array_equal(_perm_xy(amx), amy)
        np.testing.assert_array_equal(_perm_xy(apx), apy)


def test_sw_small_jump_limit(orc):
    """As the jump goes to zero, amdq -> A^-(q) dq with A^- from the exact
    Jacobian's eigen-decomposition (linearisation consistency)."""
    P = orc.params(g=G)
    q0 = np.array([1.5, 0.9, -0.4])
    eps = 1e-7
    d = np.array([0.3, -0.7, 0.5])
    ql = (q0 - 0.5 * eps * d)[:, None]
    qr = (q0 + 0.5 * eps * d)[:, None]
    _, _, am, ap, _ = orc.rp2(orc.SW_ROE, P, 1, ql, qr)
    h, u, v = q0[0], q0[1] / q0[0], q0[2] / q0[0]
    c = np.sqrt(G * h)
    J = np.array([[0, 1, 0], [c * c - u * u, 2 * u, 0], [-u * v, v, u]])
    lam, R = np.linalg.eig(J)
    Am = (R @ np.diag(np.minimum(lam.real, 0)) @ np.linalg.inv(R)).real
    np.testing.assert_allclose(am[:, 0] / eps, Am @ d, rtol=1e-5, atol=1e-6)


# ------------------------------------------------------------ Euler
def test_euler_flux_difference_identity(orc):
    P = orc.params(gamma=GAMMA)
    ql, qr = inputs.euler_random_states(100000, seed=13)
    W, s, am, ap, st = orc.rp2(orc.EULER_ROE, P, 1, ql, qr)
    df = exact.euler_flux_x(qr, GAMMA) - exact.euler_flux_x(ql, GAMMA)
    sw = sum(s[p] * W[p] for p in range(4))
    scale = np.max(np.abs(df), axis=0) + np.max(np.abs(sw), axis=0)
    assert np.max(np.abs(sw - df) / scale) < 1e-12
    assert np.max(np.abs(am + ap - df) / scale) < 1e-12
    dq = qr - ql
    assert np.max(np.abs(sum(W) - dq) / np.max(np.abs(dq), axis=0)) < 1e-12


def test_euler_eigen_and_mirror(orc):
    P = orc.params(gamma=GAMMA)
    ql, qr = inputs.euler_random_states(20000, seed=14)
    W, s, am, ap, st = orc.rp2(orc.EULER_ROE, P, 1, ql, qr)
    roe = ~((s[1] == 0) & (s[2] == 0))  # HLLE fallback edges have zero middle speeds
    assert roe.mean() > 0.8
    # shear wave (0, 0, a, a v_hat); entropy wave ~ (1, u, v, (u^2+v^2)/2)
    assert np.all(W[2][0][roe] == 0) and np.all(W[2][1][roe] == 0)
    uh = s[1][roe]
    assert rel(W[1][1][roe], W[1][0][roe] * uh) < 1e-12
    # mirror symmetry
    M = np.array([1.0, -1.0, 1.0, 1.0])[:, None]
    _, _, am2, ap2, _ = orc.rp2(orc.EULER_ROE, P, 1, M * qr, M * ql)
    scale = np.max(np.abs(am) + np.abs(ap), axis=0)
    assert np.max(np.abs(am2 - M * ap) / scale) < 1e-12
    assert np.max(np.abs(ap2 - M * am) / scale) < 1e-12


def test_euler_hlle_fallback_on_strong_rarefaction(orc):
    """Two streams moving apart fast: the Roe intermediate state has negative
    pressure, so the HLLE fallback runs; it still satisfies the flux
    identity and its bounds contain the cell speeds."""
    P = orc.params(gamma=GAMMA)
    rho, p = 1.0, 0.4
    u = 3.0
    E = p / (GAMMA - 1) + 0.5 * rho * u * u
    ql = np.array([[rho], [-rho * u], [0.0], [E]])
    qr = np.array([[rho], [rho * u], [0.0], [E]])
    W, s, am, ap, st = orc.rp2(orc.EULER_ROE, P, 1, ql, qr)
    assert st & orc.ST_FALLBACK
    assert s[1][0] == 0 and s[2][0] == 0
    df = exact.euler_flux_x(qr, GAMMA) - exact.euler_flux_x(ql, GAMMA)
    assert rel(am + ap, df) < 1e-12
    c = np.sqrt(GAMMA * p / rho)
    assert s[0][0] <= -u - c + 1e-12 and s[3][0] >= u + c - 1e-12


def test_euler_y_is_permuted_x(orc):
    P = orc.params(gamma=GAMMA)
    ql, qr = inputs.euler_random_states(20000, seed=15)
    Wx, sx, amx, apx, _ = orc.rp2(orc.EULER_ROE, P, 1, ql, qr)
    Wy, sy, amy, apy, _ = orc.rp2(orc.EULER_ROE, P, 2, _perm_xy(ql), _perm_xy(qr))
    np.testing.assert_array_equal(sx, sy)
    for p in range(4):
        np.testing.assert_array_equal(_perm_xy(Wx[p]), Wy[p])
    np.testing.assert_array_equal(_perm_xy(amx), amy)


def test_nonphysical_flagged(orc):
    P = orc.params()
    ql = np.array([[1.0, -0.5], [0.0, 0.0], [0.0, 0.0]])
    qr = np.array([[1.0, 1.0], [0.0, 0.0], [0.0, 0.0]])
    _, _, am, ap, st = orc.rp2(orc.SW_ROE, P, 1, ql, qr)
    assert st & orc.ST_NONPHYS
    assert np.all(np.isfinite(am)) and np.all(am[:, 1] == 0)
