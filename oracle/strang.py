"""Strang splitting of the 2D step: CPU oracle.

TEST INFRASTRUCTURE ONLY: the test suite is the only user.  The product path
never imports this module, and this module never imports the product package.

The paper's method advances the 2D equations by one-dimensional sweeps
(section 2 solves the normal Riemann problem of one direction at a time).
The plain step is Godunov splitting, an x-sweep then a y-sweep of its result,
each with the full dt: first order in time wherever the two directions do
not commute.  Strang splitting (Strang, SIAM J. Numer. Anal. 5, 1968;
LeVeque 2002, section 19.5) takes an x-sweep of dt/2, a y-sweep of dt and an
x-sweep of dt/2: second order in time for smooth solutions.

Each sweep is the whole-grid sweep of the plain method: ghost cells by the
boundary rule, the edge solve of every line (the C oracle's `mco_rp2`, aux
values of the two cells where the solver has them), limited correction
fluxes (upwind neighbour's wave, theta = W_up . W / W . W) and the
conservative update.
"""
import numpy as np

from . import BC_PERIODIC, DIMS, LIM_FIRST_ORDER, rp2
from .surrogate import phi


def _ghost(n, bc):
    i = np.arange(-2, n + 2)
    return np.mod(i, n) if bc == BC_PERIODIC else np.clip(i, 0, n - 1)


def sweep(solver, P, q, aux, ixy, nu, limiter, bc):
    """One sweep of the whole grid in direction ixy with Courant factor
    nu = dt / d.  q: [meqn][ny][nx]; aux: [maux][ny][nx] or None.  Returns
    (q_new, max |s| over the counted edges)."""
    meqn, mw, maux = DIMS[solver]
    lines = q if ixy == 1 else q.transpose(0, 2, 1)
    _, L, n = lines.shape
    gi = _ghost(n, bc)
    G = lines[:, :, gi]
    ne = n + 3
    ql = G[:, :, :-1].reshape(meqn, -1)
    qr = G[:, :, 1:].reshape(meqn, -1)
    ea = None
    if maux:
        al = aux if ixy == 1 else aux.transpose(0, 2, 1)
        Ga = al[:, :, gi]
        ea = np.stack([Ga[:, :, :-1].reshape(maux, -1), Ga[:, :, 1:].reshape(maux, -1)])
    waves, s, amdq, apdq, _ = rp2(solver, P, ixy, ql, qr, ea)
    waves = waves.reshape(mw, meqn, L, ne)
    s = s.reshape(mw, L, ne)
    amdq, apdq = amdq.reshape(meqn, L, ne), apdq.reshape(meqn, L, ne)
    k = np.arange(1, n + 2)
    smax = float(np.abs(s[:, :, k]).max())
    ftil = np.zeros((meqn, L, ne))
    if limiter != LIM_FIRST_ORDER:
        for p in range(mw):
            sp = s[p][:, k]
            up = np.where(sp > 0.0, k - 1, k + 1)
            wk = waves[p][:, :, k]
            wu = np.take_along_axis(waves[p], np.broadcast_to(up, wk.shape), axis=2)
            wn = wk[0] * wk[0]
            wd = wu[0] * wk[0]
            for m in range(1, meqn):
                wn = wn + wk[m] * wk[m]
                wd = wd + wu[m] * wk[m]
            ph = np.where(wn == 0.0, 0.0, phi(limiter, wd / np.where(wn == 0.0, 1.0, wn)))
            c = 0.5 * np.abs(sp) * (1.0 - nu * np.abs(sp))
            ftil[:, :, k] += c * (ph * wk)
    i = np.arange(n)
    kl, kr = i + 1, i + 2
    out = lines - nu * (apdq[:, :, kl] + amdq[:, :, kr]) - nu * (ftil[:, :, kr] - ftil[:, :, kl])
    out = out if ixy == 1 else out.transpose(0, 2, 1)
    return np.ascontiguousarray(out), smax


def strang_step(solver, P, q, dx, dy, dt, limiter, bc, aux=None):
    """x-sweep (dt/2), y-sweep (dt), x-sweep (dt/2).  Returns (q_new, smax)
    with smax = the largest Courant number of the three sweeps divided by
    dt (max(sx / (2 dx), sy / dy))."""
    q = np.asarray(q, dtype=np.float64)
    q1, s1 = sweep(solver, P, q, aux, 1, 0.5 * dt / dx, limiter, bc)
    q2, s2 = sweep(solver, P, q1, aux, 2, dt / dy, limiter, bc)
    q3, s3 = sweep(solver, P, q2, aux, 1, 0.5 * dt / dx, limiter, bc)
    return q3, max(0.5 * s1 / dx, s2 / dy, 0.5 * s3 / dx)


def godunov_step(solver, P, q, dx, dy, dt, limiter, bc, aux=None):
    """x-sweep (dt), then y-sweep (dt) of its result: the plain step"""
    q1, s1 = sweep(solver, P, np.asarray(q, dtype=np.float64), aux, 1, dt / dx, limiter, bc)
    q2, s2 = sweep(solver, P, q1, aux, 2, dt / dy, limiter, bc)
    return q2, max(s1 / dx, s2 / dy)
