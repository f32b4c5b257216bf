"""Two-level refinement coupling of the split step (subcycled fine patches,
space-time ghost interpolation, conservative fix-up): CPU oracle.

TEST INFRASTRUCTURE ONLY: the test suite is the only user.  The product path
never imports this module, and this module never imports the product package.

The paper's kernel table (section 1.2, Table 1) places "dynamic time
stepping" between the Riemann/limiter kernels and grid management: it takes
the time step of the adjacent grid and produces updated values at grid
boundaries.  The text asks that each refined grid manage its own time step,
with an update procedure on refinement boundaries made of spatial and
temporal interpolation.  The paper gives no algorithm; this module writes out
the standard one for the method it builds on, for two levels and a fixed set
of refined patches (the grid-management kernel that would choose them is out
of scope): subcycling with interpolated ghost cells (Berger and Oliger, J.
Comput. Phys. 53, 1984) and the conservative fix-up at coarse-fine edges
("refluxing", Berger and Colella, J. Comput. Phys. 82, 1989).

Hierarchy.  A coarse grid nx x ny (cell sizes dx, dy) and refined patches,
each a rectangle of whole coarse cells (ci0, cj0, cw, ch), non-overlapping,
refined by r in both directions (fine cells dx/r, dy/r) and in time (r fine
steps of dt/r per coarse step).  A coarse cell is "covered" when a patch
contains it.  Every array here is [meqn][rows][columns].

One coarse step of size dt:
  1. the coarse grid gets its ghost cells from the boundary rule and takes
     one split step (covered cells included); at every coarse edge between
     an uncovered cell u and a covered cell the effective flux seen by u is
     kept: F = f(Q_u) + (A-dQ + Ftilde) if u is left of (below) the edge,
     F = f(Q_u) - (A+dQ - Ftilde) if right of (above) it, with Q_u the
     sweep's input at u (q^n for the x-sweep, the x-swept state for the
     y-sweep) and f the physical flux in the sweep's direction;
  2. for k = 0 .. r-1 every patch gets two ghost cells on each side (corners
     included) at time t + k dt / r: a ghost cell covered by a patch (after
     the fine boundary rule: periodic wrap or clamping at the domain edge)
     copies that patch's current value; any other takes the coarse cell
     under it, interpolated in space with minmod-limited slopes at t and at
     t + dt and linearly in time; then each patch takes one split step of
     dt / r on its padded array, the x-sweep running over the ghost rows too
     so that the y-sweep reads x-swept ghost values; at each patch boundary
     edge the effective flux seen by the inside cell, F = f(Q_in) - (A+dQ -
     Ftilde) on the left/bottom side and f(Q_in) + (A-dQ + Ftilde) on the
     right/top side, is summed over the r substeps;
  3. refluxing: an uncovered coarse cell next to a patch trades the coarse
     flux of step 1 for the average of the r x r fine fluxes through the
     same coarse edge (r fine edges times r substeps): Q_u += nu (F_c -
     Fbar) when u is left of (below) the edge, nu (Fbar - F_c) otherwise,
     nu = dt / dx (dt / dy);
  4. each covered coarse cell becomes the average of its r x r fine cells.
Order of floating-point sums (the device follows it): the fine flux sum
starts from the first substep's value; Fbar = (sum over the r fine edges in
increasing position) / r^2; a cell's corrections are applied in the order
left, right, bottom, top edge; averages sum row by row, column by column.

Refluxing needs the physical flux f, so the solvers covered are those whose
fluctuations sum to a flux difference, A-dQ + A+dQ = f(Q_r) - f(Q_l):
shallow water (Roe with the Harten-Hyman fix, HLLE), Euler (Roe with the
Harten-Hyman fix and the HLLE fallback), constant-coefficient acoustics
(f = A q, A the constant coefficient matrix) and advection (f = u q).
"""
import numpy as np

from . import (ACOUSTICS, ADVECTION, BC_PERIODIC, EULER_ROE, LIM_FIRST_ORDER, SW_HLLE, SW_ROE, params,
               rp2 as _rp2)
from .surrogate import phi


def sw_flux(q, g, ixy):
    """physical shallow-water flux in direction ixy of states q [3][...]"""
    h, hu, hv = q[0], q[1], q[2]
    if ixy == 1:
        u = hu / h
        return np.stack([hu, hu * u + 0.5 * g * (h * h), hv * u])
    v = hv / h
    return np.stack([hv, hu * v, hv * v + 0.5 * g * (h * h)])


def phys_flux(solver, P, q, ixy):
    """physical flux in direction ixy of states q [meqn][...] for the solvers
    the coupling covers (module docstring)"""
    if solver in (SW_ROE, SW_HLLE):
        return sw_flux(q, P.g, ixy)
    if solver == EULER_ROE:
        r, m1, m2, E = q[0], q[1], q[2], q[3]
        p = (P.gamma - 1.0) * (E - 0.5 * (m1 * m1 + m2 * m2) / r)
        w = (m1 if ixy == 1 else m2) / r
        out = np.stack([r * w, m1 * w, m2 * w, (E + p) * w])
        out[ixy] = out[ixy] + p
        return out
    if solver == ACOUSTICS:
        out = np.zeros_like(q)
        out[0] = P.K * q[ixy]
        out[ixy] = q[0] / P.rho
        return out
    if solver == ADVECTION:
        return (P.u if ixy == 1 else P.v) * q
    raise ValueError("refinement coupling: solver not covered")


def minmod(a, b):
    return np.where((a > 0.0) & (b > 0.0), np.minimum(a, b),
                    np.where((a < 0.0) & (b < 0.0), np.maximum(a, b), 0.0))


def ghost_index(n, bc):
    i = np.arange(-2, n + 2)
    return np.mod(i, n) if bc == BC_PERIODIC else np.clip(i, 0, n - 1)


def pad(q, bc):
    """grid [m][ny][nx] -> padded [m][ny+4][nx+4], ghosts by the boundary rule"""
    m, ny, nx = q.shape
    return q[:, ghost_index(ny, bc)][:, :, ghost_index(nx, bc)].copy()


class Hierarchy:
    def __init__(self, nx, ny, dx, dy, r, boxes, bc):
        self.nx, self.ny, self.dx, self.dy, self.r, self.bc = nx, ny, dx, dy, int(r), bc
        self.boxes = [tuple(int(v) for v in b) for b in boxes]
        own = -np.ones((ny, nx), dtype=np.int64)
        for p, (i0, j0, w, h) in enumerate(self.boxes):
            if w < 1 or h < 1 or i0 < 0 or j0 < 0 or i0 + w > nx or j0 + h > ny:
                raise ValueError(f"patch {p} outside the coarse grid")
            if (own[j0:j0 + h, i0:i0 + w] >= 0).any():
                raise ValueError(f"patch {p} overlaps another")
            own[j0:j0 + h, i0:i0 + w] = p
        self.owner = own

    def fine_shape(self, p):
        i0, j0, w, h = self.boxes[p]
        return h * self.r, w * self.r

    def neighbour(self, i, j, di, dj):
        """coarse neighbour (i + di, j + dj) under the boundary rule, or None
        outside the domain when the rule is extrapolation"""
        a, b = i + di, j + dj
        if self.bc == BC_PERIODIC:
            return a % self.nx, b % self.ny
        if 0 <= a < self.nx and 0 <= b < self.ny:
            return a, b
        return None

    def interfaces(self):
        """per uncovered coarse cell next to a patch: (i, j, [4 entries]) for
        its left, right, bottom and top edges, each None or (patch, side,
        position of the coarse edge along that patch side); side names the
        patch side the edge lies on: 'R' (patch left of u), 'L' (patch
        right of u), 'T' (patch below u), 'B' (patch above u)"""
        out = []
        for j in range(self.ny):
            for i in range(self.nx):
                if self.owner[j, i] >= 0:
                    continue
                ent = []
                any_ = False
                for di, dj, side in ((-1, 0, "R"), (1, 0, "L"), (0, -1, "T"), (0, 1, "B")):
                    nb = self.neighbour(i, j, di, dj)
                    e = None
                    if nb is not None and self.owner[nb[1], nb[0]] >= 0:
                        p = int(self.owner[nb[1], nb[0]])
                        i0, j0, _, _ = self.boxes[p]
                        pos = nb[1] - j0 if side in ("R", "L") else nb[0] - i0
                        e = (p, side, pos)
                        any_ = True
                    ent.append(e)
                if any_:
                    out.append((i, j, ent))
        return out


def plain_rp(solver=SW_ROE, g=9.81, P=None):
    P = params(g=g) if P is None else P

    def rp(ixy, ql, qr):
        w, s, am, ap, _ = _rp2(solver, P, ixy, ql, qr)
        return w, s, am, ap
    return rp


def line_sweep(rp, ixy, G, nu, limiter):
    """Sweep of lines with two ghost cells at each end.  G: [m][L][n+4].
    Returns the n updated interior cells of every line [m][L][n], and at
    the n+1 edges bounding them (edge k left of interior cell k) the terms
    lf = A-dQ + Ftilde and rg = A+dQ - Ftilde [m][L][n+1] and the speeds
    [mw][L][n+1].  Same arithmetic as the whole-grid sweep of the surrogate
    oracle (A6 limiter reading: upwind neighbour's wave, theta = W_up.W /
    W.W, no correction when W.W = 0)."""
    m, L, N = G.shape
    n = N - 4
    ql = G[:, :, :-1].reshape(m, -1)
    qr = G[:, :, 1:].reshape(m, -1)
    waves, s, amdq, apdq = rp(ixy, ql, qr)
    mw = waves.shape[0]
    ne = N - 1
    waves = waves.reshape(mw, m, L, ne)
    s = s.reshape(mw, L, ne)
    amdq, apdq = amdq.reshape(m, L, ne), apdq.reshape(m, L, ne)
    k = np.arange(1, n + 2)
    ftil = np.zeros((m, L, ne))
    if limiter != LIM_FIRST_ORDER:
        for p in range(mw):
            sp = s[p][:, k]
            up = np.where(sp > 0.0, k - 1, k + 1)
            wk = waves[p][:, :, k]
            wu = np.take_along_axis(waves[p], np.broadcast_to(up, wk.shape), axis=2)
            wn = wk[0] * wk[0]
            wd = wu[0] * wk[0]
            for c in range(1, m):
                wn = wn + wk[c] * wk[c]
                wd = wd + wu[c] * wk[c]
            ph = np.where(wn == 0.0, 0.0, phi(limiter, wd / np.where(wn == 0.0, 1.0, wn)))
            cc = 0.5 * np.abs(sp) * (1.0 - nu * np.abs(sp))
            ftil[:, :, k] += cc * (ph * wk)
    i = np.arange(n)
    kl, kr = i + 1, i + 2
    inner = G[:, :, 2:-2]
    out = inner - nu * (apdq[:, :, kl] + amdq[:, :, kr]) - nu * (ftil[:, :, kr] - ftil[:, :, kl])
    lf = amdq[:, :, k] + ftil[:, :, k]
    rg = apdq[:, :, k] - ftil[:, :, k]
    return out, lf, rg, s[:, :, k]


def padded_step(rp, G, nux, nuy, limiter):
    """Split step of one ghost-padded grid G [m][ny+4][nx+4]: the x-sweep of
    every row (ghost rows included), then the y-sweep of the interior
    columns of the x-swept array.  Returns (q_new [m][ny][nx], x-record,
    y-record, max |s| over the counted x-edges, over the counted y-edges)
    with x-record = (G, lf, rg) and lf, rg [m][ny+4][nx+1] (edge i left of
    cell i), y-record = (Qs, lf, rg) with Qs the padded x-swept state and
    lf, rg [m][nx][ny+1] (edge j below cell j, per column)."""
    m, Ly, Lx = G.shape
    ny, nx = Ly - 4, Lx - 4
    xo, xlf, xrg, xs = line_sweep(rp, 1, G, nux, limiter)
    Qs = G.copy()
    Qs[:, :, 2:-2] = xo
    cols = np.ascontiguousarray(Qs[:, :, 2:-2].transpose(0, 2, 1))     # [m][nx][ny+4]
    yo, ylf, yrg, ys = line_sweep(rp, 2, cols, nuy, limiter)
    qn = np.ascontiguousarray(yo.transpose(0, 2, 1))
    smx = float(np.abs(xs[:, 2:-2, :]).max()) if nx and ny else 0.0
    smy = float(np.abs(ys).max()) if nx and ny else 0.0
    return qn, (G, xlf, xrg), (Qs, ylf, yrg), smx, smy


def _interp(H, Gp, I, J):
    """coarse solution (padded Gp) at fine global cells (I, J), limited
    linear in space"""
    r = H.r
    Ic, Jc = I // r, J // r
    xi = ((I % r) + 0.5) / r - 0.5
    eta = ((J % r) + 0.5) / r - 0.5
    Q = Gp[:, Jc + 2, Ic + 2]
    sx = minmod(Gp[:, Jc + 2, Ic + 3] - Q, Q - Gp[:, Jc + 2, Ic + 1])
    sy = minmod(Gp[:, Jc + 3, Ic + 2] - Q, Q - Gp[:, Jc + 1, Ic + 2])
    return (Q + xi * sx) + eta * sy


def fill_fine(H, p, fine, Gn, Gn1, alpha):
    """padded array of patch p at time fraction alpha of the coarse step:
    interior from fine[p], ghost cells from the covering patch (current
    values) or interpolated from the padded coarse states Gn (t) and Gn1
    (t + dt)"""
    r = H.r
    i0, j0, w, h = H.boxes[p]
    ny, nx = h * r, w * r
    m = fine[p].shape[0]
    G = np.zeros((m, ny + 4, nx + 4))
    G[:, 2:-2, 2:-2] = fine[p]
    jj, ii = np.meshgrid(np.arange(-2, ny + 2), np.arange(-2, nx + 2), indexing="ij")
    ghost = (ii < 0) | (ii >= nx) | (jj < 0) | (jj >= ny)
    gi, gj = ii[ghost], jj[ghost]
    I, J = i0 * r + gi, j0 * r + gj
    NX, NY = H.nx * r, H.ny * r
    if H.bc == BC_PERIODIC:
        I, J = np.mod(I, NX), np.mod(J, NY)
    else:
        I, J = np.clip(I, 0, NX - 1), np.clip(J, 0, NY - 1)
    own = H.owner[J // r, I // r]
    vals = np.zeros((m, gi.size))
    cov = own >= 0
    for o in np.unique(own[cov]):
        sel = own == o
        oi0, oj0, _, _ = H.boxes[o]
        vals[:, sel] = fine[o][:, J[sel] - oj0 * r, I[sel] - oi0 * r]
    unc = ~cov
    if unc.any():
        a = _interp(H, Gn, I[unc], J[unc])
        b = _interp(H, Gn1, I[unc], J[unc])
        vals[:, unc] = (1.0 - alpha) * a + alpha * b
    G[:, gj + 2, gi + 2] = vals
    return G


def _side_fluxes(xrec, yrec, flux):
    """effective fluxes seen by the inside cells at the four sides of a
    padded grid: L, R [m][ny], B, T [m][nx]; flux(q, ixy) the physical flux"""
    G, xlf, xrg = xrec
    Qs, ylf, yrg = yrec
    m, Ly, Lx = G.shape
    ny, nx = Ly - 4, Lx - 4
    rows = np.arange(2, ny + 2)
    L = flux(G[:, rows, 2], 1) - xrg[:, rows, 0]
    R = flux(G[:, rows, nx + 1], 1) + xlf[:, rows, nx]
    B = flux(Qs[:, 2, 2:-2], 2) - yrg[:, :, 0]
    T = flux(Qs[:, ny + 1, 2:-2], 2) + ylf[:, :, ny]
    return {"L": L, "R": R, "B": B, "T": T}


def step(H, qc, fine, dt, limiter, solver=SW_ROE, g=9.81, reflux=True, P=None):
    """One coarse step of the two-level hierarchy (module docstring, steps
    1-4).  qc: coarse [meqn][ny][nx]; fine: list of [meqn][h r][w r]; P the
    solver's constants (default: shallow water with gravity g).  Returns
    (qc_new, fine_new, smax_coarse, smax_fine) with smax = max |s| / d over
    the counted edges of the level (all substeps for the fine level)."""
    r = H.r
    P = params(g=g) if P is None else P
    rp = plain_rp(solver, P=P)
    flux = lambda q, ixy: phys_flux(solver, P, q, ixy)
    qc = np.asarray(qc, dtype=np.float64)
    fine = [np.asarray(f, dtype=np.float64) for f in fine]
    # 1. coarse step and the coarse fluxes at coarse-fine edges
    Gn = pad(qc, H.bc)
    qc1, (Gx, xlf, xrg), (Qs, ylf, yrg), smx, smy = padded_step(rp, Gn, dt / H.dx, dt / H.dy, limiter)
    smax_c = max(smx / H.dx, smy / H.dy)
    # 2. subcycled fine steps
    Gn1 = pad(qc1, H.bc)
    dtf, dxf, dyf = dt / r, H.dx / r, H.dy / r
    acc = [None] * len(fine)
    smax_f = 0.0
    for k in range(r):
        alpha = k / r
        padded = [fill_fine(H, p, fine, Gn, Gn1, alpha) for p in range(len(fine))]
        new = []
        for p, G in enumerate(padded):
            qn, xrec, yrec, sx, sy = padded_step(rp, G, dtf / dxf, dtf / dyf, limiter)
            smax_f = max(smax_f, sx / dxf, sy / dyf)
            F = _side_fluxes(xrec, yrec, flux)
            acc[p] = F if acc[p] is None else {s: acc[p][s] + F[s] for s in F}
            new.append(qn)
        fine = new
    # 3. refluxing
    if reflux:
        nux, nuy = dt / H.dx, dt / H.dy
        for (i, j, ent) in H.interfaces():
            q = qc1[:, j, i].copy()
            for d, e in enumerate(ent):
                if e is None:
                    continue
                p, side, pos = e
                reg = acc[p][side][:, pos * r:(pos + 1) * r]
                s = reg[:, 0]
                for l in range(1, r):
                    s = s + reg[:, l]
                Fbar = s / (r * r)
                if d == 0:      # left edge of u: u on its right, patch on its left
                    Fc = flux(Gx[:, j + 2, i + 2], 1) - xrg[:, j + 2, i]
                    q = q + nux * (Fbar - Fc)
                elif d == 1:    # right edge: u on its left
                    Fc = flux(Gx[:, j + 2, i + 2], 1) + xlf[:, j + 2, i + 1]
                    q = q + nux * (Fc - Fbar)
                elif d == 2:    # bottom edge: u above it
                    Fc = flux(Qs[:, j + 2, i + 2], 2) - yrg[:, i, j]
                    q = q + nuy * (Fbar - Fc)
                else:           # top edge: u below it
                    Fc = flux(Qs[:, j + 2, i + 2], 2) + ylf[:, i, j + 1]
                    q = q + nuy * (Fc - Fbar)
            qc1[:, j, i] = q
    # 4. averaging down
    for p, (i0, j0, w, h) in enumerate(H.boxes):
        f = fine[p]
        s = np.zeros((f.shape[0], h, w))
        for a in range(r):
            for b in range(r):
                s = s + f[:, a::r, b::r]
        qc1[:, j0:j0 + h, i0:i0 + w] = s / (r * r)
    return qc1, fine, smax_c, smax_f


def total(H, qc):
    """sum of the coarse cells times the coarse cell area (after averaging
    down, covered cells carry their patch's content)"""
    return qc.reshape(qc.shape[0], -1).sum(axis=1) * (H.dx * H.dy)


def restrict(H, fine_full):
    """fine-level samples [m][ny r][nx r] -> per-patch fine arrays"""
    r = H.r
    return [fine_full[:, j0 * r:(j0 + h) * r, i0 * r:(i0 + w) * r].copy() for (i0, j0, w, h) in H.boxes]
