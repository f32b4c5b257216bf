"""Unsplit 2D step with transverse Riemann solves: CPU oracle.

TEST INFRASTRUCTURE ONLY: the test suite is the only user.  The product path
never imports this module, and this module never imports the product package.

The paper reports that computing the Riemann problems of both directions in
one pass over the data was its simplest and fastest threading (section 2);
the unsplit form of the wave-propagation method is the variant that reads
one state for both directions.  It is the corner-transport form of LeVeque
2002, chapters 20 and 21, with first-order transverse propagation and
limited second-order corrections in the normal directions.  With
nux = dt/dx, nuy = dt/dy:

  Q_ij^{n+1} = Q_ij - nux (A+dQ_{i-1/2,j} + A-dQ_{i+1/2,j})
                    - nuy (B+dQ_{i,j-1/2} + B-dQ_{i,j+1/2})
                    - nux (F_{i+1/2,j} - F_{i-1/2,j})
                    - nuy (G_{i,j+1/2} - G_{i,j-1/2})

where every edge's normal solve (waves, speeds, fluctuations) is that of the
plain method on q^n, F and G start as the limited corrections of the plain
method, and the fluctuations that enter a cell are split by a transverse
solve into the parts moving up and down (for x-edges) or right and left (for
y-edges), which correct the fluxes of the other direction:

  an x-edge's A+dQ enters its right cell (i, j): G_{i,j+1/2} -= nux/2 B+A+dQ,
      G_{i,j-1/2} -= nux/2 B-A+dQ; its A-dQ enters the left cell (i-1, j):
      G_{i-1,j+1/2} -= nux/2 B+A-dQ, G_{i-1,j-1/2} -= nux/2 B-A-dQ;
  a y-edge's B+dQ enters the cell above (i, j): F_{i+1/2,j} -= nuy/2 A+B+dQ,
      F_{i-1/2,j} -= nuy/2 A-B+dQ; its B-dQ enters the cell below (i, j-1):
      F_{i+1/2,j-1} -= nuy/2 A+B-dQ, F_{i-1/2,j-1} -= nuy/2 A-B-dQ.

The transverse split of a vector d at an edge, in the direction across the
edge's normal (the eigenvectors of that direction's flux Jacobian, at the
edge's Roe average where the system is nonlinear):
  advection    B-d = min(w, 0) d, B+d = max(w, 0) d, w the velocity along
               the transverse direction;
  acoustics    (p, u, v), Z = sqrt(K rho), c = sqrt(K / rho); with d_t the
               velocity component along the transverse direction:
               b1 = (-d_p + Z d_t) / (2 Z) on r1 = (-Z, e_t) at speed -c,
               b3 = (d_p + Z d_t) / (2 Z) on r3 = (Z, e_t) at speed +c;
  shallow water, Roe  with u_n, u_t the Roe-averaged velocities along the
               edge normal and the transverse direction and c = sqrt(g hbar):
               b1 = ((u_t + c) d_h - d_t) / (2c) on r1 = (1, u_n e_n + (u_t - c) e_t),
               b2 = d_n - u_n d_h on e_n (speed u_t),
               b3 = (d_t - (u_t - c) d_h) / (2c) on r3 = (1, u_n e_n + (u_t + c) e_t),
               speeds u_t - c, u_t, u_t + c; the same split serves the
               HLLE normal solver (the Roe averages of the edge's two
               cells); an edge with a dry side (h <= 0, where the normal
               solve has no waves and no fluctuations) has no transverse
               part -- the split is linear in d and the average undefined;
  Euler, Roe   (rho, rho u, rho v, E) with the Roe averages u_n, u_t, H and
               c^2 = (gamma - 1)(H - |u|^2 / 2):
               b2 = (gamma - 1) / c^2 ((H - |u|^2) d_rho + u_n d_n + u_t d_t - d_E),
               b3 = d_n - u_n d_rho (the shear wave along the transverse
               direction), b1 = ((u_t + c) d_rho - d_t - c b2) / (2c),
               b4 = d_rho - b1 - b2, on r1 = (1, u_n e_n + (u_t - c) e_t,
               H - u_t c), r2 = (1, u_n e_n + u_t e_t, |u|^2 / 2),
               r3 = (0, e_n, u_n), r4 = (1, u_n e_n + (u_t + c) e_t, H + u_t c)
               at speeds u_t - c, u_t, u_t, u_t + c; where c^2 <= 0 (the edges
               where the plain solver falls back to HLLE) there is no
               transverse part;
  in each case B-d sums min(speed, 0) b r and B+d sums max(speed, 0) b r;
  variable-coefficient acoustics (aux = (rho, c) per cell, Z = rho c): the
               split of d entering cell m uses the impedances and speeds of m
               and of its neighbours across the transverse direction, b (below
               or left) and a (above or right):
               B-d = -c_b g1 (-Z_b, e_t), g1 = (-d_p + Z_m d_t) / (Z_b + Z_m),
               B+d =  c_a g2 ( Z_a, e_t), g2 = ( d_p + Z_m d_t) / (Z_m + Z_a)
               (the down/up-going waves of the transverse problems between b
               and m and between m and a; a uniform medium gives the
               constant-coefficient split).
"""
import numpy as np

from . import ACOUSTICS, ACOUSTICS_VC, ADVECTION, BC_PERIODIC, DIMS, EULER_ROE, LIM_FIRST_ORDER, SW_HLLE, SW_ROE, rp2
from .surrogate import phi

SUPPORTED = (ADVECTION, ACOUSTICS, ACOUSTICS_VC, SW_ROE, SW_HLLE, EULER_ROE)


def pad(q, bc):
    m, ny, nx = q.shape
    def gi(n):
        i = np.arange(-2, n + 2)
        return np.mod(i, n) if bc == BC_PERIODIC else np.clip(i, 0, n - 1)
    return q[:, gi(ny)][:, :, gi(nx)]


def tsplit(solver, P, ixy, ql, qr, d):
    """transverse split of d [m][n] at edges of normal direction ixy between
    states ql, qr: returns (down/left-going, up/right-going) parts"""
    if solver == ADVECTION:
        w = P.v if ixy == 1 else P.u
        return np.minimum(w, 0.0) * d, np.maximum(w, 0.0) * d
    t = 2 if ixy == 1 else 1            # component along the transverse direction
    if solver == ACOUSTICS:
        Z = np.sqrt(P.K * P.rho)
        c = np.sqrt(P.K / P.rho)
        b1 = (-d[0] + Z * d[t]) / (2.0 * Z)
        b3 = (d[0] + Z * d[t]) / (2.0 * Z)
        r1 = np.zeros((3,) + b1.shape)
        r3 = np.zeros((3,) + b1.shape)
        r1[0], r1[t] = -Z, 1.0
        r3[0], r3[t] = Z, 1.0
        return -c * b1 * r1, c * b3 * r3
    n = ixy
    if solver == EULER_ROE:
        gm = P.gamma
        rl, rr = ql[0], qr[0]
        sl, sr = np.sqrt(rl), np.sqrt(rr)
        def prim(q):
            u1, u2 = q[1] / q[0], q[2] / q[0]
            p = (gm - 1.0) * (q[3] - 0.5 * q[0] * (u1 * u1 + u2 * u2))
            return u1, u2, (q[3] + p) / q[0]
        ul1, ul2, Hl = prim(ql)
        ur1, ur2, Hr = prim(qr)
        w = sl + sr
        uh = [None, (sl * ul1 + sr * ur1) / w, (sl * ul2 + sr * ur2) / w]
        Hh = (sl * Hl + sr * Hr) / w
        un, ut = uh[n], uh[t]
        q2 = un * un + ut * ut
        c2 = (gm - 1.0) * (Hh - 0.5 * q2)
        ok = c2 > 0.0
        c = np.sqrt(np.where(ok, c2, 1.0))
        c2s = np.where(ok, c2, 1.0)
        b2 = (gm - 1.0) / c2s * ((Hh - q2) * d[0] + un * d[n] + ut * d[t] - d[3])
        b3 = d[n] - un * d[0]
        b1 = ((ut + c) * d[0] - d[t] - c * b2) / (2.0 * c)
        b4 = d[0] - b1 - b2
        lam = (ut - c, ut, ut, ut + c)
        r = [np.zeros((4,) + b1.shape) for _ in range(4)]
        r[0][0], r[0][n], r[0][t], r[0][3] = 1.0, un, ut - c, Hh - ut * c
        r[1][0], r[1][n], r[1][t], r[1][3] = 1.0, un, ut, 0.5 * q2
        r[2][n], r[2][3] = 1.0, un
        r[3][0], r[3][n], r[3][t], r[3][3] = 1.0, un, ut + c, Hh + ut * c
        bs = (b1, b2, b3, b4)
        bm = sum(np.minimum(l, 0.0) * b * rr_ for l, b, rr_ in zip(lam, bs, r))
        bp = sum(np.maximum(l, 0.0) * b * rr_ for l, b, rr_ in zip(lam, bs, r))
        return np.where(ok, bm, 0.0), np.where(ok, bp, 0.0)
    # shallow water (Roe or HLLE), Roe averages of the edge; none on a dry edge
    g = P.g
    wet = (ql[0] > 0.0) & (qr[0] > 0.0)
    hl, hr = np.where(wet, ql[0], 1.0), np.where(wet, qr[0], 1.0)
    sl, sr = np.sqrt(hl), np.sqrt(hr)
    un = (sl * (ql[n] / hl) + sr * (qr[n] / hr)) / (sl + sr)
    ut = (sl * (ql[t] / hl) + sr * (qr[t] / hr)) / (sl + sr)
    c = np.sqrt(g * 0.5 * (hl + hr))
    b1 = ((ut + c) * d[0] - d[t]) / (2.0 * c)
    b2 = d[n] - un * d[0]
    b3 = (d[t] - (ut - c) * d[0]) / (2.0 * c)
    lam = (ut - c, ut, ut + c)
    r = [np.zeros((3,) + b1.shape) for _ in range(3)]
    r[0][0], r[0][n], r[0][t] = 1.0, un, ut - c
    r[1][n] = 1.0
    r[2][0], r[2][n], r[2][t] = 1.0, un, ut + c
    bm = sum(np.minimum(l, 0.0) * b * rr for l, b, rr in zip(lam, (b1, b2, b3), r))
    bp = sum(np.maximum(l, 0.0) * b * rr for l, b, rr in zip(lam, (b1, b2, b3), r))
    return np.where(wet, bm, 0.0), np.where(wet, bp, 0.0)


def tsplit_vc(ixy, d, Zb, cb, Zm, Za, ca):
    """variable-coefficient transverse split of d entering cell m (module
    docstring); returns (towards b, towards a)"""
    t = 2 if ixy == 1 else 1
    o = 3 - t
    g1 = (-d[0] + Zm * d[t]) / (Zb + Zm)
    g2 = (d[0] + Zm * d[t]) / (Zm + Za)
    bm = np.zeros_like(d)
    bp = np.zeros_like(d)
    bm[0] = (cb * g1) * Zb
    bm[t] = -(cb * g1)
    bp[0] = (ca * g2) * Za
    bp[t] = ca * g2
    bm[o] = 0.0
    bp[o] = 0.0
    return bm, bp


def edges(solver, P, G, ixy, nu, limiter, Ga=None):
    """normal solves of every edge along the last axis of the padded lines G
    [m][L][N] (edge k between cells k and k+1); returns amdq, apdq, the
    limited correction Ftilde (zero at the two outermost edges), the
    transverse parts of both fluctuations, and the speeds"""
    m, L, N = G.shape
    ql = G[:, :, :-1].reshape(m, -1)
    qr = G[:, :, 1:].reshape(m, -1)
    ea = None
    if Ga is not None:
        ea = np.stack([Ga[:, :, :-1].reshape(2, -1), Ga[:, :, 1:].reshape(2, -1)])
    waves, s, am, ap, _ = rp2(solver, P, ixy, ql, qr, ea)
    mw = waves.shape[0]
    ne = N - 1
    amm, apm = am.reshape(m, L, ne), ap.reshape(m, L, ne)
    shp = (m, L, ne)
    if solver == ACOUSTICS_VC:
        # materials of the receiving cells and of their neighbours in the
        # adjacent lines (the outermost lines take their own, unused)
        Z = Ga[0] * Ga[1]
        c = Ga[1]
        lo = np.concatenate([[0], np.arange(L - 1)])
        hi = np.concatenate([np.arange(1, L), [L - 1]])
        def split(d, col):
            Zm = Z[:, col]
            return tsplit_vc(ixy, d.reshape(shp), Z[lo][:, col], c[lo][:, col], Zm,
                             Z[hi][:, col], c[hi][:, col])
        bmAm, bpAm = split(am, slice(0, N - 1))      # A-dQ enters the left cell of the edge
        bmAp, bpAp = split(ap, slice(1, N))          # A+dQ enters the right cell
        bmAm, bpAm, bmAp, bpAp = (x.reshape(m, -1) for x in (bmAm, bpAm, bmAp, bpAp))
    else:
        bmAm, bpAm = tsplit(solver, P, ixy, ql, qr, am)
        bmAp, bpAp = tsplit(solver, P, ixy, ql, qr, ap)
    waves = waves.reshape(mw, m, L, ne)
    s = s.reshape(mw, L, ne)
    ftil = np.zeros(shp)
    if limiter != LIM_FIRST_ORDER:
        k = np.arange(1, ne - 1)
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
    return (amm, apm, ftil, bmAm.reshape(shp), bpAm.reshape(shp), bmAp.reshape(shp), bpAp.reshape(shp), s)


def unsplit_step(solver, P, q, dx, dy, dt, limiter, bc, aux=None):
    """One unsplit step (module docstring).  q: [meqn][ny][nx].  Returns
    (q_new, smax) with smax = max(max |s_x| / dx, max |s_y| / dy) over the
    counted edges (x-edges 0..nx of every row, y-edges 0..ny of every
    column)."""
    if solver not in SUPPORTED:
        raise ValueError("unsplit step: solver not covered")
    q = np.asarray(q, dtype=np.float64)
    m, ny, nx = q.shape
    nux, nuy = dt / dx, dt / dy
    Gp = pad(q, bc)                                    # [m][ny+4][nx+4], cell (j, i) at (j+2, i+2)
    Ap = pad(np.asarray(aux, dtype=np.float64), bc) if aux is not None else None
    if solver == ACOUSTICS_VC and Ap is None:
        raise ValueError("variable-coefficient acoustics needs aux")
    # x-edges of every padded row: edge k between padded columns k and k+1
    xa, xp, xf, xbmAm, xbpAm, xbmAp, xbpAp, xs = edges(solver, P, Gp, 1, nux, limiter, Ap)
    # y-edges of every padded column: edge k between padded rows k and k+1
    Gt = np.ascontiguousarray(Gp.transpose(0, 2, 1))   # [m][nx+4][ny+4]
    At = np.ascontiguousarray(Ap.transpose(0, 2, 1)) if Ap is not None else None
    ya, yp, yf, ybmAm, ybpAm, ybmAp, ybpAp, ys = edges(solver, P, Gt, 2, nuy, limiter, At)
    # to [m][row][col] edge layouts: X[., J, k] edge left of padded column k+1;
    # Y[., k, I] edge below padded row k+1
    Yt = lambda a: np.ascontiguousarray(a.transpose(0, 2, 1))
    ya, yp, yf, ybmAm, ybpAm, ybmAp, ybpAp = map(Yt, (ya, yp, yf, ybmAm, ybpAm, ybmAp, ybpAp))
    Lyp, Lxp = ny + 4, nx + 4
    F = xf.copy()        # [m][Ly][Lx-1]
    Gf = yf.copy()       # [m][Ly-1][Lx]
    # transverse corrections from the x-edges to G.  x-edge (J, k) joins
    # padded columns k and k+1 of row J: its A+ enters cell (J, k+1), its A-
    # enters (J, k); an up-going part corrects the y-edge above the cell it
    # enters (G index J), a down-going part the y-edge below it (index J-1)
    half = 0.5 * nux
    Gf[:, :, 1:] -= half * xbpAp[:, :-1, :]
    Gf[:, :, 1:] -= half * xbmAp[:, 1:, :]
    Gf[:, :, :-1] -= half * xbpAm[:, :-1, :]
    Gf[:, :, :-1] -= half * xbmAm[:, 1:, :]
    # transverse corrections from the y-edges to F.  y-edge (k, I) joins
    # padded rows k and k+1 of column I: its B+ enters cell (k+1, I), its B-
    # enters (k, I); a right-going part corrects the x-edge right of the cell
    # it enters (F index I), a left-going part the x-edge left of it (I-1)
    halfy = 0.5 * nuy
    F[:, 1:, :] -= halfy * ybpAp[:, :, :-1]
    F[:, 1:, :] -= halfy * ybmAp[:, :, 1:]
    F[:, :-1, :] -= halfy * ybpAm[:, :, :-1]
    F[:, :-1, :] -= halfy * ybmAm[:, :, 1:]
    # update of the interior cells (J, I) = (j+2, i+2)
    J = slice(2, ny + 2)
    I = slice(2, nx + 2)
    Il, Ir = slice(1, nx + 1), slice(2, nx + 2)        # x-edges left / right of column I
    Jb, Jt = slice(1, ny + 1), slice(2, ny + 2)        # y-edges below / above row J
    out = (Gp[:, J, I]
           - nux * (xp[:, J, Il] + xa[:, J, Ir])
           - nuy * (yp[:, Jb, I] + ya[:, Jt, I])
           - nux * (F[:, J, Ir] - F[:, J, Il])
           - nuy * (Gf[:, Jt, I] - Gf[:, Jb, I]))
    smx = float(np.abs(xs[:, 2:ny + 2, 1:nx + 2]).max())
    smy = float(np.abs(ys[:, 2:nx + 2, 1:ny + 2]).max())
    return np.ascontiguousarray(out), max(smx / dx, smy / dy)
