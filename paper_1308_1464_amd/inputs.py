"""Seeded synthetic inputs shared by the device path and the CPU oracle.

This module holds no arithmetic of the method: only random draws and the
initial-condition recipes (cell-centre sampling on the unit square).  Random
numbers come from NumPy's counter-based Philox generator, seeded per case.

Recipes (cell centres ((i+1/2)dx, (j+1/2)dy) on [0,1]^2, dx = 1/nx, dy = 1/ny):
  acoustics_pulse   p = exp(-200 r^2) about (0.5, 0.5), u = v = 0
  layered_medium    rho = 1 | 2.5 split at x = 0.5, c = 1 | 0.6 split at y = 0.5
  sw_dam_break      h = 2 inside r < 0.3, 1 outside, plus i.i.d. 1e-3*U(-1,1)
                    per cell; hu = hv = 0
  euler_quadrants   split at (0.5, 0.5); quadrants NE, NW, SW, SE each draw
                    rho, u, v, p in that order, rho, p ~ U[0.1, 2],
                    u, v ~ U[-1, 1]; E = p/(gamma-1) + rho (u^2 + v^2)/2
  patch_set         n patches, sides round(exp(U(ln 16, ln 256))) drawn
                    independently for nx and ny; each a radial dam break of
                    radius 0.3 with h_out = 1 and h_in ~ U(1.5, 10), no noise
  sw_noise_device   grids too large to stage from the host, drawn on the
                    device by torch's seeded generator: h ~ U(0.8, 1.2),
                    hu, hv ~ U(-0.1, 0.1) per cell
"""
import numpy as np

G_DEFAULT = 9.81
GAMMA_DEFAULT = 1.4


def rng(seed):
    return np.random.Generator(np.random.Philox(int(seed)))


def centres(nx, ny):
    x = (np.arange(nx) + 0.5) / nx
    y = (np.arange(ny) + 0.5) / ny
    X, Y = np.meshgrid(x, y)  # [ny][nx]
    return X, Y


def acoustics_pulse(n, ny=None, width=200.0):
    ny = n if ny is None else ny
    X, Y = centres(n, ny)
    r2 = (X - 0.5) ** 2 + (Y - 0.5) ** 2
    q = np.zeros((3, ny, n))
    q[0] = np.exp(-width * r2)
    return q


def layered_medium(n, ny=None, rho=(1.0, 2.5), c=(1.0, 0.6), x0=0.5, y0=0.5):
    """Aux fields [2][ny][nx] (rho, c) of a four-block medium: rho jumps at
    x = x0, the sound speed at y = y0."""
    ny = n if ny is None else ny
    X, Y = centres(n, ny)
    return np.stack([np.where(X < x0, rho[0], rho[1]), np.where(Y < y0, c[0], c[1])])


def sw_dam_break(n, seed=0, ny=None, noise=1e-3, h_in=2.0, h_out=1.0, radius=0.3):
    ny = n if ny is None else ny
    X, Y = centres(n, ny)
    r2 = (X - 0.5) ** 2 + (Y - 0.5) ** 2
    q = np.zeros((3, ny, n))
    q[0] = np.where(r2 < radius * radius, h_in, h_out)
    if noise:
        q[0] += noise * rng(seed).uniform(-1.0, 1.0, size=(ny, n))
    return q


def euler_quadrants(n, seed=0, ny=None, gamma=GAMMA_DEFAULT):
    ny = n if ny is None else ny
    X, Y = centres(n, ny)
    g = rng(seed)
    prim = []
    for _ in range(4):  # NE, NW, SW, SE
        rho = g.uniform(0.1, 2.0)
        u = g.uniform(-1.0, 1.0)
        v = g.uniform(-1.0, 1.0)
        p = g.uniform(0.1, 2.0)
        prim.append((rho, u, v, p))
    east = X >= 0.5
    north = Y >= 0.5
    quad = np.where(north & east, 0, np.where(north & ~east, 1, np.where(~north & ~east, 2, 3)))
    q = np.zeros((4, ny, n))
    for k, (rho, u, v, p) in enumerate(prim):
        m = quad == k
        q[0][m] = rho
        q[1][m] = rho * u
        q[2][m] = rho * v
        q[3][m] = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)
    return q, prim


def patch_sides(n_patches, seed=0, lo=16, hi=256):
    g = rng(seed)
    nx = np.rint(np.exp(g.uniform(np.log(lo), np.log(hi), size=n_patches))).astype(np.int64)
    ny = np.rint(np.exp(g.uniform(np.log(lo), np.log(hi), size=n_patches))).astype(np.int64)
    h_in = g.uniform(1.5, 10.0, size=n_patches)
    return nx, ny, h_in


def patch_set(n_patches, seed=0, lo=16, hi=256):
    """List of (nx, ny, q[3][ny][nx]) dam-break patches."""
    nx, ny, h_in = patch_sides(n_patches, seed, lo, hi)
    out = []
    for k in range(n_patches):
        q = sw_dam_break(int(nx[k]), ny=int(ny[k]), noise=0.0, h_in=float(h_in[k]))
        out.append((int(nx[k]), int(ny[k]), q))
    return out


def sw_random_states(n, seed=0, hlo=1e-3, hhi=10.0, ulim=5.0):
    """Independent left/right shallow-water states: h log-uniform in
    [hlo, hhi], u, v uniform in [-ulim, ulim].  Returns ql, qr [3][n]."""
    g = rng(seed)
    out = []
    for _ in range(2):
        h = np.exp(g.uniform(np.log(hlo), np.log(hhi), size=n))
        u = g.uniform(-ulim, ulim, size=n)
        v = g.uniform(-ulim, ulim, size=n)
        out.append(np.stack([h, h * u, h * v]))
    return out[0], out[1]


def euler_random_states(n, seed=0, gamma=GAMMA_DEFAULT):
    g = rng(seed)
    out = []
    for _ in range(2):
        rho = g.uniform(0.1, 2.0, size=n)
        u = g.uniform(-1.0, 1.0, size=n)
        v = g.uniform(-1.0, 1.0, size=n)
        p = g.uniform(0.1, 2.0, size=n)
        E = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)
        out.append(np.stack([rho, rho * u, rho * v, E]))
    return out[0], out[1]


def acoustics_random_states(n, seed=0):
    g = rng(seed)
    return g.normal(size=(3, n)), g.normal(size=(3, n))


def random_field(shape, seed=0, lo=-1.0, hi=1.0):
    return rng(seed).uniform(lo, hi, size=shape)


# ------------------------------------------------------------ learned solver
def surrogate_uniforms(n, seed=0):
    """six uniforms in [0, 1) per training pair, rows (hL, uL, vL, hR, uR, vR)"""
    return rng(seed).random((6, n))


def euler_surrogate_uniforms(n, seed=0):
    """eight uniforms in [0, 1) per Euler training pair, rows
    (rhoL, uL, vL, pL, rhoR, uR, vR, pR)"""
    return rng(seed).random((8, n))


def param_uniforms(n_params, seed=0):
    """uniforms in [0, 1) for the network's initial parameters"""
    return rng(seed).random(n_params)


def batch_orders(epochs, n_batches, seed=0):
    """per epoch, a random order of the batch indices (flat list)"""
    g = rng(seed)
    return [int(v) for _ in range(epochs) for v in g.permutation(n_batches)]


def amr_ring_boxes(n, tile=64, radius=0.3, band=0.75):
    """Refined patches for the dam break on an n x n coarse grid: the tiles
    of tile x tile coarse cells whose centre lies within band * tile cells of
    the circular front (radius `radius` about the centre of the unit
    square).  Returns a list of (ci0, cj0, cw, ch)."""
    import math
    out = []
    for j0 in range(0, n - tile + 1, tile):
        for i0 in range(0, n - tile + 1, tile):
            cx, cy = (i0 + 0.5 * tile) / n - 0.5, (j0 + 0.5 * tile) / n - 0.5
            if abs(math.hypot(cx, cy) - radius) * n < band * tile:
                out.append((i0, j0, tile, tile))
    return out


def sw_noise_device(n, seed, dtype_name="float64"):
    """shallow-water state [3][n][n] made on cuda:0 by torch's seeded device
    generator, for grids too large to stage from the host: h uniform in
    [0.8, 1.2], hu and hv uniform in [-0.1, 0.1]"""
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    q = torch.empty((3, n, n), dtype=getattr(torch, dtype_name), device="cuda")
    q[0].uniform_(0.8, 1.2, generator=g)
    q[1].uniform_(-0.1, 0.1, generator=g)
    q[2].uniform_(-0.1, 0.1, generator=g)
    return q
