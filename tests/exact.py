"""Closed-form and exact solutions used to pin the oracle.

Nothing here calls the oracle or the device library.  Each routine is a
textbook solution written from its mathematical statement:
  - shallow-water exact Riemann solver (Toro, "Shock-Capturing Methods for
    Free-Surface Shallow Flows", 2001, ch. 5: depth function, Newton
    iteration, wave sampling),
  - Euler exact Riemann solver (Toro, "Riemann Solvers and Numerical Methods
    for Fluid Dynamics", 2009, ch. 4),
  - linear acoustics middle state and spectral periodic solution,
  - Lax-Wendroff amplification factors (von Neumann analysis).
"""
import numpy as np


# ---------------------------------------------------------------- fluxes
def sw_flux_x(q, g):
    h, hu, hv = q
    u = hu / h
    return np.stack([hu, hu * u + 0.5 * g * h * h, hv * u])


def euler_flux_x(q, gamma):
    rho, m, n, E = q
    u = m / rho
    p = (gamma - 1.0) * (E - 0.5 * (m * m + n * n) / rho)
    return np.stack([m, m * u + p, n * u, (E + p) * u])


def acoustics_matrix_x(rho, K):
    return np.array([[0.0, K, 0.0], [1.0 / rho, 0.0, 0.0], [0.0, 0.0, 0.0]])


def acoustics_matrix_y(rho, K):
    return np.array([[0.0, 0.0, K], [0.0, 0.0, 0.0], [1.0 / rho, 0.0, 0.0]])


# ---------------------------------------------- shallow water exact Riemann
def _sw_fK(h, hK, g):
    """Depth function and derivative: rarefaction if h <= hK, shock otherwise."""
    cK = np.sqrt(g * hK)
    if h <= hK:
        c = np.sqrt(g * h)
        return 2.0 * (c - cK), g / c
    # g_K(h) = sqrt(g/2 (1/h + 1/hK)), d g_K/dh = -g / (4 h^2 g_K)
    gk = np.sqrt(0.5 * g * (h + hK) / (h * hK))
    f = (h - hK) * gk
    df = gk - (h - hK) * 0.25 * g / (h * h * gk)
    return f, df


def sw_star(hL, uL, hR, uR, g):
    """Star-region depth and velocity (wet bed)."""
    cL, cR = np.sqrt(g * hL), np.sqrt(g * hR)
    # two-rarefaction initial guess
    h = (0.5 * (cL + cR) - 0.25 * (uR - uL)) ** 2 / g
    h = max(h, 1e-8)
    for _ in range(100):
        fL, dL = _sw_fK(h, hL, g)
        fR, dR = _sw_fK(h, hR, g)
        F = fL + fR + uR - uL
        dh = F / (dL + dR)
        hn = max(h - dh, 1e-12)
        if abs(hn - h) <= 1e-15 * h:
            h = hn
            break
        h = hn
    fL, _ = _sw_fK(h, hL, g)
    fR, _ = _sw_fK(h, hR, g)
    u = 0.5 * (uL + uR) + 0.5 * (fR - fL)
    return h, u


def sw_exact(hL, uL, vL, hR, uR, vR, g, xi):
    """Sample the exact solution at similarity coordinates xi = x/t.
    Returns h, u, v arrays."""
    xi = np.asarray(xi, dtype=float)
    hs, us = sw_star(hL, uL, hR, uR, g)
    cL, cR, cs = np.sqrt(g * hL), np.sqrt(g * hR), np.sqrt(g * hs)
    h = np.empty_like(xi)
    u = np.empty_like(xi)
    v = np.where(xi < us, vL, vR).astype(float)
    for k, x in enumerate(xi):
        if x < us:  # left of the contact
            if hs > hL:  # left shock
                qL = np.sqrt(0.5 * (hs + hL) * hs) / hL
                sL = uL - cL * qL
                h[k], u[k] = (hL, uL) if x < sL else (hs, us)
            else:  # left rarefaction
                head, tail = uL - cL, us - cs
                if x <= head:
                    h[k], u[k] = hL, uL
                elif x >= tail:
                    h[k], u[k] = hs, us
                else:
                    c = (uL + 2.0 * cL - x) / 3.0
                    h[k], u[k] = c * c / g, (uL + 2.0 * cL + 2.0 * x) / 3.0
        else:
            if hs > hR:  # right shock
                qR = np.sqrt(0.5 * (hs + hR) * hs) / hR
                sR = uR + cR * qR
                h[k], u[k] = (hR, uR) if x > sR else (hs, us)
            else:
                head, tail = uR + cR, us + cs
                if x >= head:
                    h[k], u[k] = hR, uR
                elif x <= tail:
                    h[k], u[k] = hs, us
                else:
                    c = (-uR + 2.0 * cR + x) / 3.0
                    h[k], u[k] = c * c / g, (uR - 2.0 * cR + 2.0 * x) / 3.0
    return h, u, v


# ------------------------------------------------------ Euler exact Riemann
def _eu_fK(p, rK, pK, gamma):
    cK = np.sqrt(gamma * pK / rK)
    if p > pK:  # shock
        A = 2.0 / ((gamma + 1.0) * rK)
        B = (gamma - 1.0) / (gamma + 1.0) * pK
        sq = np.sqrt(A / (p + B))
        return (p - pK) * sq, sq * (1.0 - 0.5 * (p - pK) / (B + p))
    r = p / pK
    f = 2.0 * cK / (gamma - 1.0) * (r ** ((gamma - 1.0) / (2.0 * gamma)) - 1.0)
    df = 1.0 / (rK * cK) * r ** (-(gamma + 1.0) / (2.0 * gamma))
    return f, df


def euler_star(rL, uL, pL, rR, uR, pR, gamma):
    p = max(0.5 * (pL + pR), 1e-8)
    for _ in range(200):
        fL, dL = _eu_fK(p, rL, pL, gamma)
        fR, dR = _eu_fK(p, rR, pR, gamma)
        pn = max(p - (fL + fR + uR - uL) / (dL + dR), 1e-12)
        if abs(pn - p) <= 1e-15 * p:
            p = pn
            break
        p = pn
    fL, _ = _eu_fK(p, rL, pL, gamma)
    fR, _ = _eu_fK(p, rR, pR, gamma)
    return p, 0.5 * (uL + uR) + 0.5 * (fR - fL)


def euler_exact(rL, uL, vL, pL, rR, uR, vR, pR, gamma, xi):
    """Exact solution sampled at xi = x/t; returns rho, u, v, p."""
    xi = np.asarray(xi, dtype=float)
    ps, us = euler_star(rL, uL, pL, rR, uR, pR, gamma)
    g1 = (gamma - 1.0) / (gamma + 1.0)
    cL, cR = np.sqrt(gamma * pL / rL), np.sqrt(gamma * pR / rR)
    out = np.empty((4, xi.size))
    for k, x in enumerate(xi):
        if x < us:
            if ps > pL:
                rs = rL * (ps / pL + g1) / (g1 * ps / pL + 1.0)
                S = uL - cL * np.sqrt((gamma + 1.0) / (2.0 * gamma) * ps / pL
                                      + (gamma - 1.0) / (2.0 * gamma))
                out[:, k] = (rL, uL, vL, pL) if x < S else (rs, us, vL, ps)
            else:
                rs = rL * (ps / pL) ** (1.0 / gamma)
                cs = cL * (ps / pL) ** ((gamma - 1.0) / (2.0 * gamma))
                if x <= uL - cL:
                    out[:, k] = (rL, uL, vL, pL)
                elif x >= us - cs:
                    out[:, k] = (rs, us, vL, ps)
                else:
                    c = 2.0 / (gamma + 1.0) * (cL + 0.5 * (gamma - 1.0) * (uL - x))
                    u = 2.0 / (gamma + 1.0) * (cL + 0.5 * (gamma - 1.0) * uL + x)
                    r = rL * (c / cL) ** (2.0 / (gamma - 1.0))
                    out[:, k] = (r, u, vL, pL * (c / cL) ** (2.0 * gamma / (gamma - 1.0)))
        else:
            if ps > pR:
                rs = rR * (ps / pR + g1) / (g1 * ps / pR + 1.0)
                S = uR + cR * np.sqrt((gamma + 1.0) / (2.0 * gamma) * ps / pR
                                      + (gamma - 1.0) / (2.0 * gamma))
                out[:, k] = (rR, uR, vR, pR) if x > S else (rs, us, vR, ps)
            else:
                rs = rR * (ps / pR) ** (1.0 / gamma)
                cs = cR * (ps / pR) ** ((gamma - 1.0) / (2.0 * gamma))
                if x >= uR + cR:
                    out[:, k] = (rR, uR, vR, pR)
                elif x <= us + cs:
                    out[:, k] = (rs, us, vR, ps)
                else:
                    c = 2.0 / (gamma + 1.0) * (cR - 0.5 * (gamma - 1.0) * (uR - x))
                    u = 2.0 / (gamma + 1.0) * (-cR + 0.5 * (gamma - 1.0) * uR + x)
                    r = rR * (c / cR) ** (2.0 / (gamma - 1.0))
                    out[:, k] = (r, u, vR, pR * (c / cR) ** (2.0 * gamma / (gamma - 1.0)))
    return out


# ------------------------------------------------------- linear acoustics
def acoustics_middle_state(pL, uL, pR, uR, rho, K):
    """Exact Riemann middle state of p_t + K u_x = 0, u_t + p_x / rho = 0."""
    Z = np.sqrt(K * rho)
    p = 0.5 * (pL + pR) - 0.5 * Z * (uR - uL)
    u = 0.5 * (uL + uR) - 0.5 * (pR - pL) / Z
    return p, u


def acoustics_spectral(p0, t, rho, K):
    """Exact periodic solution on [0,1]^2 from pressure p0 (zero initial
    velocity), by Fourier modes: each mode oscillates at c |k|."""
    ny, nx = p0.shape
    c = np.sqrt(K / rho)
    Z = rho * c
    kx = 2.0 * np.pi * np.fft.fftfreq(nx, d=1.0 / nx)
    ky = 2.0 * np.pi * np.fft.fftfreq(ny, d=1.0 / ny)
    KX, KY = np.meshgrid(kx, ky)
    kk = np.sqrt(KX * KX + KY * KY)
    P = np.fft.fft2(p0)
    cosw = np.cos(c * kk * t)
    sinw = np.sin(c * kk * t)
    safe = np.where(kk > 0, kk, 1.0)
    # p_hat(t) = P cos(c k t); u_hat(t) = -i (k/|k|) P sin(c k t) / Z
    p = np.real(np.fft.ifft2(P * cosw))
    u = np.real(np.fft.ifft2(-1j * (KX / safe) * P * sinw / Z))
    v = np.real(np.fft.ifft2(-1j * (KY / safe) * P * sinw / Z))
    return np.stack([p, u, v])


# -------------------------------------------------- von Neumann factors
def lw_scalar_factor(nu, xi):
    """Lax-Wendroff amplification factor of one sweep at Courant number nu."""
    return 1.0 - nu * nu * (1.0 - np.cos(xi)) - 1j * nu * np.sin(xi)


def lw_matrix_factor(A, nu, xi):
    """Lax-Wendroff amplification matrix I - i nu A sin(xi) - nu^2 A^2 (1 - cos xi)."""
    I = np.eye(A.shape[0])
    return I - 1j * nu * A * np.sin(xi) - nu * nu * (A @ A) * (1.0 - np.cos(xi))
