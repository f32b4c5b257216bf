"""Learned normal Riemann solver for shallow water (the surrogate): CPU oracle.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only users.  The product path never imports this
module, and this module never imports the product package.

The paper's method solves one normal Riemann problem per cell edge and turns
its waves into fluctuations and limited correction fluxes (section 2,
"Threading the Riemann solver"; section 1.2 and Table 1 for the limiters).
The surrogate replaces only that per-edge solve for the shallow-water
equations by a small network; everything downstream is the method as the
plain oracle in ``mco.c`` computes it.  The paper has no learned component:
the network, its inputs and outputs, the projection and the fallback rules
are this project's reading, and each step below says what it computes.

  features    per edge, in the edge's normal frame (h, normal momentum,
              transverse momentum): mean depth h0 = (hL + hR)/2, c0 =
              sqrt(g h0), mean velocities ubar, vbar, and the conserved jump
              scaled to dq^ = (dh/h0, d(hu)/(h0 c0), d(hv)/(h0 c0)) with norm
              m and direction e = dq^/m.  Inputs: (ubar/c0, vbar/c0, m, e).
  network     MLP 6-128-128-128-128-8; after each hidden layer the tanh form
              of GELU, 0.5 x (1 + tanh(sqrt(2/pi) (x + 0.044715 x^3))).
  decoding    speeds s_a = c0 o0, s_b = c0 o1; waves W_a = m S (o2, o3, o4),
              W_b = m S (o5, o6, o7) with S = diag(h0, h0 c0, h0 c0).
  targets     from the plain Roe solver with the Harten-Hyman fix: s_a, s_b
              are its acoustic speeds s1 < 0 < s3 and W_a = A-dQ / s1,
              W_b = A+dQ / s3, so that exact outputs reproduce Roe's
              fluctuations.
  projection  the smallest change of (W_a, W_b) at fixed speeds that makes
              s_a W_a + s_b W_b equal f(qR) - f(qL): with r the residual and
              D = s_a^2 + s_b^2, W_a += s_a r / D and W_b += s_b r / D.  Then
              A-dQ + A+dQ = f(qR) - f(qL), so the update stays conservative.
  fallback    flagged edges use the plain Roe solver, or HLLE where Roe's
              middle depth is not positive.  Flags: outside the training box
              (h < 1e-3, h > 10, |u| > 5 or |v| > 5 on a side), near-dry
              (min h < 1e-2), not subsonic on a side (|u| >= c, which covers
              every transonic edge), or a degenerate projection (D not > 0).
              Flags are decided in FP32, as the device decides them.
  training    masked mean-squared error over the 8 outputs; Adam (Kingma and
              Ba 2015, Algorithm 1).
  step        the split wave-propagation step of ``mco.c`` written over whole
              sweeps (FVMHP ch. 6 and 19), with the edge solves above.

FP64 throughout.  With ``emulate=True`` the network's matrix operands are
rounded to bfloat16 (through FP32, nearest-even) and each layer's sums to
FP32, which is what the device's BF16 matrix cores with FP32 accumulation
compute up to the order of the FP32 additions.
"""
import numpy as np

from . import (BC_EXTRAP, BC_PERIODIC, LIM_FIRST_ORDER, LIM_MC, LIM_MINMOD, LIM_NONE,
               LIM_SUPERBEE, LIM_VANLEER, SW_HLLE, SW_ROE, params, rp2 as _rp2)

WIDTHS = (6, 128, 128, 128, 128, 8)
NLAYERS = len(WIDTHS) - 1
NPARAMS = sum(WIDTHS[i + 1] * WIDTHS[i] + WIDTHS[i + 1] for i in range(NLAYERS))

# training box and flag thresholds (decided in FP32)
H_LO, H_HI, U_MAX, H_DRY = 1e-3, 10.0, 5.0, 1e-2
FLAG_OOD, FLAG_DRY, FLAG_NONSUB, FLAG_PROJ = 1, 2, 4, 8

GELU_K = np.sqrt(2.0 / np.pi)
GELU_A = 0.044715


# ---------------------------------------------------------------- parameters
def layer_slices():
    """(weight slice, bias slice, out, in) per layer in the flat vector:
    W_l row-major [out][in] followed by b_l [out], layer after layer."""
    out, off = [], 0
    for l in range(NLAYERS):
        ni, no = WIDTHS[l], WIDTHS[l + 1]
        ws = slice(off, off + no * ni)
        off += no * ni
        bs = slice(off, off + no)
        off += no
        out.append((ws, bs, no, ni))
    return out


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    assert theta.shape == (NPARAMS,)
    return [(theta[ws].reshape(no, ni), theta[bs]) for ws, bs, no, ni in layer_slices()]


def pack(layers):
    return np.concatenate([np.concatenate([W.ravel(), b.ravel()]) for W, b in layers])


# ---------------------------------------------------------------- rounding
def f32(x):
    return np.asarray(x, dtype=np.float64).astype(np.float32).astype(np.float64)


def bf16(x):
    """Round to bfloat16 through FP32 (nearest, ties to even); FP64 result."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float64).astype(np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    u = ((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


# ---------------------------------------------------------------- network
def gelu(x):
    return 0.5 * x * (1.0 + np.tanh(GELU_K * (x + GELU_A * x * x * x)))


def gelu_grad(x):
    t = np.tanh(GELU_K * (x + GELU_A * x * x * x))
    return 0.5 * (1.0 + t) + 0.5 * x * (1.0 - t * t) * GELU_K * (1.0 + 3.0 * GELU_A * x * x)


def forward(theta, X, emulate=False):
    """Network outputs [n][8] for inputs X [n][6], plus the cache the
    backward pass needs (layer inputs as used, pre-activations)."""
    a = np.asarray(X, dtype=np.float64)
    ins, zs = [], []
    for l, (W, b) in enumerate(unpack(theta)):
        if emulate:
            a, W, b = bf16(a), bf16(W), f32(b)
        z = a @ W.T + b
        if emulate:
            z = f32(z)
        ins.append(a)
        zs.append(z)
        a = gelu(z) if l < NLAYERS - 1 else z
    return a, (ins, zs)


def loss(out, Y, mask):
    """Masked mean-squared error: sum over kept rows and all 8 outputs,
    divided by 8 times the number of kept rows."""
    w = np.asarray(mask, dtype=np.float64)[:, None]
    cnt = max(float(w.sum()), 1.0)
    d = out - Y
    return float((w * d * d).sum() / (out.shape[1] * cnt)), 2.0 * w * d / (out.shape[1] * cnt)


def backward(theta, cache, dout, emulate=False):
    """Gradient of the loss w.r.t. the flat parameter vector, by the chain
    rule through each affine map and GELU.  With emulate, each layer's
    output gradient is rounded to bfloat16 before both products (the bias
    gradient uses it unrounded) and the sums to FP32."""
    ins, zs = cache
    layers = unpack(theta)
    grads = [None] * NLAYERS
    dz = np.asarray(dout, dtype=np.float64)
    for l in range(NLAYERS - 1, -1, -1):
        W, _ = layers[l]
        db = dz.sum(axis=0)
        dzq = bf16(dz) if emulate else dz
        dW = dzq.T @ ins[l]
        if emulate:
            dW, db = f32(dW), f32(db)
        grads[l] = (dW, db)
        if l > 0:
            da = dzq @ (bf16(W) if emulate else W)
            if emulate:
                da = f32(da)
            dz = da * gelu_grad(zs[l - 1])
            if emulate:
                dz = f32(dz)
    return pack(grads)


def loss_and_grad(theta, X, Y, mask, emulate=False):
    out, cache = forward(theta, X, emulate)
    L, dout = loss(out, Y, mask)
    return L, backward(theta, cache, dout, emulate)


def adam(theta, grad, m, v, t, lr, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma and Ba 2015, Algorithm 1) at step t >= 1.
    Returns the new (theta, m, v)."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------------------- edges
def to_normal(q, ixy):
    """(h, normal momentum, transverse momentum) of [3][n] states."""
    q = np.asarray(q, dtype=np.float64)
    return q if ixy == 1 else q[[0, 2, 1]]


def from_normal(w, ixy):
    return w if ixy == 1 else w[[0, 2, 1]]


def sw_flux(q, g):
    """normal flux (hu, hu^2/h + g h^2/2, hu hv/h) of normal-frame states"""
    h, mu, mv = q
    u = mu / h
    return np.stack([mu, mu * u + 0.5 * g * h * h, mv * u])


def features(ql, qr, g):
    """Network inputs [n][6] and the decoding scales (h0, c0, m) of
    normal-frame edge states ql, qr [3][n]."""
    hL, muL, mvL = ql
    hR, muR, mvR = qr
    h0 = 0.5 * (hL + hR)
    c0 = np.sqrt(g * h0)
    ub = 0.5 * (muL / hL + muR / hR)
    vb = 0.5 * (mvL / hL + mvR / hR)
    dq = np.stack([(hR - hL) / h0, (muR - muL) / (h0 * c0), (mvR - mvL) / (h0 * c0)])
    m = np.sqrt(dq[0] * dq[0] + dq[1] * dq[1] + dq[2] * dq[2])
    e = np.where(m > 0.0, dq / np.where(m > 0.0, m, 1.0), 0.0)
    X = np.stack([ub / c0, vb / c0, m, e[0], e[1], e[2]], axis=1)
    return X, h0, c0, m


def flags(ql, qr, g):
    """Fallback flag bits per edge, decided in FP32 on normal-frame states."""
    f = np.float32
    gg = f(g)
    out = np.zeros(np.asarray(ql).shape[1], dtype=np.int32)
    hmin = None
    for q in (ql, qr):
        h, mu, mv = (np.asarray(x, dtype=np.float64).astype(f) for x in q)
        ood = (h < f(H_LO)) | (h > f(H_HI)) | (np.abs(mu) > f(U_MAX) * h) | \
              (np.abs(mv) > f(U_MAX) * h)
        nonsub = mu * mu >= ((gg * h) * h) * h
        out |= np.where(ood, FLAG_OOD, 0) | np.where(nonsub, FLAG_NONSUB, 0)
        hmin = h if hmin is None else np.minimum(hmin, h)
    out |= np.where(hmin < f(H_DRY), FLAG_DRY, 0)
    return out.astype(np.int32)


def decode(out, h0, c0, m):
    """speeds [2][n] and waves [2][3][n] from network outputs [n][8]"""
    o = np.asarray(out, dtype=np.float64).T
    S = np.stack([h0, h0 * c0, h0 * c0])
    s = np.stack([c0 * o[0], c0 * o[1]])
    W = np.stack([m * S * o[2:5], m * S * o[5:8]])
    return s, W


def project(s, W, df):
    """Smallest change of the two waves (Euclidean, at fixed speeds) after
    which s_a W_a + s_b W_b = df.  Returns (W, ok) with ok false where the
    speeds are degenerate."""
    r = df - (s[0] * W[0] + s[1] * W[1])
    D = s[0] * s[0] + s[1] * s[1]
    ok = np.isfinite(D) & (D > 0.0)
    Dn = np.where(ok, D, 1.0)
    Wp = np.stack([W[0] + s[0] * r / Dn, W[1] + s[1] * r / Dn])
    return Wp, ok


def entropy_fix_active(ql, qr, waves, g):
    """True where Roe's middle depths are not positive or the Harten-Hyman
    fix splits a wave: the characteristic speed of family 1 (left state and
    ql + W1) or family 3 (qr - W3 and right state) changes sign from
    negative to positive across the wave (normal-frame states)."""
    q1 = ql + waves[0]
    q2 = qr - waves[2]
    ok = (q1[0] > 0.0) & (q2[0] > 0.0)
    h1 = np.where(ok, q1[0], 1.0)
    h2 = np.where(ok, q2[0], 1.0)
    l1l = ql[1] / ql[0] - np.sqrt(g * ql[0])
    l1r = q1[1] / h1 - np.sqrt(g * h1)
    l3l = q2[1] / h2 + np.sqrt(g * h2)
    l3r = qr[1] / qr[0] + np.sqrt(g * qr[0])
    return ~ok | ((l1l < 0.0) & (l1r > 0.0)) | ((l3l < 0.0) & (l3r > 0.0))


def labels(ql, qr, g):
    """Training targets [n][8], network inputs [n][6] and the mask of edges
    that enter the loss, for normal-frame (x-normal) states ql, qr [3][n].
    An edge is kept when no flag is set, the jump is not zero, the acoustic
    speeds satisfy s1 < 0 < s3, Roe's middle depths are positive and the
    entropy fix leaves the fluctuations alone (so that W_a = A-dQ / s1 and
    W_b = A+dQ / s3 stay bounded)."""
    P = params(g=g)
    waves, speeds, amdq, apdq, _ = _rp2(SW_ROE, P, 1, ql, qr)
    X, h0, c0, m = features(ql, qr, g)
    s1, s3 = speeds[0], speeds[2]
    keep = (flags(ql, qr, g) == 0) & (m > 0.0) & (s1 < 0.0) & (s3 > 0.0) & \
        ~entropy_fix_active(ql, qr, waves, g)
    S = np.stack([h0, h0 * c0, h0 * c0])
    den = np.where(keep, m, 1.0) * S
    Wa = amdq / np.where(keep, s1, -1.0) / den
    Wb = apdq / np.where(keep, s3, 1.0) / den
    Y = np.concatenate([np.stack([s1 / c0, s3 / c0]), Wa, Wb]).T
    Y = np.where(keep[:, None], Y, 0.0)
    return Y, X, keep


def states_from_uniforms(U):
    """Left/right states [3][n] from six uniforms per pair in [0, 1):
    rows (hL, uL, vL, hR, uR, vR); h log-uniform in [1e-3, 10], u and v
    uniform in [-5, 5]."""
    U = np.asarray(U, dtype=np.float64)
    lo, hi = np.log(H_LO), np.log(H_HI)
    out = []
    for k in (0, 3):
        h = np.exp(lo + (hi - lo) * U[k])
        u = -U_MAX + 2.0 * U_MAX * U[k + 1]
        v = -U_MAX + 2.0 * U_MAX * U[k + 2]
        out.append(np.stack([h, h * u, h * v]))
    return out[0], out[1]


def rp2(theta, ixy, ql, qr, g, emulate=True, outputs=None):
    """Surrogate edge solves for states ql, qr [3][n] in grid orientation.
    Returns waves [3][3][n] (slot 1 empty on network edges), speeds [3][n],
    amdq, apdq [3][n] and the flag bits per edge.  ``outputs`` replaces the
    network's outputs (for checks with exact targets)."""
    nl, nr = to_normal(ql, ixy), to_normal(qr, ixy)
    n = nl.shape[1]
    fl = flags(nl, nr, g)
    X, h0, c0, m = features(nl, nr, g)
    if outputs is None:
        outputs, _ = forward(theta, X, emulate)
    s, W = decode(outputs, h0, c0, m)
    df = sw_flux(nr, g) - sw_flux(nl, g)
    W, ok = project(s, W, df)
    fl = fl | np.where(ok, 0, FLAG_PROJ).astype(np.int32)

    waves = np.zeros((3, 3, n))
    speeds = np.zeros((3, n))
    waves[0], waves[2] = W[0], W[1]
    speeds[0], speeds[2] = s[0], s[1]
    amdq = np.minimum(s[0], 0.0) * W[0] + np.minimum(s[1], 0.0) * W[1]
    apdq = np.maximum(s[0], 0.0) * W[0] + np.maximum(s[1], 0.0) * W[1]

    fb = np.nonzero(fl)[0]
    if fb.size:
        P = params(g=g)
        a, b = nl[:, fb], nr[:, fb]
        rw, rs, ram, rap, _ = _rp2(SW_ROE, P, 1, a, b)
        bad = ~(a[0] + rw[0][0] > 0.0)
        if bad.any():
            hw, hs, ham, hap, _ = _rp2(SW_HLLE, P, 1, a[:, bad], b[:, bad])
            rw[:, :, bad], rs[:, bad], ram[:, bad], rap[:, bad] = hw, hs, ham, hap
        waves[:, :, fb], speeds[:, fb], amdq[:, fb], apdq[:, fb] = rw, rs, ram, rap
    waves = np.stack([from_normal(waves[p], ixy) for p in range(3)])
    return waves, speeds, from_normal(amdq, ixy), from_normal(apdq, ixy), fl


# ---------------------------------------------------------------- split step
def phi(limiter, theta):
    """Wave-limiter functions (paper, Table 1; FVMHP ch. 6)."""
    t = np.asarray(theta, dtype=np.float64)
    if limiter == LIM_NONE:
        return np.ones_like(t)
    if limiter == LIM_MINMOD:
        return np.maximum(0.0, np.minimum(1.0, t))
    if limiter == LIM_SUPERBEE:
        return np.maximum(0.0, np.maximum(np.minimum(1.0, 2.0 * t), np.minimum(2.0, t)))
    if limiter == LIM_VANLEER:
        return (t + np.abs(t)) / (1.0 + np.abs(t))
    if limiter == LIM_MC:
        return np.maximum(0.0, np.minimum(np.minimum(0.5 * (1.0 + t), 2.0), 2.0 * t))
    return np.zeros_like(t)


def _ghost(n, bc):
    i = np.arange(-2, n + 2)
    return np.mod(i, n) if bc == BC_PERIODIC else np.clip(i, 0, n - 1)


def sweep(rp, q, ixy, nu, d, limiter, bc):
    """One sweep of the whole grid: every line along x (ixy = 1) or y
    (ixy = 2) gets its ghost cells, edge solves, limited correction fluxes
    and conservative update.  rp(ixy, ql, qr) -> (waves, speeds, amdq, apdq,
    flags) on [3][N] edge states.  Returns (q*, smax, flags)."""
    lines = q if ixy == 1 else q.transpose(0, 2, 1)   # [3][L][n]
    _, L, n = lines.shape
    G = lines[:, :, _ghost(n, bc)]                     # [3][L][n+4]
    ne = n + 3
    ql = G[:, :, :-1].reshape(3, -1)
    qr = G[:, :, 1:].reshape(3, -1)
    waves, s, amdq, apdq, fl = rp(ixy, ql, qr)
    waves = waves.reshape(3, 3, L, ne)
    s = s.reshape(3, L, ne)
    amdq, apdq = amdq.reshape(3, L, ne), apdq.reshape(3, L, ne)

    k = np.arange(1, n + 2)
    smax = float((np.abs(s[:, :, k]) / d).max())
    ftil = np.zeros((3, L, ne))
    if limiter != LIM_FIRST_ORDER:
        for p in range(3):
            sp = s[p][:, k]
            up = np.where(sp > 0.0, k - 1, k + 1)
            wk = waves[p][:, :, k]
            wu = np.take_along_axis(waves[p], np.broadcast_to(up, wk.shape), axis=2)
            wn = wk[0] * wk[0] + wk[1] * wk[1] + wk[2] * wk[2]
            wd = wu[0] * wk[0] + wu[1] * wk[1] + wu[2] * wk[2]
            ph = np.where(wn == 0.0, 0.0, phi(limiter, wd / np.where(wn == 0.0, 1.0, wn)))
            c = 0.5 * np.abs(sp) * (1.0 - nu * np.abs(sp))
            ftil[:, :, k] += c * (ph * wk)
    i = np.arange(n)
    kl, kr = i + 1, i + 2
    out = lines - nu * (apdq[:, :, kl] + amdq[:, :, kr]) - nu * (ftil[:, :, kr] - ftil[:, :, kl])
    out = out if ixy == 1 else out.transpose(0, 2, 1)
    return np.ascontiguousarray(out), smax, fl


def step2d(rp, q, dx, dy, dt, limiter, bc):
    """Godunov-split step: x-sweep on q^n with full dt, then the y-sweep on
    the result with its ghost cells refilled.  Returns (q^{n+1}, smax,
    number of flagged edges)."""
    q = np.asarray(q, dtype=np.float64)
    qs, sx, fx = sweep(rp, q, 1, dt / dx, dx, limiter, bc)
    qn, sy, fy = sweep(rp, qs, 2, dt / dy, dy, limiter, bc)
    return qn, max(sx, sy), int(np.count_nonzero(fx) + np.count_nonzero(fy))


def plain_rp(g, solver=SW_ROE):
    """edge solver of the plain method, in the form sweep() takes"""
    P = params(g=g)

    def rp(ixy, ql, qr):
        w, s, am, ap, _ = _rp2(solver, P, ixy, ql, qr)
        return w, s, am, ap, np.zeros(ql.shape[1], dtype=np.int32)
    return rp


def surrogate_rp(theta, g, emulate=True):
    def rp(ixy, ql, qr):
        return rp2(theta, ixy, ql, qr, g, emulate)
    return rp


def init_params(U):
    """Initial parameters from uniforms U [NPARAMS] in [0, 1): weights
    uniform in +-sqrt(6 / (fan_in + fan_out)) (Glorot and Bengio 2010),
    biases zero."""
    U = np.asarray(U, dtype=np.float64)
    theta = np.zeros(NPARAMS)
    for ws, bs, no, ni in layer_slices():
        a = np.sqrt(6.0 / (ni + no))
        theta[ws] = -a + 2.0 * a * U[ws]
    return theta
