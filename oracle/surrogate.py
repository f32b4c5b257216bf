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

from . import (BC_EXTRAP, BC_PERIODIC, EULER_ROE, LIM_FIRST_ORDER, LIM_MC, LIM_MINMOD, LIM_NONE,
               LIM_SUPERBEE, LIM_VANLEER, SW_HLLE, SW_ROE, params, rp2 as _rp2)

WIDTHS = (6, 128, 128, 128, 128, 8)          # shallow water
EU_WIDTHS = (7, 128, 128, 128, 128, 15)      # Euler
NLAYERS = len(WIDTHS) - 1


def nparams(widths):
    return sum(widths[i + 1] * widths[i] + widths[i + 1] for i in range(len(widths) - 1))


NPARAMS = nparams(WIDTHS)
EU_NPARAMS = nparams(EU_WIDTHS)


def widths_of(theta):
    return {NPARAMS: WIDTHS, EU_NPARAMS: EU_WIDTHS}[len(theta)]

# training box and flag thresholds (decided in FP32)
H_LO, H_HI, U_MAX, H_DRY = 1e-3, 10.0, 5.0, 1e-2
FLAG_OOD, FLAG_DRY, FLAG_NONSUB, FLAG_PROJ = 1, 2, 4, 8

GELU_K = np.sqrt(2.0 / np.pi)
GELU_A = 0.044715


# ---------------------------------------------------------------- parameters
def layer_slices(widths=WIDTHS):
    """(weight slice, bias slice, out, in) per layer in the flat vector:
    W_l row-major [out][in] followed by b_l [out], layer after layer."""
    out, off = [], 0
    for l in range(len(widths) - 1):
        ni, no = widths[l], widths[l + 1]
        ws = slice(off, off + no * ni)
        off += no * ni
        bs = slice(off, off + no)
        off += no
        out.append((ws, bs, no, ni))
    return out


def unpack(theta):
    theta = np.asarray(theta, dtype=np.float64)
    return [(theta[ws].reshape(no, ni), theta[bs])
            for ws, bs, no, ni in layer_slices(widths_of(theta))]


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


def bf16_spacing(q, v):
    """Distance from the bfloat16 value q = bf16(v) to its neighbour on the
    side of v (away from zero when |v| >= |q|), and the distance from v to
    the rounding midpoint between the two.  bfloat16 keeps 8 significant
    bits, so the spacing at |q| in [2^e, 2^(e+1)) is 2^(e-7); just below a
    power of two it is half that."""
    q = np.asarray(q, dtype=np.float64)
    v = np.asarray(v, dtype=np.float64)
    aq = np.abs(q)
    _, e = np.frexp(np.where(aq > 0, aq, 1.0))          # aq = m 2^e, m in [0.5, 1)
    up = np.ldexp(1.0, e - 8)                            # spacing above |q|
    pow2 = np.ldexp(0.5, e) == aq
    down = np.where(pow2, 0.5 * up, up)                  # spacing below |q|
    away = np.abs(v) >= aq
    side = np.where(away, up, down)
    dist = np.where(v == q, 0.5 * np.minimum(up, down), 0.5 * side - np.abs(v - q))
    side = np.where(aq > 0, side, np.abs(v) + np.ldexp(1.0, -126))
    return side, dist


def rounding_spread(theta, X, inputs=False, rel=2.0 ** -17):
    """How far, per row and output, an evaluation of the network with BF16
    operands and FP32 sums may lie from forward(theta, X, emulate=True)
    when its values differ from the emulation's by rounding error only.

    Two such evaluations agree on an operand (an input, a hidden
    activation) until the value it rounds lies near a rounding midpoint;
    once one operand rounds to the other BF16 neighbour, the values after it
    move by about their own BF16 spacing and their roundings decorrelate.
    The model taken here is the fully decorrelated one: every hidden operand
    (and every input when ``inputs``, i.e. when the inputs are computed
    apart on each side) carries an independent difference of rounding
    errors, each uniform on [-u/2, u/2] on either side, so of variance
    u^2 / 6, u the BF16 spacing at the operand.  To first order the output
    changes by the sum of these times d out / d operand (back-propagation
    through the emulated network); its standard deviation is returned as
    ``sigma``.  ``floor`` is the FP32 rounding of the final sums, rel times
    the sum of their absolute terms (rel = 2^-17 = 128 units of FP32
    rounding: any order of a 128-term FP32 sum).

    Returns (sigma, floor), each [n][nout]."""
    a = np.asarray(X, dtype=np.float64)
    layers = unpack(theta)
    nl = len(layers)
    zs, Wq, spc = [], [], []
    for l, (W, b) in enumerate(layers):
        q = bf16(a)
        u, _ = bf16_spacing(q, a)
        spc.append(u if (l > 0 or inputs) else np.zeros_like(u))
        Wl = bf16(W)
        Wq.append(Wl)
        z = f32(q @ Wl.T + f32(b))
        zs.append(z)
        if l < nl - 1:
            a = gelu(z)
        else:
            out_s = np.abs(q) @ np.abs(Wl).T + np.abs(f32(b))
    n, nout = out_s.shape
    var = np.zeros((n, nout))
    for j in range(nout):
        dz = np.zeros((n, nout))
        dz[:, j] = 1.0
        for l in range(nl - 1, -1, -1):
            da = dz @ Wq[l]
            var[:, j] += ((da * spc[l]) ** 2).sum(axis=1) / 6.0
            if l > 0:
                dz = da * gelu_grad(zs[l - 1])
    return np.sqrt(var), rel * out_s


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
    """Smallest change of the waves W [k][meqn][n] (Euclidean, at fixed
    speeds s [k][n]) after which sum_p s_p W_p = df: W_p += s_p r / D with
    r = df - sum_p s_p W_p and D = sum_p s_p^2.  Returns (W, ok) with ok
    false where the speeds are degenerate."""
    r = df - s[0] * W[0]
    D = s[0] * s[0]
    for p in range(1, s.shape[0]):
        r = r - s[p] * W[p]
        D = D + s[p] * s[p]
    ok = np.isfinite(D) & (D > 0.0)
    Dn = np.where(ok, D, 1.0)
    Wp = np.stack([W[p] + s[p] * r / Dn for p in range(s.shape[0])])
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
    lines = q if ixy == 1 else q.transpose(0, 2, 1)   # [meqn][L][n]
    meqn, L, n = lines.shape
    G = lines[:, :, _ghost(n, bc)]                     # [meqn][L][n+4]
    ne = n + 3
    ql = G[:, :, :-1].reshape(meqn, -1)
    qr = G[:, :, 1:].reshape(meqn, -1)
    waves, s, amdq, apdq, fl = rp(ixy, ql, qr)
    mw = waves.shape[0]
    waves = waves.reshape(mw, meqn, L, ne)
    s = s.reshape(mw, L, ne)
    amdq, apdq = amdq.reshape(meqn, L, ne), apdq.reshape(meqn, L, ne)

    k = np.arange(1, n + 2)
    smax = float((np.abs(s[:, :, k]) / d).max())
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


def init_params(U, widths=WIDTHS):
    """Initial parameters from uniforms U [nparams] in [0, 1): weights
    uniform in +-sqrt(6 / (fan_in + fan_out)) (Glorot and Bengio 2010),
    biases zero."""
    U = np.asarray(U, dtype=np.float64)
    theta = np.zeros(nparams(widths))
    for ws, bs, no, ni in layer_slices(widths):
        a = np.sqrt(6.0 / (ni + no))
        theta[ws] = -a + 2.0 * a * U[ws]
    return theta


# ---------------------------------------------------------------- Euler
# The same construction for the Euler equations (gamma-law gas), normal frame
# (rho, normal momentum, transverse momentum, E), with rho0 = (rhoL+rhoR)/2,
# p0 = (pL+pR)/2, c0 = sqrt(gamma p0/rho0):
#   inputs   (ubar/c0, vbar/c0, m, e) where the scaled conserved jump
#            (drho/rho0, d(rho u)/(rho0 c0), d(rho v)/(rho0 c0), dE/(rho0 c0^2))
#            = m e, |e| = 1 (7 inputs; invariant under rho -> a rho,
#            u -> b u, p -> a b^2 p)
#   outputs  three speeds c0 (o0, o1, o2) and three waves m S (o3..o6),
#            m S (o7..o10), m S (o11..o14), S = diag(rho0, rho0 c0, rho0 c0,
#            rho0 c0^2): the two acoustic waves and one contact wave
#   targets  the plain Euler Roe solver (Harten-Hyman on families 1 and 4):
#            speeds s1, u_hat, s4 and waves W1, W2 + W3, W4 (the entropy and
#            shear waves travel at the same speed u_hat, so their sum gives
#            the same fluctuations; exact outputs reproduce Roe's)
#   box      rho, p in [0.05, 10], |u|, |v| <= 2 (training draws: rho, p
#            log-uniform, u, v uniform)
#   flags    FP32, products only (p rho = (gamma-1)(E rho - |rho u|^2/2)):
#            outside the box on a side, or not subsonic on a side
#            ((rho u)^2 >= gamma p rho); degenerate projection
#   fallback the plain Euler solver (Roe + HH, HLLE where Roe fails)
EU_RHO = (0.05, 10.0)
EU_P = (0.05, 10.0)
EU_U = 2.0


def eu_pressure(q, gm):
    return (gm - 1.0) * (q[3] - 0.5 * (q[1] * q[1] + q[2] * q[2]) / q[0])


def eu_flux(q, gm):
    """normal flux of normal-frame Euler states [4][n]"""
    p = eu_pressure(q, gm)
    u = q[1] / q[0]
    return np.stack([q[1], q[1] * u + p, q[2] * u, (q[3] + p) * u])


def eu_to_normal(q, ixy):
    q = np.asarray(q, dtype=np.float64)
    return q if ixy == 1 else q[[0, 2, 1, 3]]


eu_from_normal = eu_to_normal


def eu_features(ql, qr, gm):
    pl, pr = eu_pressure(ql, gm), eu_pressure(qr, gm)
    r0 = 0.5 * (ql[0] + qr[0])
    p0 = 0.5 * (pl + pr)
    c0 = np.sqrt(gm * p0 / r0)
    ub = 0.5 * (ql[1] / ql[0] + qr[1] / qr[0])
    vb = 0.5 * (ql[2] / ql[0] + qr[2] / qr[0])
    S = np.stack([r0, r0 * c0, r0 * c0, r0 * c0 * c0])
    dq = (qr - ql) / S
    m = np.sqrt(dq[0] * dq[0] + dq[1] * dq[1] + dq[2] * dq[2] + dq[3] * dq[3])
    e = np.where(m > 0.0, dq / np.where(m > 0.0, m, 1.0), 0.0)
    X = np.stack([ub / c0, vb / c0, m, e[0], e[1], e[2], e[3]], axis=1)
    return X, S, c0, m


def eu_flags(ql, qr, gm):
    f = np.float32
    g1 = f(gm - 1.0)
    gg = f(gm)
    out = np.zeros(np.asarray(ql).shape[1], dtype=np.int32)
    for q in (ql, qr):
        r, mu, mv, E = (np.asarray(x, dtype=np.float64).astype(f) for x in q)
        pr = g1 * (E * r - f(0.5) * (mu * mu + mv * mv))        # p rho
        ood = ~(r >= f(EU_RHO[0])) | ~(r <= f(EU_RHO[1])) | \
            ~(pr >= f(EU_P[0]) * r) | ~(pr <= f(EU_P[1]) * r) | \
            ~(np.abs(mu) <= f(EU_U) * r) | ~(np.abs(mv) <= f(EU_U) * r)
        nonsub = mu * mu >= gg * pr
        out |= np.where(ood, FLAG_OOD, 0) | np.where(nonsub, FLAG_NONSUB, 0)
    return out.astype(np.int32)


EU_SLOTS = (0, 1, 3)   # record slots of the three network waves (slot 2 empty)


def eu_decode(out, S, c0, m):
    o = np.asarray(out, dtype=np.float64).T
    s = np.stack([c0 * o[0], c0 * o[1], c0 * o[2]])
    W = np.stack([m * S * o[3:7], m * S * o[7:11], m * S * o[11:15]])
    return s, W


def eu_roe_plain(ql, qr, gm):
    """plain Euler solver on normal-frame states, with its per-edge HLLE
    fallback marked (HLLE leaves slots 1 and 2 empty at zero speed)"""
    P = params(gamma=gm)
    w, s, am, ap, _ = _rp2(EULER_ROE, P, 1, ql, qr)
    hll = (s[1] == 0.0) & (s[2] == 0.0) & ~w[1].any(axis=0) & ~w[2].any(axis=0)
    return w, s, am, ap, hll


def eu_fix_active(ql, qr, w, gm):
    """Roe intermediate states next to the acoustic waves not physical, or the
    Harten-Hyman transonic test true on family 1 or 4"""
    q1 = ql + w[0]
    q3 = qr - w[3]
    ok = (q1[0] > 0.0) & (q3[0] > 0.0)
    q1s = np.where(ok, q1, 1.0)
    q3s = np.where(ok, q3, 1.0)
    p1, p3 = eu_pressure(q1s, gm), eu_pressure(q3s, gm)
    ok &= (p1 > 0.0) & (p3 > 0.0)
    p1, p3 = np.where(ok, p1, 1.0), np.where(ok, p3, 1.0)
    pl, pr = eu_pressure(ql, gm), eu_pressure(qr, gm)
    l1l = ql[1] / ql[0] - np.sqrt(gm * pl / ql[0])
    l1r = q1s[1] / q1s[0] - np.sqrt(gm * p1 / q1s[0])
    l4l = q3s[1] / q3s[0] + np.sqrt(gm * p3 / q3s[0])
    l4r = qr[1] / qr[0] + np.sqrt(gm * pr / qr[0])
    return ~ok | ((l1l < 0.0) & (l1r > 0.0)) | ((l4l < 0.0) & (l4r > 0.0))


def eu_labels(ql, qr, gm):
    """Targets [n][15], inputs [n][7] and the loss mask for normal-frame
    (x-normal) Euler states: kept when no flag is set, the jump is not zero,
    the plain solver took Roe (no HLLE), s1 < 0 < s4, and the entropy fix
    leaves the fluctuations alone."""
    w, s, am, ap, hll = eu_roe_plain(ql, qr, gm)
    X, S, c0, m = eu_features(ql, qr, gm)
    keep = (eu_flags(ql, qr, gm) == 0) & (m > 0.0) & ~hll & (s[0] < 0.0) & (s[3] > 0.0) & \
        ~eu_fix_active(ql, qr, w, gm)
    den = np.where(keep, m, 1.0) * S
    Y = np.concatenate([np.stack([s[0] / c0, s[1] / c0, s[3] / c0]),
                        w[0] / den, (w[1] + w[2]) / den, w[3] / den]).T
    Y = np.where(keep[:, None], Y, 0.0)
    return Y, X, keep


def eu_states_from_uniforms(U, gm=1.4):
    """Left/right Euler states [4][n] from eight uniforms per pair, rows
    (rhoL, uL, vL, pL, rhoR, uR, vR, pR): rho, p log-uniform in the box,
    u, v uniform in [-2, 2]."""
    U = np.asarray(U, dtype=np.float64)
    out = []
    for k in (0, 4):
        r = np.exp(np.log(EU_RHO[0]) + (np.log(EU_RHO[1]) - np.log(EU_RHO[0])) * U[k])
        u = -EU_U + 2.0 * EU_U * U[k + 1]
        v = -EU_U + 2.0 * EU_U * U[k + 2]
        p = np.exp(np.log(EU_P[0]) + (np.log(EU_P[1]) - np.log(EU_P[0])) * U[k + 3])
        out.append(np.stack([r, r * u, r * v, p / (gm - 1.0) + 0.5 * r * (u * u + v * v)]))
    return out[0], out[1]


def eu_rp2(theta, ixy, ql, qr, gm, emulate=True, outputs=None):
    """Euler surrogate edge solves (grid orientation in and out): waves
    [4][4][n] (slot 2 empty on network edges), speeds [4][n],
    amdq, apdq [4][n], flag bits."""
    nl, nr = eu_to_normal(ql, ixy), eu_to_normal(qr, ixy)
    n = nl.shape[1]
    fl = eu_flags(nl, nr, gm)
    X, S, c0, m = eu_features(nl, nr, gm)
    if outputs is None:
        outputs, _ = forward(theta, np.where(fl[:, None] == 0, X, 0.0), emulate)
    s, W = eu_decode(outputs, S, c0, m)
    W, ok = project(s, W, eu_flux(nr, gm) - eu_flux(nl, gm))
    fl = fl | np.where(ok, 0, FLAG_PROJ).astype(np.int32)
    waves = np.zeros((4, 4, n))
    speeds = np.zeros((4, n))
    amdq = np.zeros((4, n))
    apdq = np.zeros((4, n))
    for k, slot in enumerate(EU_SLOTS):
        waves[slot], speeds[slot] = W[k], s[k]
        amdq = amdq + np.minimum(s[k], 0.0) * W[k]
        apdq = apdq + np.maximum(s[k], 0.0) * W[k]
    fb = np.nonzero(fl)[0]
    if fb.size:
        rw, rs, ram, rap, _ = eu_roe_plain(nl[:, fb], nr[:, fb], gm)
        waves[:, :, fb], speeds[:, fb], amdq[:, fb], apdq[:, fb] = rw, rs, ram, rap
    waves = np.stack([eu_from_normal(waves[p], ixy) for p in range(4)])
    return waves, speeds, eu_from_normal(amdq, ixy), eu_from_normal(apdq, ixy), fl


def eu_surrogate_rp(theta, gm=1.4, emulate=True):
    def rp(ixy, ql, qr):
        return eu_rp2(theta, ixy, ql, qr, gm, emulate)
    return rp
