"""Pins of the surrogate oracle (oracle/surrogate.py) against things other
than itself: torch's bfloat16 rounding, GELU and autograd, finite
differences, Adam's closed-form first step, the Roe identity, a least-squares
solver, and the plain C oracle's split step."""
import numpy as np
import pytest
import torch

import oracle as O
from oracle import surrogate as S
from paper_1308_1464_amd import inputs

G = 9.81


def small_net(seed=0, scale=1.0):
    th = S.init_params(inputs.rng(seed).random(S.NPARAMS))
    th[[bs for _, bs, _, _ in S.layer_slices()][0]] = 0.1  # non-zero biases too
    return th * scale


def torch_net(theta):
    mods = []
    for l, (W, b) in enumerate(S.unpack(theta)):
        lin = torch.nn.Linear(W.shape[1], W.shape[0], dtype=torch.float64)
        lin.weight.data = torch.tensor(W)
        lin.bias.data = torch.tensor(b)
        mods.append(lin)
        if l < S.NLAYERS - 1:
            mods.append(torch.nn.GELU(approximate="tanh"))
    return torch.nn.Sequential(*mods)


# ------------------------------------------------------------ rounding, GELU
def test_bf16_matches_torch_rounding():
    x = inputs.rng(1).normal(size=20000) * np.exp(inputs.rng(2).uniform(-20, 20, 20000))
    ties = np.array([1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -(1.0 + 2.0 ** -8), 2.0 ** -130])
    x = np.concatenate([x, ties])
    want = torch.tensor(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(S.bf16(x), want)
    assert S.bf16(1.0 + 2.0 ** -8) == 1.0            # tie to even
    assert S.bf16(1.0 + 3 * 2.0 ** -8) == 1.0 + 2.0 ** -6


def test_gelu_against_torch_and_identities():
    x = np.linspace(-12, 12, 4001)
    want = torch.nn.functional.gelu(torch.tensor(x), approximate="tanh").numpy()
    np.testing.assert_allclose(S.gelu(x), want, rtol=1e-14, atol=1e-15)
    # tanh form: gelu(x) - gelu(-x) = x exactly (up to rounding)
    np.testing.assert_allclose(S.gelu(x) - S.gelu(-x), x, rtol=0, atol=4e-15 * 12)
    assert S.gelu(0.0) == 0.0
    # derivative against central differences
    h = 1e-6
    fd = (S.gelu(x + h) - S.gelu(x - h)) / (2 * h)
    np.testing.assert_allclose(S.gelu_grad(x), fd, rtol=1e-7, atol=1e-8)
    assert abs(S.gelu_grad(0.0) - 0.5) < 1e-15


# ------------------------------------------------------------ network
def test_forward_matches_torch_fp64():
    th = small_net(3)
    X = inputs.rng(4).normal(size=(257, 6))
    out, _ = S.forward(th, X)
    want = torch_net(th)(torch.tensor(X)).detach().numpy()
    np.testing.assert_allclose(out, want, rtol=1e-12, atol=1e-13)


def test_param_layout_and_count():
    assert S.NPARAMS == 51464
    sl = S.layer_slices()
    assert sl[0][2:] == (128, 6) and sl[-1][2:] == (8, 128)
    th = np.arange(S.NPARAMS, dtype=float)
    np.testing.assert_array_equal(S.pack(S.unpack(th)), th)
    W0, b0 = S.unpack(th)[0]
    assert W0[1, 0] == 6 and b0[0] == 768     # row-major [out][in], bias after


def test_backward_against_finite_differences():
    th = small_net(5)
    r = inputs.rng(6)
    X = r.normal(size=(37, 6))
    Y = r.normal(size=(37, 8))
    mask = r.random(37) < 0.8
    L, gr = S.loss_and_grad(th, X, Y, mask)
    idx = np.concatenate([r.choice(S.NPARAMS, 60, replace=False),
                          [0, 5, 767, 768, 895, S.NPARAMS - 1, S.NPARAMS - 9]])
    h = 1e-6
    for i in idx:
        tp, tm = th.copy(), th.copy()
        tp[i] += h
        tm[i] -= h
        Lp, _ = S.loss(S.forward(tp, X)[0], Y, mask)
        Lm, _ = S.loss(S.forward(tm, X)[0], Y, mask)
        fd = (Lp - Lm) / (2 * h)
        assert abs(gr[i] - fd) <= 1e-6 * max(abs(fd), 1e-3), (i, gr[i], fd)


def test_backward_against_torch_autograd():
    th = small_net(7)
    r = inputs.rng(8)
    X = r.normal(size=(64, 6))
    Y = r.normal(size=(64, 8))
    mask = np.ones(64, bool)
    L, gr = S.loss_and_grad(th, X, Y, mask)
    net = torch_net(th)
    lt = ((net(torch.tensor(X)) - torch.tensor(Y)) ** 2).mean()
    lt.backward()
    tg = np.concatenate([np.concatenate([m.weight.grad.numpy().ravel(), m.bias.grad.numpy()])
                         for m in net if isinstance(m, torch.nn.Linear)])
    assert abs(L - lt.item()) < 1e-12 * abs(L)
    np.testing.assert_allclose(gr, tg, rtol=1e-10, atol=1e-14)


def test_emulated_network_within_bf16_bounds():
    th = small_net(9)
    X = inputs.rng(10).normal(size=(512, 6))
    o64, _ = S.forward(th, X)
    oem, (ins, zs) = S.forward(th, X, emulate=True)
    rel = np.linalg.norm(oem - o64) / np.linalg.norm(o64)
    assert 1e-4 < rel < 2e-2          # the emulation is active, and bounded
    for a in ins:                      # every layer input is a bfloat16 value
        np.testing.assert_array_equal(S.bf16(a), a)
    for z in zs:
        np.testing.assert_array_equal(S.f32(z), z)
    # emulated gradient close to the exact one
    Y = inputs.rng(11).normal(size=(512, 8))
    m = np.ones(512, bool)
    _, g64 = S.loss_and_grad(th, X, Y, m)
    _, gem = S.loss_and_grad(th, X, Y, m, emulate=True)
    assert np.linalg.norm(gem - g64) / np.linalg.norm(g64) < 2e-2


def bf16_neighbour(q, upward):
    """the next bfloat16 value above (upward) or below q, q a bfloat16 value"""
    b = np.ascontiguousarray(np.asarray(q, dtype=np.float64).astype(np.float32)).view(np.uint32).astype(np.int64)
    neg = b >= 0x80000000
    mag_up = upward != neg                # the magnitude grows
    zero = (b & 0x7FFFFFFF) == 0
    step = np.where(mag_up, 0x10000, -0x10000)
    nb = np.where(zero, np.where(upward, 0x00010000, 0x80010000), b + step)
    return nb.astype(np.uint32).view(np.float32).astype(np.float64)


def perturbed_forward(theta, X, rel, in_rel, in_abs, rng, push):
    """The emulated network, with every value moved by at most the error the
    bound allows before it is rounded to BF16 (push: each moved the whole
    allowance toward its nearest rounding midpoint, so that every operand
    that can round the other way does; else by a uniform random fraction in
    either direction) and each final sum by up to rel times its absolute
    sum.  Written apart from the bound: plain forward pass, explicit
    perturbation."""
    a = np.asarray(X, dtype=np.float64)
    layers = S.unpack(theta)
    d = in_rel * np.abs(a) + in_abs
    for l, (W, b) in enumerate(layers):
        q0 = S.bf16(a)
        if push:
            # the BF16 neighbour of q0 on the side of a, by stepping the bit
            # pattern (bfloat16 is the upper half of an FP32 word)
            other = bf16_neighbour(q0, a >= q0)
            mid = 0.5 * (q0 + other)
            a = a + np.sign(mid - a) * d
        else:
            a = a + d * rng.uniform(-1.0, 1.0, a.shape)
        q = S.bf16(a)
        Wq = S.bf16(W)
        s = np.abs(q) @ np.abs(Wq).T + np.abs(S.f32(b))
        z = q @ Wq.T + S.f32(b)
        if l < len(layers) - 1:
            z = S.f32(z)
            a = S.gelu(z)
            d = rel * (1.2 * s + np.abs(a))
        else:
            a = z + rel * s * rng.uniform(-1.0, 1.0, z.shape)
    return a


@pytest.mark.parametrize("model", ["sw", "euler"])
def test_rounding_spread_covers_other_roundings(model):
    """rounding_spread measures what it claims: evaluations that move every
    value by an FP32-sized error before it is rounded (toward the nearest
    rounding midpoint, the worst case, or at random) stay within 6 sigma
    plus the floor on every row and output (seen: at most about 3.2 sigma);
    and sigma is not vacuous (its median is below 1 % of the outputs).  The
    GPU network tests use this 6-sigma bound."""
    rng = inputs.rng(91)
    if model == "sw":
        th = small_net(3)
        X = np.concatenate([rng.uniform(-1, 1, (3000, 2)), rng.uniform(0, 2, (3000, 1)),
                            rng.normal(size=(3000, 3))], axis=1)
        X[:, 3:] /= np.linalg.norm(X[:, 3:], axis=1, keepdims=True)
    else:
        th = S.init_params(inputs.rng(4).random(S.nparams(S.EU_WIDTHS)), S.EU_WIDTHS)
        X = rng.normal(size=(3000, 7))
    X = S.f32(X)
    out, _ = S.forward(th, X, emulate=True)
    for inp, in_rel in ((False, 0.0), (True, 2.0 ** -17)):
        sig, floor = S.rounding_spread(th, X, inputs=inp)
        assert sig.shape == out.shape and (sig > 0).all() and (floor > 0).all()
        worst = 0.0
        for push in (True, False, True, False):
            alt = perturbed_forward(th, X, 2.0 ** -17, in_rel, 0.0, rng, push)
            worst = max(worst, (np.abs(alt - out) / (sig + floor)).max())
        assert worst <= 6.0, (inp, worst)
        assert np.median(sig / (np.abs(out) + 1e-3)) < 1e-2


def test_bf16_spacing_hand_cases():
    u, d = S.bf16_spacing(np.array([1.0, 1.0, 1.0, -2.0]),
                          np.array([1.0 + 2.0 ** -9, 1.0 - 2.0 ** -10, 1.0, -2.0 - 2.0 ** -8]))
    np.testing.assert_array_equal(u, [2.0 ** -7, 2.0 ** -8, 2.0 ** -7, 2.0 ** -6])
    np.testing.assert_array_equal(d, [2.0 ** -8 - 2.0 ** -9, 2.0 ** -9 - 2.0 ** -10, 2.0 ** -9,
                                      2.0 ** -7 - 2.0 ** -8])


def test_adam_first_step_closed_form_and_torch():
    r = inputs.rng(12)
    th = r.normal(size=50)
    g = r.normal(size=50)
    t1, m1, v1 = S.adam(th, g, np.zeros(50), np.zeros(50), 1, 1e-3)
    # step 1: m_hat = g, v_hat = g^2, so the move is lr g / (|g| + eps)
    np.testing.assert_allclose(t1, th - 1e-3 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    # several steps against torch.optim.Adam
    p = torch.nn.Parameter(torch.tensor(th))
    opt = torch.optim.Adam([p], lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    x, m, v = th.copy(), np.zeros(50), np.zeros(50)
    for t in range(1, 8):
        gt = r.normal(size=50)
        x, m, v = S.adam(x, gt, m, v, t, 1e-2)
        p.grad = torch.tensor(gt)
        opt.step()
    np.testing.assert_allclose(x, p.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_init_params_ranges():
    th = S.init_params(inputs.rng(13).random(S.NPARAMS))
    for ws, bs, no, ni in S.layer_slices():
        a = np.sqrt(6.0 / (ni + no))
        assert np.abs(th[ws]).max() <= a and np.abs(th[ws]).max() > 0.9 * a
        assert not th[bs].any()


# ------------------------------------------------------------ edges
def test_states_from_uniforms_ranges():
    U = np.array([[0.0, 1.0 - 1e-16, 0.5]] * 6)
    ql, qr = S.states_from_uniforms(U)
    np.testing.assert_allclose(ql[0], [1e-3, 10.0, np.sqrt(1e-3 * 10.0)], rtol=1e-12)
    np.testing.assert_allclose(ql[1] / ql[0], [-5.0, 5.0, 0.0], atol=1e-12)


def test_features_scale_invariance_and_zero_jump():
    ql, qr = inputs.sw_random_states(500, seed=14, hlo=0.5, hhi=2.0, ulim=1.0)
    X, h0, c0, m = S.features(ql, qr, G)
    lam = 3.7
    sc = np.array([lam, lam ** 1.5, lam ** 1.5])[:, None]
    X2, h02, _, m2 = S.features(ql * sc, qr * sc, G)
    np.testing.assert_allclose(X2, X, rtol=1e-12, atol=1e-13)
    np.testing.assert_allclose(np.linalg.norm(X[:, 3:], axis=1), 1.0, rtol=1e-14)
    Xz, _, _, mz = S.features(ql, ql, G)
    assert not mz.any() and not Xz[:, 2:].any()
    # a hand-computed case: hL = 1, hR = 3, uL = 1, uR = -1, v = 0
    Xh, h0h, c0h, mh = S.features(np.array([[1.0], [1.0], [0.0]]),
                                  np.array([[3.0], [-3.0], [0.0]]), G)
    c = np.sqrt(2 * G)
    np.testing.assert_allclose(Xh[0, :3], [0.0, 0.0, np.hypot(1.0, 4 / (2 * c))], rtol=1e-14)


def test_flags_hand_built():
    def st(h, u, v):
        return np.array([[h], [h * u], [h * v]], dtype=float)
    ok = S.flags(st(1.0, 0.1, 0.2), st(1.2, -0.3, 0.0), G)
    assert ok[0] == 0
    assert S.flags(st(5e-4, 0, 0), st(1, 0, 0), G)[0] & S.FLAG_OOD
    assert S.flags(st(11.0, 0, 0), st(1, 0, 0), G)[0] & S.FLAG_OOD
    assert S.flags(st(9.0, 0, 5.5), st(9, 0, 0), G)[0] & S.FLAG_OOD
    assert S.flags(st(5e-3, 0, 0), st(1, 0, 0), G)[0] & S.FLAG_DRY
    assert not S.flags(st(2e-2, 0, 0), st(1, 0, 0), G)[0] & S.FLAG_DRY
    # transonic: u - c changes sign between the sides
    c = np.sqrt(G)
    assert S.flags(st(1.0, 0.9 * c, 0), st(1.0, 1.1 * c, 0), G)[0] & S.FLAG_NONSUB
    assert S.flags(st(1.0, -1.2 * c, 0), st(1.0, -1.1 * c, 0), G)[0] & S.FLAG_NONSUB
    assert not S.flags(st(1.0, 0.99 * c, 0), st(1.0, -0.99 * c, 0), G)[0]


def test_labels_satisfy_roe_identity():
    U = inputs.rng(15).random((6, 40000))
    ql, qr = S.states_from_uniforms(U)
    Y, X, keep = S.labels(ql, qr, G)
    assert 0.05 < keep.mean() < 0.2
    k = keep
    _, h0, c0, m = S.features(ql[:, k], qr[:, k], G)
    s, W = S.decode(Y[k], h0, c0, m)
    df = S.sw_flux(qr[:, k], G) - S.sw_flux(ql[:, k], G)
    res = s[0] * W[0] + s[1] * W[1] - df
    scale = np.abs(df).max(axis=0) + np.abs(s[0] * W[0]).max(axis=0)
    assert (np.abs(res).max(axis=0) / scale).max() < 1e-11
    assert (s[0] < 0).all() and (s[1] > 0).all()
    assert np.abs(Y[k]).max() < 10 and not Y[~k].any()


def test_projection_is_least_norm():
    r = inputs.rng(16)
    n = 300
    s = r.normal(size=(2, n))
    W = r.normal(size=(2, 3, n))
    df = r.normal(size=(3, n))
    Wp, ok = S.project(s, W, df)
    assert ok.all()
    np.testing.assert_allclose(s[0] * Wp[0] + s[1] * Wp[1], df, rtol=1e-12, atol=1e-12)
    for i in range(0, n, 37):   # least-norm correction by a library solver
        A = np.hstack([s[0, i] * np.eye(3), s[1, i] * np.eye(3)])
        rhs = df[:, i] - A @ np.concatenate([W[0, :, i], W[1, :, i]])
        d = np.linalg.lstsq(A, rhs, rcond=None)[0]
        np.testing.assert_allclose(np.concatenate([Wp[0, :, i], Wp[1, :, i]]),
                                   np.concatenate([W[0, :, i], W[1, :, i]]) + d, rtol=1e-12,
                                   atol=1e-12)
    _, ok0 = S.project(np.zeros((2, 1)), W[:, :, :1], df[:, :1])
    assert not ok0.any()


@pytest.mark.parametrize("ixy", [1, 2])
def test_rp2_exact_outputs_reproduce_roe(ixy):
    """With the exact targets in place of the network, decoding, projection
    and the fluctuation split give Roe's fluctuations back."""
    ql, qr = inputs.sw_random_states(20000, seed=17, hlo=0.05, hhi=4.0, ulim=1.5)
    nl, nr = S.to_normal(ql, ixy), S.to_normal(qr, ixy)
    Y, _, keep = S.labels(nl, nr, G)
    assert keep.mean() > 0.5
    w, s, am, ap, fl = S.rp2(None, ixy, ql, qr, G, outputs=Y)
    P = O.params(g=G)
    rw, rs, ram, rap, _ = O.rp2(O.SW_ROE, P, ixy, ql, qr)
    # the plain solver the rule falls back to: Roe, or HLLE where Roe's
    # middle depth hL + alpha_1 is not positive
    hll = ~(nl[0] + S.to_normal(rw[0], ixy)[0] > 0.0)
    assert hll.any() and not (hll & keep).any()
    hw, hs, ham, hap, _ = O.rp2(O.SW_HLLE, P, ixy, ql, qr)
    rw[:, :, hll], rs[:, hll], ram[:, hll], rap[:, hll] = \
        hw[:, :, hll], hs[:, hll], ham[:, hll], hap[:, hll]
    scale = np.abs(ram).max(axis=0) + np.abs(rap).max(axis=0) + 1e-300
    err = (np.abs(am - ram).max(axis=0) + np.abs(ap - rap).max(axis=0)) / scale
    assert err.max() < 1e-11
    # flagged and degenerate edges are the plain solver's own output
    fb = fl != 0
    assert fb.any() and (fl[keep] == 0).all()
    np.testing.assert_array_equal(w[:, :, fb], rw[:, :, fb])
    np.testing.assert_array_equal(s[:, fb], rs[:, fb])


@pytest.mark.parametrize("ixy", [1, 2])
def test_rp2_conservation_any_network(ixy):
    th = small_net(18, scale=0.5)
    ql, qr = inputs.sw_random_states(3000, seed=19, hlo=0.02, hhi=8.0, ulim=3.0)
    w, s, am, ap, fl = S.rp2(th, ixy, ql, qr, G)
    nl, nr = S.to_normal(ql, ixy), S.to_normal(qr, ixy)
    df = S.from_normal(S.sw_flux(nr, G) - S.sw_flux(nl, G), ixy)
    net = fl == 0
    assert net.mean() > 0.1 and (~net).any()
    scale = np.abs(df).max(axis=0) + np.abs(am).max(axis=0) + np.abs(ap).max(axis=0)
    assert ((np.abs(am + ap - df).max(axis=0) / scale)[net]).max() < 1e-12
    assert not w[1][:, net].any() and not s[1][net].any()
    # fallback edges: Roe where its middle depth is positive, else HLLE
    rw, rs, ram, rap, _ = O.rp2(O.SW_ROE, O.params(g=G), ixy, ql[:, ~net], qr[:, ~net])
    good = S.to_normal(ql[:, ~net], ixy)[0] + rw[0][0] > 0
    np.testing.assert_array_equal(am[:, ~net][:, good], ram[:, good])


# ------------------------------------------------------------ split step
def test_phi_matches_c_oracle():
    th = np.concatenate([np.linspace(-3, 5, 801), [0.0, 0.5, 1.0, 2.0, 3.0, -1e-300]])
    for lim in (O.LIM_NONE, O.LIM_MINMOD, O.LIM_SUPERBEE, O.LIM_VANLEER, O.LIM_MC):
        want = np.array([O.phi(lim, t) for t in th])
        np.testing.assert_array_equal(S.phi(lim, th), want)


@pytest.mark.parametrize("bc", [O.BC_PERIODIC, O.BC_EXTRAP])
@pytest.mark.parametrize("lim", [O.LIM_MC, O.LIM_MINMOD, O.LIM_SUPERBEE, O.LIM_VANLEER,
                                 O.LIM_NONE, O.LIM_FIRST_ORDER])
def test_numpy_sweep_equals_c_step(bc, lim):
    q = inputs.sw_dam_break(37, seed=20, ny=29)
    q[1] = 0.1 * inputs.random_field((29, 37), seed=21)
    q[2] = 0.1 * inputs.random_field((29, 37), seed=22)
    P = O.params(g=G)
    dx, dy = 1 / 37, 1 / 29
    sm0, _ = O.max_speed(O.SW_ROE, P, q, dx, dy, bc)
    dt = 0.8 / sm0
    want, smw, _ = O.step2d(O.SW_ROE, P, q, dx, dy, dt, lim, bc)
    got, smg, nf = S.step2d(S.plain_rp(G), q, dx, dy, dt, lim, bc)
    np.testing.assert_array_equal(got, want)
    assert smg == smw and nf == 0


def test_surrogate_step_conserves_periodic():
    th = small_net(23, scale=0.3)
    q = inputs.sw_dam_break(24, seed=24, ny=20)
    dx, dy = 1 / 24, 1 / 20
    sm0, _ = O.max_speed(O.SW_ROE, O.params(g=G), q, dx, dy, O.BC_PERIODIC)
    qn, sm, nf = S.step2d(S.surrogate_rp(th, G), q, dx, dy, 0.5 / sm0, O.LIM_MC,
                          O.BC_PERIODIC)
    for m in range(3):
        tot = np.abs(q[m]).sum() + 1.0
        assert abs(qn[m].sum() - q[m].sum()) < 1e-13 * tot
    assert np.isfinite(qn).all() and sm > 0


# ------------------------------------------------------------ Euler model
GM = 1.4


def eu_states(n, seed, rlo=0.2, rhi=3.0, ulim=0.6):
    r = inputs.rng(seed)
    out = []
    for _ in range(2):
        rho = r.uniform(rlo, rhi, n)
        u = r.uniform(-ulim, ulim, n)
        v = r.uniform(-ulim, ulim, n)
        p = r.uniform(rlo, rhi, n)
        out.append(np.stack([rho, rho * u, rho * v, p / (GM - 1) + 0.5 * rho * (u * u + v * v)]))
    return out


def test_eu_param_count_and_ranges():
    assert S.EU_NPARAMS == 7 * 128 + 128 + 3 * (128 * 128 + 128) + 128 * 15 + 15
    U = np.array([[0.0, 1.0 - 1e-16, 0.5]] * 8)
    ql, _ = S.eu_states_from_uniforms(U, GM)
    np.testing.assert_allclose(ql[0], [0.05, 10.0, np.sqrt(0.5)], rtol=1e-12)
    np.testing.assert_allclose(ql[1] / ql[0], [-2.0, 2.0, 0.0], atol=1e-12)
    np.testing.assert_allclose(S.eu_pressure(ql, GM), [0.05, 10.0, np.sqrt(0.5)], rtol=1e-12)


def test_eu_features_scale_invariance():
    ql, qr = eu_states(500, 30)
    X, _, _, _ = S.eu_features(ql, qr, GM)
    a, b = 2.7, 0.6      # rho -> a rho, u -> b u, p -> a b^2 p
    sc = np.array([a, a * b, a * b, a * b * b])[:, None]
    X2, _, _, _ = S.eu_features(ql * sc, qr * sc, GM)
    np.testing.assert_allclose(X2, X, rtol=1e-11, atol=1e-12)
    np.testing.assert_allclose(np.linalg.norm(X[:, 3:], axis=1), 1.0, rtol=1e-14)


def test_eu_flags_hand_built():
    def st(rho, u, v, p):
        return np.array([[rho], [rho * u], [rho * v], [p / (GM - 1) + 0.5 * rho * (u * u + v * v)]])
    assert S.eu_flags(st(1, 0.1, 0.2, 1), st(0.5, -0.2, 0, 0.4), GM)[0] == 0
    assert S.eu_flags(st(0.04, 0, 0, 1), st(1, 0, 0, 1), GM)[0] & S.FLAG_OOD
    assert S.eu_flags(st(1, 0, 0, 11.0), st(1, 0, 0, 1), GM)[0] & S.FLAG_OOD
    assert S.eu_flags(st(1, 0, 0, 0.04), st(1, 0, 0, 1), GM)[0] & S.FLAG_OOD
    assert S.eu_flags(st(1, 0, 2.1, 9.0), st(1, 0, 0, 9.0), GM)[0] & S.FLAG_OOD
    c = np.sqrt(GM)           # rho = p = 1
    assert S.eu_flags(st(1, 1.01 * c, 0, 1), st(1, 0.5, 0, 1), GM)[0] & S.FLAG_NONSUB
    assert not S.eu_flags(st(1, 0.99 * c, 0, 1), st(1, -0.99 * c, 0, 1), GM)[0]


def test_eu_labels_satisfy_roe_identity():
    U = inputs.rng(31).random((8, 40000))
    ql, qr = S.eu_states_from_uniforms(U, GM)
    Y, X, keep = S.eu_labels(ql, qr, GM)
    assert 0.15 < keep.mean() < 0.4
    k = keep
    _, Sc, c0, m = S.eu_features(ql[:, k], qr[:, k], GM)
    s, W = S.eu_decode(Y[k], Sc, c0, m)
    df = S.eu_flux(qr[:, k], GM) - S.eu_flux(ql[:, k], GM)
    res = s[0] * W[0] + s[1] * W[1] + s[2] * W[2] - df
    scale = np.abs(df).max(axis=0) + np.abs(s[0] * W[0]).max(axis=0) + np.abs(s[2] * W[2]).max(axis=0)
    assert (np.abs(res).max(axis=0) / scale).max() < 1e-11
    assert (s[0] < 0).all() and (s[2] > 0).all() and (s[0] < s[1]).all() and (s[1] < s[2]).all()
    assert np.abs(Y[k]).max() < 20 and not Y[~k].any()


@pytest.mark.parametrize("ixy", [1, 2])
def test_eu_rp2_exact_outputs_reproduce_roe(ixy):
    ql, qr = eu_states(20000, 32 + ixy)
    nl, nr = S.eu_to_normal(ql, ixy), S.eu_to_normal(qr, ixy)
    Y, _, keep = S.eu_labels(nl, nr, GM)
    assert keep.mean() > 0.5
    w, s, am, ap, fl = S.eu_rp2(None, ixy, ql, qr, GM, outputs=Y)
    rw, rs, ram, rap, _ = O.rp2(O.EULER_ROE, O.params(gamma=GM), ixy, ql, qr)
    scale = np.abs(ram).max(axis=0) + np.abs(rap).max(axis=0) + 1e-300
    err = (np.abs(am - ram).max(axis=0) + np.abs(ap - rap).max(axis=0)) / scale
    assert err.max() < 1e-11
    fb = fl != 0
    assert fb.any() and (fl[keep] == 0).all()
    np.testing.assert_array_equal(w[:, :, fb], rw[:, :, fb])
    np.testing.assert_array_equal(s[:, fb], rs[:, fb])


@pytest.mark.parametrize("ixy", [1, 2])
def test_eu_rp2_conservation_any_network(ixy):
    th = S.init_params(inputs.rng(34).random(S.EU_NPARAMS), S.EU_WIDTHS) * 0.5
    ql, qr = eu_states(3000, 35, rlo=0.06, rhi=8.0, ulim=1.5)
    w, s, am, ap, fl = S.eu_rp2(th, ixy, ql, qr, GM)
    nl, nr = S.eu_to_normal(ql, ixy), S.eu_to_normal(qr, ixy)
    df = S.eu_from_normal(S.eu_flux(nr, GM) - S.eu_flux(nl, GM), ixy)
    net = fl == 0
    assert net.mean() > 0.2 and (~net).any()
    scale = np.abs(df).max(axis=0) + np.abs(am).max(axis=0) + np.abs(ap).max(axis=0)
    assert ((np.abs(am + ap - df).max(axis=0) / scale)[net]).max() < 1e-12
    assert not w[2][:, net].any() and not s[2][net].any()


@pytest.mark.parametrize("bc", [O.BC_PERIODIC, O.BC_EXTRAP])
def test_numpy_sweep_equals_c_step_euler(bc):
    q, _ = inputs.euler_quadrants(33, seed=36, ny=27)
    P = O.params(gamma=GM)
    dx, dy = 1 / 33, 1 / 27
    sm0, _ = O.max_speed(O.EULER_ROE, P, q, dx, dy, bc)
    dt = 0.7 / sm0
    want, smw, _ = O.step2d(O.EULER_ROE, P, q, dx, dy, dt, O.LIM_MC, bc)
    got, smg, _ = S.step2d(S.plain_rp(9.81, O.EULER_ROE), q, dx, dy, dt, O.LIM_MC, bc)
    np.testing.assert_array_equal(got, want)
    assert smg == smw
