"""GPU tests of the learned Euler edge solver (mc_sur_* with
MC_EULER_SURROGATE) against the surrogate oracle (oracle/surrogate.py, the
eu_* functions) and the plain FP64 oracle.

Tolerances (the arithmetic is the shallow-water surrogate's, see
test_gpu_surrogate.py):
  pair generation   FP64 on both sides, stored as FP32: within 4 FP32 ulps
                    plus 1e-12 of the row's largest label (the Euler labels
                    W2 + W3 can cancel, where the FP64 order of operations
                    shows at that level); keep decisions identical
  network forward   every output within 6 sigma (plus the FP32 floor) of
                    the oracle's BF16/FP32 emulation (tests/sur_bounds.py);
                    in Frobenius norm, within the root expected sum of squares
                    of BF16 rounding flips (tests/sur_bounds.py flip_rms);
                    cosine >= 0.999 to FP64
  gradient          5e-4 and 1e-2 relative per layer
  edge solves       fallback decisions identical (FP32 product-only flags on
                    both sides); A-dQ + A+dQ = f(qR) - f(qL) to FP32
                    round-off; network edges: each fluctuation component
                    within the bound the network's spread carries through
                    the oracle's decoding and projection (features in FP32
                    here, FP64 in the oracle)
  step              the oracle's sweep with the oracle's network (emulated),
                    relative L1 1e-4 after 3 steps
"""
import numpy as np
import pytest

import sur_bounds as sb
from paper_1308_1464_amd import inputs
from paper_1308_1464_amd import manyclaw as mc

pytestmark = pytest.mark.gpu

GM = 1.4
MODEL = mc.MC_EULER_SURROGATE


def _t():
    import torch
    return torch


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def S():
    from oracle import surrogate as S_
    return S_


@pytest.fixture(scope="module")
def O():
    import oracle as O_
    return O_


def dev(a, dtype=None):
    t = _t()
    x = t.from_numpy(np.ascontiguousarray(a)).to("cuda")
    return x if dtype is None else x.to(dtype)


def host(x):
    _t().cuda.synchronize()
    return x.detach().cpu().numpy()


def net_with(theta):
    sur = mc.mc_sur_create(8192, MODEL)
    mc.mc_sur_set_params(sur, dev(theta.astype(np.float32)))
    _t().cuda.synchronize()
    return sur


def random_theta(S, seed, bias=0.05):
    th = S.init_params(inputs.param_uniforms(S.EU_NPARAMS, seed), S.EU_WIDTHS)
    r = inputs.rng(seed + 1)
    for _, bs, _, _ in S.layer_slices(S.EU_WIDTHS):
        th[bs] = bias * r.normal(size=th[bs].shape)
    return th


def gen_pairs(n, seed):
    t = _t()
    U = inputs.euler_surrogate_uniforms(n, seed)
    sur = mc.mc_sur_create(64, MODEL)
    X = t.empty((n, 8), dtype=t.float32, device="cuda")
    Y = t.empty((n, 16), dtype=t.float32, device="cuda")
    keep = t.empty(n, dtype=t.int32, device="cuda")
    mc.mc_sur_gen(sur, mc.params(gamma=GM), n, dev(U), X, Y, keep)
    out = U, host(X), host(Y), host(keep)
    mc.mc_sur_destroy(sur)
    return out


def test_dims(S):
    say("case: mc_sur_dims")
    assert mc.mc_sur_dims(MODEL) == (S.EU_NPARAMS, 7, 15, 16) == (
        mc.MC_SUR_EU_NPARAMS, mc.MC_SUR_EU_NIN, mc.MC_SUR_EU_NOUT, 16)
    assert mc.mc_sur_dims(mc.MC_SW_SURROGATE) == (S.NPARAMS, 6, 8, 8)
    with pytest.raises(mc.ManyclawError):
        mc.mc_sur_dims(mc.MC_EULER_ROE)


# ------------------------------------------------------------ data
def test_gen_matches_oracle(S):
    n = 200003
    say("case: Euler mc_sur_gen n =", n)
    U, X, Y, keep = gen_pairs(n, 61)
    ql, qr = S.eu_states_from_uniforms(U, GM)
    Yo, Xo, ko = S.eu_labels(ql, qr, GM)
    mism = np.count_nonzero(keep.astype(bool) != ko)
    say("keep fraction", ko.mean(), "mismatches", mism)
    assert mism == 0
    ulp = np.spacing(np.abs(Xo).astype(np.float32)).astype(np.float64)
    assert (np.abs(X[:, :7] - Xo) <= 2 * ulp + 1e-30).all()
    assert not X[:, 7:].any()
    k = ko
    uy = np.spacing(np.abs(Yo[k]).astype(np.float32)).astype(np.float64)
    rowmax = np.abs(Yo[k]).max(axis=1, keepdims=True)
    err = np.abs(Y[k, :15] - Yo[k])
    say("label error in FP32 ulps: max", (err / (uy + 1e-30)).max())
    assert (err <= 4 * uy + 1e-12 * rowmax).all()
    assert not Y[~k].any() and not Y[:, 15].any()


def test_compact_rows_of_16():
    t = _t()
    n = 30001
    say("case: Euler mc_sur_compact n =", n)
    r = inputs.rng(62)
    X = r.normal(size=(n, 8)).astype(np.float32)
    Y = r.normal(size=(n, 16)).astype(np.float32)
    keep = (r.random(n) < 0.4).astype(np.int32)
    sur = mc.mc_sur_create(64, MODEL)
    Xc = t.empty((n, 8), dtype=t.float32, device="cuda")
    Yc = t.empty((n, 16), dtype=t.float32, device="cuda")
    nk = mc.mc_sur_compact(sur, n, dev(X), dev(Y), dev(keep), Xc, Yc)
    assert nk == keep.sum()
    np.testing.assert_array_equal(host(Xc)[:nk], X[keep == 1])
    np.testing.assert_array_equal(host(Yc)[:nk], Y[keep == 1])
    mc.mc_sur_destroy(sur)


# ------------------------------------------------------------ network
def test_init_params_matches_oracle(S):
    t = _t()
    say("case: Euler mc_sur_init_params")
    sur = mc.mc_sur_create(64, MODEL)
    U = inputs.param_uniforms(S.EU_NPARAMS, 63)
    mc.mc_sur_init_params(sur, dev(U))
    p = t.empty(S.EU_NPARAMS, dtype=t.float32, device="cuda")
    mc.mc_sur_get_params(sur, p)
    np.testing.assert_allclose(host(p), S.init_params(U, S.EU_WIDTHS).astype(np.float32),
                               rtol=1e-6, atol=1e-7)
    mc.mc_sur_destroy(sur)


def test_forward_matches_oracle(S):
    t = _t()
    n = 70001
    say("case: Euler mc_sur_forward n =", n)
    _, X, _, _ = gen_pairs(n, 64)
    th = random_theta(S, 65)
    sur = net_with(th)
    out = t.empty((n, 16), dtype=t.float32, device="cuda")
    mc.mc_sur_forward(sur, n, dev(X), out)
    o = host(out)
    assert not o[:, 15].any()
    o = o[:, :15]
    th32 = th.astype(np.float32).astype(np.float64)
    X7 = X[:, :7].astype(np.float64)
    oe, _ = S.forward(th32, X7, emulate=True)
    o64, _ = S.forward(th32, X7)
    re = np.linalg.norm(o - oe) / np.linalg.norm(oe)
    cos = (o * o64).sum() / (np.linalg.norm(o) * np.linalg.norm(o64))
    bnd = sb.network_bound(S, th32, X7)
    ratio = np.abs(o - oe) / bnd
    say(f"forward: |gpu - emulated| / bound max {ratio.max():.3f}; rel err vs emulated {re:.2e}, "
        f"cosine vs fp64 {cos:.8f}")
    assert ratio.max() <= 1.0
    # aggregate: within the expected flip-model spread of the whole array
    rb = sb.flip_rms(S, th32, X7) / np.linalg.norm(oe)
    say(f"relative Frobenius error {re:.2e} against the expected flip spread {rb:.2e}")
    assert re <= rb and cos >= 0.999
    mc.mc_sur_destroy(sur)


def test_loss_grad_matches_oracle(S):
    t = _t()
    n = 3000
    say("case: Euler mc_sur_loss_grad n =", n)
    _, X, Y, keep = gen_pairs(4 * n, 66)
    k = np.nonzero(keep)[0][:n]
    n = len(k)
    X, Y = X[k], Y[k]
    th = random_theta(S, 67)
    sur = net_with(th)
    grad = t.empty(S.EU_NPARAMS, dtype=t.float32, device="cuda")
    loss = t.empty(1, dtype=t.float32, device="cuda")
    mc.mc_sur_loss_grad(sur, n, dev(X), dev(Y), grad, loss)
    g = host(grad).astype(np.float64)
    L = float(host(loss)[0])
    th32 = th.astype(np.float32).astype(np.float64)
    m = np.ones(n, bool)
    X7, Y15 = X[:, :7].astype(np.float64), Y[:, :15].astype(np.float64)
    Le, ge = S.loss_and_grad(th32, X7, Y15, m, emulate=True)
    L64, g64 = S.loss_and_grad(th32, X7, Y15, m)
    say("loss gpu", L, "emulated", Le, "fp64", L64)
    assert abs(L - Le) <= 1e-4 * Le
    for l, (ws, bs, no, ni) in enumerate(S.layer_slices(S.EU_WIDTHS)):
        for name, sl in (("W", ws), ("b", bs)):
            re = np.linalg.norm(g[sl] - ge[sl]) / np.linalg.norm(ge[sl])
            r64 = np.linalg.norm(g[sl] - g64[sl]) / np.linalg.norm(g64[sl])
            cos = (g[sl] * g64[sl]).sum() / (np.linalg.norm(g[sl]) * np.linalg.norm(g64[sl]))
            say(f"layer {l} {name}: rel err vs emulated {re:.2e}, vs fp64 {r64:.2e}, cosine vs fp64 {cos:.7f}")
            # the emulation rounds the same BF16 operands; the device differs
            # from it only by FP32 summation order and the BF16 roundings that
            # order flips (seen: at most 3e-5)
            assert re < 1e-4 and r64 < 1e-2 and cos >= 0.999
    mc.mc_sur_destroy(sur)


def test_train_reduces_loss():
    from paper_1308_1464_amd import surrogate as sg
    say("case: short Euler training run")
    sur, info = sg.train(seed=70, n_pairs=1 << 18, epochs=3, batch=2048, n_val=1 << 16, model=MODEL)
    say("losses", info["train_loss"], "val", info["val_loss"], "kept", info["n_kept"],
        "seconds", info["train_seconds"])
    L = info["train_loss"]
    assert L[-1] < 0.5 * L[0] and np.isfinite(info["val_loss"])
    mc.mc_sur_destroy(sur)


# ------------------------------------------------------------ edge solves
def edge_states(n, seed):
    """training-box pairs, near-equal pairs and pairs that must fall back
    (supersonic, outside the box), rounded to FP32"""
    r = inputs.rng(seed)
    a, b = inputs.euler_random_states(n, seed=seed)
    rho = 0.5 + r.random(n)
    u, v = 0.2 * r.normal(size=n), 0.2 * r.normal(size=n)
    p = 0.5 + r.random(n)
    near_l = np.stack([rho, rho * u, rho * v, p / (GM - 1.0) + 0.5 * rho * (u * u + v * v)])
    near_r = near_l * (1.0 + 1e-3 * r.normal(size=(4, n)))
    far = near_l[:, : n // 10].copy()
    far[0] *= 40.0                                    # rho outside the box
    ql = np.concatenate([a, near_l, far], axis=1)
    qr = np.concatenate([b, near_r, near_r[:, : n // 10]], axis=1)
    return ql.astype(np.float32).astype(np.float64), qr.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("ixy", [1, 2])
def test_rp2_matches_oracle(S, ixy):
    t = _t()
    ql, qr = edge_states(30000, 71 + ixy)
    n = ql.shape[1]
    say("case: Euler surrogate mc_rp2 ixy =", ixy, "n =", n)
    th = random_theta(S, 73)
    sur = net_with(th)
    ctx = mc.mc_ctx_create(MODEL, mc.MC_F32, mc.params(gamma=GM), 8, 8, 0.125, 0.125)
    mc.mc_ctx_set_surrogate(ctx, sur)
    w = t.empty((4, 4, n), dtype=t.float32, device="cuda")
    s = t.empty((4, n), dtype=t.float32, device="cuda")
    am = t.empty((4, n), dtype=t.float32, device="cuda")
    ap = t.empty((4, n), dtype=t.float32, device="cuda")
    mc.mc_sur_edge_stats(ctx)
    mc.mc_rp2(ctx, ixy, n, dev(ql.astype(np.float32)), dev(qr.astype(np.float32)), None, w, s, am, ap)
    W, Sp, AM, AP = host(w), host(s), host(am), host(ap)
    ne, nfb = mc.mc_sur_edge_stats(ctx)
    th32 = th.astype(np.float32).astype(np.float64)
    wo, so, amo, apo, flo = S.eu_rp2(th32, ixy, ql, qr, GM, emulate=True)
    say("fallback edges gpu", nfb, "oracle", np.count_nonzero(flo), "of", n)
    assert ne == n and nfb == np.count_nonzero(flo)
    nl, nr = S.eu_to_normal(ql, ixy), S.eu_to_normal(qr, ixy)
    fl_, fr_ = S.eu_flux(nl, GM), S.eu_flux(nr, GM)
    df = S.eu_from_normal(fr_ - fl_, ixy)
    net = flo == 0
    fs = S.eu_from_normal(np.abs(fr_) + np.abs(fl_), ixy)
    cons = (np.abs(AM + AP - df) / (fs.max(axis=0) + 1e-30))[:, net]
    say("conservation residual / |f|: max", cons.max())
    assert cons.max() < 2e-5
    bam, bap = sb.fluct_bound(S, th32, ixy, ql, qr, GM, euler=True)
    sb.check_fluct(say, AM, AP, amo, apo, bam, bap, fs, net)
    scale = np.abs(amo).max(axis=0) + np.abs(apo).max(axis=0) + 1e-30
    err = (np.abs(AM - amo).max(axis=0) + np.abs(AP - apo).max(axis=0)) / scale
    # fallback edges: the plain FP32 Euler solver of the library, to
    # round-off (for y-normal edges the two momenta enter |rho u|^2 in the
    # other order, a few ulps that cancellation can raise to 1e-5), and the
    # FP64 oracle to FP32 accuracy (the entropy fix and the acoustic
    # amplitudes cancel on near-sonic edges)
    cp = mc.mc_ctx_create(mc.MC_EULER_ROE, mc.MC_F32, mc.params(gamma=GM), 8, 8, 0.125, 0.125)
    am2, ap2 = t.empty_like(am), t.empty_like(ap)
    mc.mc_rp2(cp, ixy, n, dev(ql.astype(np.float32)), dev(qr.astype(np.float32)), None, t.empty_like(w),
              t.empty_like(s), am2, ap2)
    AM2, AP2 = host(am2), host(ap2)
    mc.mc_ctx_destroy(cp)
    e32 = (np.abs(AM - AM2).max(axis=0) + np.abs(AP - AP2).max(axis=0)) / scale
    say("fallback vs FP32 Roe: max", e32[~net].max(), "vs FP64 oracle: median",
        np.median(err[~net]), "max", err[~net].max())
    assert e32[~net].max() < (1e-6 if ixy == 1 else 1e-5)
    assert np.median(err[~net]) < 1e-6 and err[~net].max() < 2e-3
    # the network's waves sit in slots 0, 1 and 3
    assert not W[2][:, net].any() and not Sp[2][net].any()
    mc.mc_ctx_destroy(ctx)
    mc.mc_sur_destroy(sur)


# ------------------------------------------------------------ the split step
def run_sur_steps(sur, q0, dts, limiter, bc):
    t = _t()
    _, ny, nx = q0.shape
    ctx = mc.mc_ctx_create(MODEL, mc.MC_F32, mc.params(gamma=GM), nx, ny, 1.0 / nx, 1.0 / ny)
    mc.mc_ctx_set_surrogate(ctx, sur)
    a = dev(q0.astype(np.float32))
    b = t.empty_like(a)
    st = mc.state(a, b)
    cfl = t.zeros(16, dtype=t.uint8, device="cuda")
    for dt in dts:
        mc.mc_step2d(ctx, st, None, float(dt), limiter, bc, cfl)
    q = host(a if st.cur == 0 else b).astype(np.float64)
    c = mc.cfl_from_tensor(cfl)
    stats = mc.mc_sur_edge_stats(ctx)
    mc.mc_ctx_destroy(ctx)
    return q, c, stats


@pytest.mark.parametrize("bc", [0, 1])
def test_step_matches_oracle(S, O, bc):
    nx, ny = 72, 64
    say("case: Euler surrogate step", nx, "x", ny, "bc", bc)
    q0, _ = inputs.euler_quadrants(nx, seed=74, ny=ny)
    q0 = q0.astype(np.float32).astype(np.float64)
    th = random_theta(S, 75, bias=0.0) * 0.5
    sur = net_with(th)
    th32 = th.astype(np.float32).astype(np.float64)
    P = O.params(gamma=GM)
    sm0, _ = O.max_speed(O.EULER_ROE, P, q0, 1 / nx, 1 / ny, bc)
    # the untrained network's speeds exceed the physical ones: a zero-dt
    # oracle step measures them, and dt keeps the Courant number at 0.4
    _, sm1, _ = S.step2d(S.eu_surrogate_rp(th32, GM), q0, 1 / nx, 1 / ny, 0.0, O.LIM_MC, bc)
    dts = [0.4 / max(sm0, sm1)] * 3
    q, c, (ne, nfb) = run_sur_steps(sur, q0, dts, mc.MC_LIM_MC, bc)
    qo = q0
    for dt in dts:
        qo, smo, _ = S.step2d(S.eu_surrogate_rp(th32, GM), qo, 1 / nx, 1 / ny, dt, O.LIM_MC, bc)
    err = [np.abs(q[m] - qo[m]).sum() / np.abs(qo[m]).sum() for m in (0, 3)]
    say("rel L1 rho, E", err, "smax gpu", c.smax, "oracle", smo, "edges", ne, "fallback", nfb)
    assert max(err) < 1e-4
    # momenta against rho c (they may vanish in a quadrant)
    pr = (GM - 1.0) * (qo[3] - 0.5 * (qo[1] ** 2 + qo[2] ** 2) / qo[0])
    rc = np.abs(np.sqrt(GM * pr * qo[0])).sum()
    assert all(np.abs(q[m] - qo[m]).sum() / rc < 1e-4 for m in (1, 2))
    assert abs(c.smax - smo) <= 1e-3 * smo
    assert ne == 3 * ((nx + 3) * ny + (ny + 3) * nx)
    mc.mc_sur_destroy(sur)


def test_step_conserves_periodic(S):
    nx = ny = 64
    say("case: Euler surrogate step conservation", nx)
    q0, _ = inputs.euler_quadrants(nx, seed=76)
    q0 = q0.astype(np.float32).astype(np.float64)
    sur = net_with(random_theta(S, 77) * 0.5)
    q, c, _ = run_sur_steps(sur, q0, [1e-3] * 5, mc.MC_LIM_MC, 0)
    for m in range(4):
        drift = abs(q[m].sum() - q0[m].sum()) / np.abs(q0[m]).sum()
        say("field", m, "relative drift", drift)
        assert drift < 2e-6
    mc.mc_sur_destroy(sur)


def test_model_must_match_context():
    say("case: surrogate model / context solver mismatch")
    sw = mc.mc_sur_create(64, mc.MC_SW_SURROGATE)
    eu = mc.mc_sur_create(64, MODEL)
    c_eu = mc.mc_ctx_create(MODEL, mc.MC_F32, mc.params(), 8, 8, 0.1, 0.1)
    c_sw = mc.mc_ctx_create(mc.MC_SW_SURROGATE, mc.MC_F32, mc.params(), 8, 8, 0.1, 0.1)
    with pytest.raises(mc.ManyclawError):
        mc.mc_ctx_set_surrogate(c_eu, sw)
    with pytest.raises(mc.ManyclawError):
        mc.mc_ctx_set_surrogate(c_sw, eu)
    mc.mc_ctx_set_surrogate(c_eu, eu)
    mc.mc_ctx_set_surrogate(c_sw, sw)
    with pytest.raises(mc.ManyclawError):
        mc.mc_sur_create(64, mc.MC_EULER_ROE)
    for c in (c_eu, c_sw):
        mc.mc_ctx_destroy(c)
    mc.mc_sur_destroy(sw)
    mc.mc_sur_destroy(eu)
