"""Element-wise bounds for the GPU tests of the learned edge solvers, from
the surrogate oracle (oracle/surrogate.py).

A network output of the device and the oracle's BF16/FP32 emulation of it
differ only by rounding: the device sums in another order and evaluates
GELU in FP32, so a value close to a BF16 rounding midpoint can round to the
other neighbour, and the values after it then round independently of the
emulation's.  `rounding_spread` gives the standard deviation sigma of that
difference under the fully decorrelated model (pinned in
tests/test_oracle_surrogate.py: worst-case and random re-roundings stay
within 6 sigma plus the FP32 floor, seen up to about 3.2 sigma), so every
output is held to K_SIGMA sigma plus the floor.

The fluctuations of an edge are smooth functions of the network outputs
(decoding, projection onto the flux difference, upwind split), so their
bound is the sum over outputs of |d fluctuation / d output| times that
output's bound, the derivatives by central differences of the oracle's
edge solve with the outputs given; plus the effect of the device's FP32
arithmetic between states and fluctuations, as the change of the oracle's
fluctuations over a few FP32 units of each state value (input_bound).
"""
import numpy as np

K_SIGMA = 6.0
FP32_FLOOR = 2.0 ** -17     # 128 units of FP32 rounding, relative to the magnitudes involved


def network_bound(S, th, X, inputs=False):
    """per row and output: K_SIGMA sigma + the FP32 floor of the final sums"""
    sig, floor = S.rounding_spread(th, X, inputs=inputs)
    return K_SIGMA * sig + floor


def fluct_bound(S, th, ixy, ql, qr, par, euler=False):
    """(bound on |A-dQ(device) - A-dQ(oracle)|, same for A+dQ), each
    [meqn][n], for the network edges of the oracle's edge solve in grid
    orientation; the network inputs are computed apart on each side (FP32
    on the device), so their roundings count too."""
    if euler:
        nl, nr = S.eu_to_normal(ql, ixy), S.eu_to_normal(qr, ixy)
        fl = S.eu_flags(nl, nr, par)
        X = S.eu_features(nl, nr, par)[0]
        X = np.where(fl[:, None] == 0, X, 0.0)

        def solve(O, a=ql, b=qr):
            return S.eu_rp2(th, ixy, a, b, par, True, outputs=O)
    else:
        nl, nr = S.to_normal(ql, ixy), S.to_normal(qr, ixy)
        X = S.features(nl, nr, par)[0]

        def solve(O, a=ql, b=qr):
            return S.rp2(th, ixy, a, b, par, True, outputs=O)
    O, _ = S.forward(th, X, emulate=True)
    bam, bap = input_bound(solve, O, ql, qr)
    ob = network_bound(S, th, X, inputs=True)
    for j in range(O.shape[1]):
        h = 1e-6 * (1.0 + np.abs(O[:, j]))
        Op, Om = O.copy(), O.copy()
        Op[:, j] += h
        Om[:, j] -= h
        _, _, amp, app, _ = solve(Op)
        _, _, amm, apm, _ = solve(Om)
        bam += np.abs(amp - amm) / (2.0 * h) * ob[:, j]
        bap += np.abs(app - apm) / (2.0 * h) * ob[:, j]
    return bam, bap


INPUT_ULPS = 8.0          # FP32 units per state value covering the device's feature and decode arithmetic


def input_bound(solve, O, ql, qr, ulps=INPUT_ULPS):
    """The device computes an edge's features, decoding and projection in
    FP32: on an edge whose fluctuations are steep in the states (an upwind
    split near a zero speed, a near-cancelling projection) its rounding
    moves them more than the FP32 floor of their magnitudes.  Bound: for
    every state value of either side, half the change of the oracle's
    fluctuations (network outputs held at O) over +-ulps FP32 units of that
    value, summed over the values.  Returns (for A-dQ, for A+dQ), [meqn][n]."""
    bam = np.zeros(ql.shape)
    bap = np.zeros(ql.shape)
    for side in (0, 1):
        q = ql if side == 0 else qr
        for m in range(q.shape[0]):
            h = ulps * np.spacing(np.abs(q[m]).astype(np.float32)).astype(np.float64)
            res = []
            for sg in (1.0, -1.0):
                qq = q.copy()
                qq[m] = q[m] + sg * h
                a, b = (qq, qr) if side == 0 else (ql, qq)
                _, _, am, ap, _ = solve(O, a, b)
                res.append((am, ap))
            bam += 0.5 * np.abs(res[0][0] - res[1][0])
            bap += 0.5 * np.abs(res[0][1] - res[1][1])
    return np.nan_to_num(bam), np.nan_to_num(bap)


def check_fluct(say, AM, AP, amo, apo, bam, bap, fs, net):
    """assert the element-wise bound on every network edge and component;
    fs: |f(qL)| + |f(qR)| per component (grid orientation)"""
    floor_am = FP32_FLOOR * (np.abs(amo) + np.abs(apo) + fs)
    r_am = np.abs(AM - amo) / (bam + floor_am)
    r_ap = np.abs(AP - apo) / (bap + floor_am)
    worst = max(r_am[:, net].max(), r_ap[:, net].max())
    rel = (np.abs(AM - amo) + np.abs(AP - apo)) / (np.abs(amo) + np.abs(apo) + 1e-30)
    say(f"fluctuations / element-wise bound: max {worst:.3f}, median "
        f"{np.median(np.maximum(r_am, r_ap)[:, net]):.2e}; relative error median "
        f"{np.median(rel[:, net]):.2e}, max {rel[:, net].max():.2e}; bound / |fluct| median "
        f"{np.median(((bam + bap) / (np.abs(amo) + np.abs(apo) + 1e-30))[:, net]):.2e}")
    assert worst <= 1.0, worst



GELU_D1 = 1.13            # max |gelu'| over the real line
SUM_REL = 2.0 ** -21      # typical FP32 summation difference: 8 roundings of the sum of |terms|
GELU_REL = 2.0 ** -22     # typical device GELU error (exp2, reciprocal, three products): 4 ulps


def flip_rms(S, th, X, sum_rel=SUM_REL, gelu_rel=GELU_REL):
    """Root of the expected sum of squares of (device - emulation) over all
    rows and outputs, when the two differ through BF16 rounding flips: a
    hidden operand whose pre-rounding values differ by d (the typical FP32
    difference of its sum in another order, sum_rel times the sum of its
    absolute terms, through GELU's slope, plus the device GELU's typical
    error) rounds to the other neighbour with probability min(1, 2 d / u)
    for a position uniform within its spacing u, and then moves the outputs
    by u times d out / d operand (back-propagation through the emulated
    network); flips are taken as independent.  The inputs are the same FP32
    values on both sides.  Over many rows the sum of squares concentrates
    at this expectation; the worst-case rounding model (the FP32 floor
    2^-17 and decorrelated operands, rounding_spread) bounds each element
    but overstates the sum about 60-fold."""
    a = np.asarray(X, dtype=np.float64)
    layers = S.unpack(th)
    nl = len(layers)
    Wq, zs, pu2 = [], [], []
    for l, (W, b) in enumerate(layers):
        q = S.bf16(a)
        u, _ = S.bf16_spacing(q, a)
        W16 = S.bf16(W)
        Wq.append(W16)
        z = S.f32(q @ W16.T + S.f32(b))
        zs.append(z)
        if l == 0:
            pu2.append(np.zeros_like(u))
        dz = sum_rel * (np.abs(q) @ np.abs(W16).T + np.abs(S.f32(b)))
        if l < nl - 1:
            a = S.gelu(z)
            da = np.minimum(GELU_D1, np.abs(S.gelu_grad(z))) * dz + gelu_rel * np.abs(a)
            qn = S.bf16(a)
            un, _ = S.bf16_spacing(qn, a)
            p = np.minimum(1.0, 2.0 * da / un)
            pu2.append(p * un * un)
    n, nout = zs[-1].shape
    tot = 0.0
    for j in range(nout):
        dz = np.zeros((n, nout))
        dz[:, j] = 1.0
        for l in range(nl - 1, -1, -1):
            dA = dz @ Wq[l]
            tot += float((dA * dA * pu2[l]).sum())
            if l > 0:
                dz = dA * S.gelu_grad(zs[l - 1])
    return np.sqrt(tot)
