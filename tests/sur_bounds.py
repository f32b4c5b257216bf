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
edge solve with the outputs given.
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

        def solve(O):
            return S.eu_rp2(th, ixy, ql, qr, par, True, outputs=O)
    else:
        nl, nr = S.to_normal(ql, ixy), S.to_normal(qr, ixy)
        X = S.features(nl, nr, par)[0]

        def solve(O):
            return S.rp2(th, ixy, ql, qr, par, True, outputs=O)
    O, _ = S.forward(th, X, emulate=True)
    ob = network_bound(S, th, X, inputs=True)
    bam = np.zeros((ql.shape[0], ql.shape[1]))
    bap = np.zeros_like(bam)
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
