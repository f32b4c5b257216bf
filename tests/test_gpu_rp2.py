"""GPU parity of mc_rp2 (the batched edge Riemann solve) against the oracle,
element by element, on seeded random states."""
import numpy as np
import pytest

import gpu_util as gu
from paper_1308_1464_amd import inputs
from paper_1308_1464_amd import manyclaw as mc

pytestmark = pytest.mark.gpu

ORC = {mc.MC_ADVECTION: 0, mc.MC_ACOUSTICS: 1, mc.MC_ACOUSTICS_VC: 2, mc.MC_SW_ROE: 3,
       mc.MC_EULER_ROE: 4, mc.MC_SW_HLLE: 5}


def _states(solver, n, seed):
    if solver == mc.MC_ADVECTION:
        g = inputs.rng(seed)
        return g.normal(size=(1, n)), g.normal(size=(1, n)), None
    if solver in (mc.MC_ACOUSTICS, mc.MC_ACOUSTICS_VC):
        ql, qr = inputs.acoustics_random_states(n, seed)
        aux = None
        if solver == mc.MC_ACOUSTICS_VC:
            g = inputs.rng(seed + 100)
            aux = g.uniform(0.5, 3.0, size=(2, 2, n))
        return ql, qr, aux
    if solver == mc.MC_EULER_ROE:
        ql, qr = inputs.euler_random_states(n, seed)
        return ql, qr, None
    ql, qr = inputs.sw_random_states(n, seed, hlo=1e-2, hhi=10.0, ulim=5.0)
    return ql, qr, None


def _run_gpu(solver, dtype, ixy, ql, qr, aux, prm):
    T = gu.npdt(dtype)
    meqn, mw, maux = mc.mc_solver_dims(solver)
    n = ql.shape[1]
    dql, dqr = gu.dev(ql, T), gu.dev(qr, T)
    daux = gu.dev(aux, T) if aux is not None else None
    W = gu.empty((mw, meqn, n), T)
    S = gu.empty((mw, n), T)
    am = gu.empty((meqn, n), T)
    ap = gu.empty((meqn, n), T)
    with gu.context(solver, dtype, prm, 8, 8, 0.1, 0.1) as h:
        mc.mc_rp2(h, ixy, n, dql, dqr, daux, W, S, am, ap)
        st = mc.mc_status_get(h)
    return gu.host(W), gu.host(S), gu.host(am), gu.host(ap), st


def _cmp(a, b):
    den = np.abs(b).max()
    return np.abs(a - b).max() / (den if den > 0 else 1.0)


@pytest.mark.parametrize("solver", [mc.MC_ADVECTION, mc.MC_ACOUSTICS, mc.MC_ACOUSTICS_VC,
                                    mc.MC_SW_ROE, mc.MC_SW_HLLE, mc.MC_EULER_ROE])
@pytest.mark.parametrize("dtype", [mc.MC_F64, mc.MC_F32])
@pytest.mark.parametrize("ixy", [1, 2])
def test_rp2_matches_oracle(orc, solver, dtype, ixy):
    n = 100003  # several thousand workgroups' worth plus a ragged tail
    print(f"rp2 parity solver={solver} dtype={dtype} ixy={ixy} n={n}", flush=True)
    ql, qr, aux = _states(solver, n, seed=17 + solver)
    T = gu.npdt(dtype)
    # the oracle sees exactly the values the device sees
    ql, qr = ql.astype(T).astype(np.float64), qr.astype(T).astype(np.float64)
    if aux is not None:
        aux = aux.astype(T).astype(np.float64)
    prm = mc.params(u=0.7, v=-1.3, rho=1.3, K=2.0)
    P = orc.params(u=0.7, v=-1.3, rho=1.3, K=2.0)
    W, S, am, ap, st = _run_gpu(solver, dtype, ixy, ql, qr, aux, prm)
    W0, S0, am0, ap0, st0 = orc.rp2(ORC[solver], P, ixy, ql, qr, aux)
    tol = 1e-13 if dtype == mc.MC_F64 else 2e-5
    keep = np.ones(n, dtype=bool)
    if solver == mc.MC_EULER_ROE:
        # Roe/HLLE switch is a discontinuous decision: compare edges where
        # both sides took the same branch, and require that almost all did
        fb_gpu = (S[1] == 0) & (S[2] == 0)
        fb_orc = (S0[1] == 0) & (S0[2] == 0)
        keep = fb_gpu == fb_orc
        assert keep.mean() > 0.999, keep.mean()
    for name, a, b in (("waves", W, W0), ("speeds", S, S0), ("amdq", am, am0), ("apdq", ap, ap0)):
        err = _cmp(a[..., keep], b[..., keep])
        assert err <= tol, (name, err)
    assert (st & mc.MC_ST_FALLBACK) == (st0 & 2) or solver != mc.MC_EULER_ROE


def test_rp2_edge_cases(orc):
    prm = mc.params()
    P = orc.params()
    # n = 0 is a no-op; n = 1 works; unphysical depth is flagged and zeroed
    with gu.context(mc.MC_SW_ROE, mc.MC_F64, prm, 4, 4, 1.0, 1.0) as h:
        mc.mc_rp2(h, 1, 0, 0, 0, None, 0, 0, 0, 0)
    ql = np.array([[1.0, -0.5], [0.2, 0.0], [0.1, 0.0]])
    qr = np.array([[1.5, 1.0], [-0.3, 0.0], [0.0, 0.0]])
    W, S, am, ap, st = _run_gpu(mc.MC_SW_ROE, mc.MC_F64, 1, ql, qr, None, prm)
    W0, S0, am0, ap0, st0 = orc.rp2(3, P, 1, ql, qr)
    assert st & mc.MC_ST_NONPHYS and st0 & 1
    assert np.all(am[:, 1] == 0) and np.all(ap[:, 1] == 0)
    np.testing.assert_allclose(am[:, 0], am0[:, 0], rtol=1e-14, atol=1e-15)
    # invalid arguments are rejected on the host
    with gu.context(mc.MC_SW_ROE, mc.MC_F64, prm, 4, 4, 1.0, 1.0) as h:
        with pytest.raises(mc.ManyclawError):
            mc.mc_rp2(h, 3, 10, 1, 1, None, 1, 1, 1, 1)
        with pytest.raises(mc.ManyclawError):
            mc.mc_rp2(h, 1, -1, 1, 1, None, 1, 1, 1, 1)
        with pytest.raises(mc.ManyclawError):
            mc.mc_rp2(h, 1, 10, None, 1, None, 1, 1, 1, 1)
