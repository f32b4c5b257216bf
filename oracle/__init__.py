"""Plain FP64 CPU oracle of the 2D wave-propagation step (ctypes binding).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are the only users.  The product path never imports this
package, and this package never imports the product package.

The arithmetic lives in ``mco.c`` (solvers, limiters, split step, time-step
rule) and ``surrogate.py`` (the learned shallow-water edge solver: network
forward/backward, Adam, labels, projection, fallback and a whole-sweep split
step, in NumPy); this module only marshals NumPy arrays.  Constants below
mirror the enum values of ``mco.h``.
"""
import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "liboracle.so")

ADVECTION, ACOUSTICS, ACOUSTICS_VC, SW_ROE, EULER_ROE, SW_HLLE = range(6)
LIM_NONE, LIM_MINMOD, LIM_SUPERBEE, LIM_VANLEER, LIM_MC, LIM_FIRST_ORDER = range(6)
BC_PERIODIC, BC_EXTRAP = 0, 1
ST_NONPHYS, ST_FALLBACK, ST_BADARG, ST_STALLED = 1, 2, 4, 8

DIMS = {  # solver: (meqn, mwaves, maux)
    ADVECTION: (1, 1, 0),
    ACOUSTICS: (3, 2, 0),
    ACOUSTICS_VC: (3, 2, 2),
    SW_ROE: (3, 3, 0),
    EULER_ROE: (4, 4, 0),
    SW_HLLE: (3, 3, 0),
}


class Params(ctypes.Structure):
    _fields_ = [("g", ctypes.c_double), ("gamma", ctypes.c_double),
                ("rho", ctypes.c_double), ("K", ctypes.c_double),
                ("u", ctypes.c_double), ("v", ctypes.c_double)]


def params(g=9.81, gamma=1.4, rho=1.0, K=1.0, u=1.0, v=1.0):
    return Params(g, gamma, rho, K, u, v)


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(LIBPATH)
        dp = ctypes.POINTER(ctypes.c_double)
        L.mco_rp2.argtypes = [ctypes.c_int, ctypes.POINTER(Params), ctypes.c_int, ctypes.c_int64,
                              dp, dp, dp, dp, dp, dp, dp]
        L.mco_rp2.restype = ctypes.c_int
        L.mco_phi.argtypes = [ctypes.c_int, ctypes.c_double]
        L.mco_phi.restype = ctypes.c_double
        L.mco_step2d.argtypes = [ctypes.c_int, ctypes.POINTER(Params), ctypes.c_int, ctypes.c_int,
                                 ctypes.c_double, ctypes.c_double, dp, dp, ctypes.c_double,
                                 ctypes.c_int, ctypes.c_int, dp, dp, ctypes.c_int]
        L.mco_step2d.restype = ctypes.c_int
        L.mco_max_speed.argtypes = [ctypes.c_int, ctypes.POINTER(Params), ctypes.c_int, ctypes.c_int,
                                    ctypes.c_double, ctypes.c_double, dp, dp, ctypes.c_int, dp,
                                    ctypes.c_int]
        L.mco_max_speed.restype = ctypes.c_int
        L.mco_run2d.argtypes = [ctypes.c_int, ctypes.POINTER(Params), ctypes.c_int, ctypes.c_int,
                                ctypes.c_double, ctypes.c_double, dp, dp, ctypes.c_int,
                                ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                dp, dp, ctypes.POINTER(ctypes.c_int), ctypes.c_int]
        L.mco_run2d.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def rp2(solver, P, ixy, ql, qr, aux=None):
    """n independent edge solves; ql, qr: [meqn][n]; aux: [2][maux][n] or None.
    Returns waves [mwaves][meqn][n], speeds [mwaves][n], amdq, apdq [meqn][n],
    status bits."""
    meqn, mwaves, maux = DIMS[solver]
    ql = _f64(ql).reshape(meqn, -1)
    qr = _f64(qr).reshape(meqn, -1)
    n = ql.shape[1]
    auxa = _f64(aux).reshape(2, maux, n) if maux else None
    waves = np.empty((mwaves, meqn, n))
    speeds = np.empty((mwaves, n))
    amdq = np.empty((meqn, n))
    apdq = np.empty((meqn, n))
    st = lib().mco_rp2(solver, ctypes.byref(P), ixy, n, _p(ql), _p(qr), _p(auxa),
                       _p(waves), _p(speeds), _p(amdq), _p(apdq))
    return waves, speeds, amdq, apdq, st


def phi(limiter, theta):
    return lib().mco_phi(limiter, float(theta))


def step2d(solver, P, q, dx, dy, dt, limiter, bc, aux=None, nthreads=1):
    """One split step.  q: [meqn][ny][nx].  Returns (q_next, smax, status)."""
    q = _f64(q)
    meqn, ny, nx = q.shape
    auxa = _f64(aux) if aux is not None else None
    out = np.empty_like(q)
    sm = ctypes.c_double(0.0)
    st = lib().mco_step2d(solver, ctypes.byref(P), nx, ny, dx, dy, _p(q), _p(auxa), dt,
                          limiter, bc, _p(out), ctypes.pointer(sm), nthreads)
    if st & ST_BADARG:
        raise ValueError("mco_step2d: bad argument")
    return out, sm.value, st


def max_speed(solver, P, q, dx, dy, bc, aux=None, nthreads=1):
    q = _f64(q)
    meqn, ny, nx = q.shape
    auxa = _f64(aux) if aux is not None else None
    sm = ctypes.c_double(0.0)
    st = lib().mco_max_speed(solver, ctypes.byref(P), nx, ny, dx, dy, _p(q), _p(auxa), bc,
                             ctypes.pointer(sm), nthreads)
    if st & ST_BADARG:
        raise ValueError("mco_max_speed: bad argument")
    return sm.value, st


def run2d(solver, P, q, dx, dy, limiter, bc, cfl_target, cfl_max, nsteps, aux=None,
          nthreads=1):
    """nsteps accepted steps under the variable time-step rule.
    Returns (q_final, dt_history, t, n_rejected, status)."""
    q = _f64(q).copy()
    meqn, ny, nx = q.shape
    auxa = _f64(aux) if aux is not None else None
    dts = np.zeros(max(nsteps, 1))
    t = ctypes.c_double(0.0)
    nrej = ctypes.c_int(0)
    st = lib().mco_run2d(solver, ctypes.byref(P), nx, ny, dx, dy, _p(q), _p(auxa), limiter, bc,
                         cfl_target, cfl_max, nsteps, _p(dts), ctypes.pointer(t),
                         ctypes.pointer(nrej), nthreads)
    if st & ST_BADARG:
        raise ValueError("mco_run2d: bad argument")
    return q, dts[:nsteps], t.value, nrej.value, st
