"""ctypes binding of libmanyclaw.so (include/manyclaw.h).

Argument marshalling only: every function forwards to the C entry point of
the same name; all arithmetic runs in the HIP kernels.  Arrays are torch
tensors on the GPU (torch supplies device memory and the stream) or raw
device addresses (int).  The library is loaded on first use; if it is missing
or cannot be loaded an ImportError is raised -- there is no fallback path.
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIBPATH = os.path.join(HERE, "libmanyclaw.so")

MC_OK, MC_EINVAL, MC_ENOMEM, MC_EHIP, MC_ECFL, MC_ENONPHYS, MC_EUNSUPPORTED = 0, -1, -2, -3, -4, -5, -6
MC_ESCRATCH = -7
(MC_ADVECTION, MC_ACOUSTICS, MC_ACOUSTICS_VC, MC_SW_ROE, MC_EULER_ROE, MC_SW_HLLE, MC_SW_SURROGATE,
 MC_EULER_SURROGATE) = range(8)
MC_LIM_NONE, MC_LIM_MINMOD, MC_LIM_SUPERBEE, MC_LIM_VANLEER, MC_LIM_MC, MC_LIM_FIRST_ORDER = range(6)
MC_BC_PERIODIC, MC_BC_EXTRAP = 0, 1
MC_F64, MC_F32 = 0, 1
MC_ST_NONPHYS, MC_ST_FALLBACK, MC_ST_CFL = 1, 2, 4
MC_MAX_RETRIES = 8


class mc_params(ctypes.Structure):
    _fields_ = [("g", ctypes.c_double), ("gamma", ctypes.c_double), ("rho", ctypes.c_double),
                ("K", ctypes.c_double), ("u", ctypes.c_double), ("v", ctypes.c_double),
                ("cfl_target", ctypes.c_double), ("cfl_max", ctypes.c_double)]


class mc_state(ctypes.Structure):
    _fields_ = [("q", ctypes.c_void_p * 2), ("cur", ctypes.c_int32)]


class mc_cfl(ctypes.Structure):
    _fields_ = [("smax", ctypes.c_double), ("cfl", ctypes.c_double)]


class mc_clock(ctypes.Structure):
    _fields_ = [("t", ctypes.c_double), ("dt", ctypes.c_double), ("cfl", ctypes.c_double),
                ("smax", ctypes.c_double), ("cur", ctypes.c_int32), ("n_acc", ctypes.c_int32),
                ("n_rej", ctypes.c_int32), ("status", ctypes.c_int32),
                ("cfl_target", ctypes.c_double), ("cfl_max", ctypes.c_double),
                ("rej_run", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class mc_patch(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("offset", ctypes.c_int64),
                ("dx", ctypes.c_double), ("dy", ctypes.c_double), ("t", ctypes.c_double),
                ("dt", ctypes.c_double), ("cfl", ctypes.c_double), ("smax", ctypes.c_double),
                ("bc", ctypes.c_int32), ("status", ctypes.c_int32), ("n_acc", ctypes.c_int32),
                ("n_rej", ctypes.c_int32), ("cur", ctypes.c_int32), ("reserved", ctypes.c_int32)]


_STRERR = {0: "ok", -1: "invalid argument", -2: "out of device memory", -3: "HIP runtime error",
           -4: "step rejected by the CFL rule", -5: "non-physical state", -6: "unsupported",
           -7: "request exceeds the static device array"}


class ManyclawError(RuntimeError):
    def __init__(self, fn, code, why=None):
        msg = f"{fn} failed: {code} ({_STRERR.get(code, 'unknown error')})"
        super().__init__(msg + (f": {why}" if why else ""))
        self.code = code


# exported symbols and their C signatures (restype, argtypes)
_VP = ctypes.c_void_p
_SIGS = {
    "mc_ctx_create": (ctypes.c_int, [ctypes.POINTER(_VP), ctypes.c_int, ctypes.c_int,
                                     ctypes.POINTER(mc_params), ctypes.c_int32, ctypes.c_int32,
                                     ctypes.c_double, ctypes.c_double, _VP]),
    "mc_ctx_destroy": (None, [_VP]),
    "mc_ctx_set_tile": (ctypes.c_int, [_VP, ctypes.c_int32]),
    "mc_tune_rows": (ctypes.c_int, [_VP, ctypes.POINTER(mc_state), _VP, ctypes.c_double, ctypes.c_int,
                                    ctypes.c_int, ctypes.POINTER(ctypes.c_int32)]),
    "mc_rp2": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.c_int64, _VP, _VP, _VP, _VP, _VP, _VP, _VP]),
    "mc_step2d": (ctypes.c_int, [_VP, ctypes.POINTER(mc_state), _VP, ctypes.c_double, ctypes.c_int,
                                 ctypes.c_int, _VP]),
    "mc_max_speed": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int, _VP]),
    "mc_clock_init": (ctypes.c_int, [_VP, _VP, _VP, _VP, ctypes.c_int]),
    "mc_run2d": (ctypes.c_int, [_VP, _VP, _VP, _VP, _VP, ctypes.c_int32, ctypes.c_int, ctypes.c_int,
                                ctypes.c_int]),
    "mc_status_get": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_int32)]),
    "mc_copy_probe": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int64]),
    "mc_step2d_patches": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int32, _VP, _VP, ctypes.c_int32,
                                         ctypes.c_int, ctypes.c_int]),
    "mc_step2d_patches_noalloc": (ctypes.c_int, [_VP, _VP, _VP, ctypes.c_int32, _VP, _VP, ctypes.c_int32,
                                                 ctypes.c_int]),
    "mc_patches_tune": (ctypes.c_int, [_VP, _VP, ctypes.c_int32, ctypes.c_int,
                                       ctypes.POINTER(ctypes.c_int32)]),
    "mc_patches_set_rows": (ctypes.c_int, [_VP, _VP, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32)]),
    "mc_solver_dims": (ctypes.c_int, [ctypes.c_int, ctypes.POINTER(ctypes.c_int32),
                                      ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
    "mc_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "mc_step2d_strang": (ctypes.c_int, [_VP, ctypes.POINTER(mc_state), _VP, ctypes.c_double, ctypes.c_int,
                                        ctypes.c_int, _VP]),
    "mc_step2d_unsplit": (ctypes.c_int, [_VP, ctypes.POINTER(mc_state), _VP, ctypes.c_double, ctypes.c_int,
                                         ctypes.c_int, _VP]),
    "mc_amr_create": (ctypes.c_int, [ctypes.POINTER(_VP), _VP, ctypes.c_int32, ctypes.c_int32, _VP,
                                     ctypes.c_int32]),
    "mc_amr_destroy": (None, [_VP]),
    "mc_amr_dims": (ctypes.c_int, [_VP, ctypes.c_int32, ctypes.POINTER(ctypes.c_int32),
                                   ctypes.POINTER(ctypes.c_int32)]),
    "mc_amr_set": (ctypes.c_int, [_VP, ctypes.c_int32, _VP]),
    "mc_amr_get": (ctypes.c_int, [_VP, ctypes.c_int32, _VP]),
    "mc_amr_step": (ctypes.c_int, [_VP, ctypes.c_double, ctypes.c_int32, _VP]),
    "mc_sur_dims": (ctypes.c_int, [ctypes.c_int32] + [ctypes.POINTER(ctypes.c_int32)] * 4),
    "mc_sur_create": (ctypes.c_int, [ctypes.POINTER(_VP), ctypes.c_int32, ctypes.c_int32, _VP]),
    "mc_sur_destroy": (None, [_VP]),
    "mc_sur_set_params": (ctypes.c_int, [_VP, _VP]),
    "mc_sur_get_params": (ctypes.c_int, [_VP, _VP]),
    "mc_sur_init_params": (ctypes.c_int, [_VP, _VP]),
    "mc_sur_gen": (ctypes.c_int, [_VP, ctypes.POINTER(mc_params), ctypes.c_int64, _VP, _VP, _VP, _VP]),
    "mc_sur_compact": (ctypes.c_int, [_VP, ctypes.c_int64, _VP, _VP, _VP, _VP, _VP,
                                      ctypes.POINTER(ctypes.c_int64)]),
    "mc_sur_forward": (ctypes.c_int, [_VP, ctypes.c_int64, _VP, _VP]),
    "mc_sur_loss_grad": (ctypes.c_int, [_VP, ctypes.c_int64, _VP, _VP, _VP, _VP]),
    "mc_sur_adam": (ctypes.c_int, [_VP, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                   ctypes.c_float]),
    "mc_sur_train": (ctypes.c_int, [_VP, ctypes.c_int64, _VP, _VP, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_float, ctypes.POINTER(ctypes.c_int32),
                                    ctypes.POINTER(ctypes.c_float)]),
    "mc_sur_eval": (ctypes.c_int, [_VP, ctypes.c_int64, _VP, _VP, ctypes.POINTER(ctypes.c_double)]),
    "mc_ctx_set_surrogate": (ctypes.c_int, [_VP, _VP]),
    "mc_sur_edge_stats": (ctypes.c_int, [_VP, ctypes.POINTER(ctypes.c_int64),
                                         ctypes.POINTER(ctypes.c_int64)]),
}

MC_SUR_NPARAMS, MC_SUR_NIN, MC_SUR_NOUT = 51464, 6, 8
MC_SUR_EU_NPARAMS, MC_SUR_EU_NIN, MC_SUR_EU_NOUT = 52495, 7, 15

_lib = None


def lib():
    """Load libmanyclaw.so (raises ImportError when it is absent).

    torch is imported first: its wheel carries its own HIP runtime under the
    same soname, and the library must bind to that one instance.  Loading
    the library before torch would map the system runtime as well, and two
    HIP runtimes in one process do not share the device."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIBPATH):
            raise ImportError(f"{LIBPATH} is not built; run paper_1308_1464_amd/build.py")
        import torch  # noqa: F401  (binds the library to torch's HIP runtime)
        L = ctypes.CDLL(LIBPATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def strerror(code):
    return lib().mc_strerror(int(code)).decode()


def _ptr(x):
    """device address of a tensor, an int address, or None"""
    if x is None:
        return None
    if isinstance(x, int):
        return x
    return x.data_ptr()


def _check(fn, rc):
    if rc != MC_OK:
        raise ManyclawError(fn, rc)
    return rc


def _stream_handle(stream):
    if stream is None:
        import torch
        return torch.cuda.current_stream().cuda_stream
    if isinstance(stream, int):
        return stream
    return stream.cuda_stream


def params(g=9.81, gamma=1.4, rho=1.0, K=1.0, u=1.0, v=1.0, cfl_target=0.9, cfl_max=1.0):
    return mc_params(g, gamma, rho, K, u, v, cfl_target, cfl_max)


def mc_solver_dims(solver):
    m, w, a = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check("mc_solver_dims", lib().mc_solver_dims(solver, ctypes.byref(m), ctypes.byref(w),
                                                  ctypes.byref(a)))
    return m.value, w.value, a.value


# solver, dtype and grid of each live context, for argument checks the C
# ABI cannot make (sizes of caller-owned device buffers, which it receives as
# bare addresses)
_CTX = {}
_MEQN = {MC_ADVECTION: 1, MC_ACOUSTICS: 3, MC_ACOUSTICS_VC: 3, MC_SW_ROE: 3, MC_EULER_ROE: 4,
         MC_SW_HLLE: 3, MC_SW_SURROGATE: 3, MC_EULER_SURROGATE: 4}
_MWAVES = {MC_ADVECTION: 1, MC_ACOUSTICS: 2, MC_ACOUSTICS_VC: 2, MC_SW_ROE: 3, MC_EULER_ROE: 4,
           MC_SW_HLLE: 3, MC_SW_SURROGATE: 3, MC_EULER_SURROGATE: 4}
_MAUX = {MC_ACOUSTICS_VC: 2}


def _nbytes(t):
    """bytes of a tensor argument; None for raw addresses and None"""
    return t.numel() * t.element_size() if hasattr(t, "numel") else None


def _arg(fn, t, nbytes=0, dtype=None):
    """Check one device-buffer argument before its address crosses the ABI.
    Raw int addresses and None pass through (the C side checks NULL).  A
    tensor must live on the GPU (a host address handed to a kernel faults the
    device), be contiguous (the kernels index it densely), hold elements of
    `dtype` (a torch dtype name, e.g. "float64") when one is given (anything
    else would be reinterpreted bit for bit), and span at least nbytes."""
    if t is None or isinstance(t, int):
        return
    if not hasattr(t, "data_ptr") or not hasattr(t, "numel"):
        raise ManyclawError(fn, MC_EINVAL, f"expected a tensor or an int address, got {type(t).__name__}")
    dev = getattr(t, "device", None)
    if dev is None or getattr(dev, "type", None) != "cuda":
        raise ManyclawError(fn, MC_EINVAL, f"tensor on {dev}, not on the GPU")
    if not t.is_contiguous():
        raise ManyclawError(fn, MC_EINVAL, "tensor is not contiguous")
    if dtype is not None and str(t.dtype) != "torch." + dtype:
        raise ManyclawError(fn, MC_EINVAL, f"tensor of {t.dtype}, expected torch.{dtype}")
    if t.numel() * t.element_size() < nbytes:
        raise ManyclawError(fn, MC_EINVAL,
                            f"tensor of {t.numel() * t.element_size()} bytes, needs {nbytes}")


def _need(fn, t, nbytes, dtype=None):
    _arg(fn, t, nbytes, dtype)


def _dtname(dtype):
    return "float64" if dtype == MC_F64 else "float32"


def _check_grid(fn, ctx, states=(), aux=None):
    """state buffers of meqn * nx * ny and aux of maux * nx * ny elements of
    the context's dtype, on the GPU and contiguous"""
    info = _CTX.get(getattr(ctx, "value", None))
    if info is None or len(info) < 4 or info[0] not in _MEQN:
        for b in states:
            _arg(fn, b)
        _arg(fn, aux)
        return
    solver, dtype, nx, ny = info[:4]
    esz = 8 if dtype == MC_F64 else 4
    cells = int(nx) * int(ny)
    for b in states:
        _arg(fn, b, _MEQN[solver] * cells * esz, _dtname(dtype))
    if _MAUX.get(solver, 0):
        _arg(fn, aux, _MAUX[solver] * cells * esz, _dtname(dtype))
    else:
        _arg(fn, aux)


def mc_ctx_create(solver, dtype, prm, nx, ny, dx, dy, stream=None):
    h = _VP()
    _check("mc_ctx_create", lib().mc_ctx_create(ctypes.byref(h), solver, dtype, ctypes.byref(prm),
                                                nx, ny, dx, dy, _stream_handle(stream)))
    _CTX[h.value] = (solver, dtype, nx, ny)
    return h


def mc_ctx_destroy(ctx):
    _CTX.pop(getattr(ctx, "value", ctx), None)
    lib().mc_ctx_destroy(ctx)


def _check_pools(fn, ctx, patches_host, n, pools):
    """each pool must hold meqn * nx * ny elements of the context's dtype from
    every patch's offset, on the GPU and contiguous (raw addresses pass
    through)"""
    info = _CTX.get(getattr(ctx, "value", None))
    if info is None or info[0] not in _MEQN or n < 1:
        for t in pools:
            _arg(fn, t)
        return
    need = max(int(patches_host[k].offset) + _MEQN[info[0]] * int(patches_host[k].nx) * int(patches_host[k].ny)
               for k in range(n))
    esz = 8 if info[1] == MC_F64 else 4
    for t in pools:
        _arg(fn, t, need * esz, _dtname(info[1]))


def mc_ctx_set_tile(ctx, rows):
    return _check("mc_ctx_set_tile", lib().mc_ctx_set_tile(ctx, rows))


def mc_rp2(ctx, ixy, n, q_left, q_right, aux, waves, speeds, amdq, apdq):
    info = _CTX.get(getattr(ctx, "value", None))
    arrs = (q_left, q_right, waves, speeds, amdq, apdq, aux)
    if info is not None and info[0] in _MEQN and n > 0:
        m, w, esz = _MEQN[info[0]], _MWAVES[info[0]], 8 if info[1] == MC_F64 else 4
        for t, k in zip(arrs, (m, m, w * m, w, m, m, 2 * _MAUX.get(info[0], 0))):
            _arg("mc_rp2", t, k * n * esz, _dtname(info[1]) if k else None)
    else:
        for t in arrs:
            _arg("mc_rp2", t)
    return _check("mc_rp2", lib().mc_rp2(ctx, ixy, n, _ptr(q_left), _ptr(q_right), _ptr(aux),
                                         _ptr(waves), _ptr(speeds), _ptr(amdq), _ptr(apdq)))


def mc_step2d(ctx, st, aux, dt, limiter, bc, cfl_out=None):
    """st: an mc_state (its cur is flipped by the call)"""
    _check_grid("mc_step2d", ctx, getattr(st, "bufs", ()), aux)
    _arg("mc_step2d", cfl_out, 16)
    return _check("mc_step2d", lib().mc_step2d(ctx, ctypes.byref(st), _ptr(aux), dt, limiter, bc,
                                               _ptr(cfl_out)))


def mc_tune_rows(ctx, st, aux, dt, limiter, bc):
    """times the split step's rows per work item (writes st's other buffer,
    st.cur unchanged) and keeps the fastest; returns it (0: occupancy rule)"""
    _check_grid("mc_tune_rows", ctx, getattr(st, "bufs", ()), aux)
    rows = ctypes.c_int32(0)
    _check("mc_tune_rows", lib().mc_tune_rows(ctx, ctypes.byref(st), _ptr(aux), dt, limiter, bc,
                                              ctypes.byref(rows)))
    return rows.value


def mc_step2d_strang(ctx, st, aux, dt, limiter, bc, cfl_out=None):
    """Strang-split step; st: an mc_state (its cur is flipped by the call)"""
    _check_grid("mc_step2d_strang", ctx, getattr(st, "bufs", ()), aux)
    _arg("mc_step2d_strang", cfl_out, 16)
    return _check("mc_step2d_strang", lib().mc_step2d_strang(ctx, ctypes.byref(st), _ptr(aux), dt, limiter,
                                                             bc, _ptr(cfl_out)))


def mc_step2d_unsplit(ctx, st, aux, dt, limiter, bc, cfl_out=None):
    """unsplit step with transverse solves; st: an mc_state (cur flips)"""
    _check_grid("mc_step2d_unsplit", ctx, getattr(st, "bufs", ()), aux)
    _arg("mc_step2d_unsplit", cfl_out, 16)
    return _check("mc_step2d_unsplit", lib().mc_step2d_unsplit(ctx, ctypes.byref(st), _ptr(aux), dt, limiter,
                                                               bc, _ptr(cfl_out)))


def mc_max_speed(ctx, q, aux, bc, out):
    _check_grid("mc_max_speed", ctx, (q,), aux)
    _arg("mc_max_speed", out, 16)
    return _check("mc_max_speed", lib().mc_max_speed(ctx, _ptr(q), _ptr(aux), bc, _ptr(out)))


def mc_clock_init(ctx, clk, q, aux, bc):
    _check_grid("mc_clock_init", ctx, (q,), aux)
    _arg("mc_clock_init", clk, ctypes.sizeof(mc_clock))
    return _check("mc_clock_init", lib().mc_clock_init(ctx, _ptr(clk), _ptr(q), _ptr(aux), bc))


def mc_run2d(ctx, q0, q1, aux, clk, nsteps, limiter, bc, use_graph=False):
    _check_grid("mc_run2d", ctx, (q0, q1), aux)
    _arg("mc_run2d", clk, ctypes.sizeof(mc_clock))
    return _check("mc_run2d", lib().mc_run2d(ctx, _ptr(q0), _ptr(q1), _ptr(aux), _ptr(clk), nsteps,
                                             limiter, bc, 1 if use_graph else 0))


def mc_copy_probe(ctx, dst, src, nbytes):
    _arg("mc_copy_probe", dst, nbytes)
    _arg("mc_copy_probe", src, nbytes)
    return _check("mc_copy_probe", lib().mc_copy_probe(ctx, _ptr(dst), _ptr(src), nbytes))


def patch_array(descs):
    """host array of mc_patch from a list of dicts (or mc_patch)"""
    arr = (mc_patch * len(descs))()
    for k, d in enumerate(descs):
        if isinstance(d, mc_patch):
            arr[k] = d
        else:
            for f, v in d.items():
                setattr(arr[k], f, v)
    return arr


def mc_step2d_patches(ctx, patches_host, patches_dev, n, pool0, pool1, nsteps, limiter,
                      use_graph=False):
    """patches_host: ctypes array of mc_patch; patches_dev: device buffer (tensor) of at least
    n * sizeof(mc_patch) = n * 88 bytes"""
    if hasattr(patches_host, "__len__") and len(patches_host) < n:
        raise ManyclawError("mc_step2d_patches", MC_EINVAL, "fewer host descriptors than n")
    _check_pools("mc_step2d_patches", ctx, patches_host, n, (pool0, pool1))
    _arg("mc_step2d_patches", patches_dev, max(int(n), 0) * ctypes.sizeof(mc_patch))
    return _check("mc_step2d_patches", lib().mc_step2d_patches(
        ctx, ctypes.cast(patches_host, _VP), _ptr(patches_dev), n, _ptr(pool0), _ptr(pool1), nsteps,
        limiter, 1 if use_graph else 0))


def mc_step2d_patches_noalloc(ctx, patches_host, patches_dev, n, pool0, pool1, nsteps, limiter):
    """mc_step2d_patches without device allocation (the schedule goes into the library's
    static device array); same arguments and checks, no graph"""
    fn = "mc_step2d_patches_noalloc"
    if hasattr(patches_host, "__len__") and len(patches_host) < n:
        raise ManyclawError(fn, MC_EINVAL, "fewer host descriptors than n")
    _check_pools(fn, ctx, patches_host, n, (pool0, pool1))
    _arg(fn, patches_dev, max(int(n), 0) * ctypes.sizeof(mc_patch))
    return _check(fn, lib().mc_step2d_patches_noalloc(
        ctx, ctypes.cast(patches_host, _VP), _ptr(patches_dev), n, _ptr(pool0), _ptr(pool1), nsteps,
        limiter))


def mc_patches_tune(ctx, patches_host, n, limiter):
    rows = (ctypes.c_int32 * 4)()
    _check("mc_patches_tune", lib().mc_patches_tune(ctx, ctypes.cast(patches_host, _VP), n, limiter, rows))
    return list(rows)


def mc_patches_set_rows(ctx, patches_host, n, rows):
    r = (ctypes.c_int32 * 4)(*rows)
    return _check("mc_patches_set_rows", lib().mc_patches_set_rows(ctx, ctypes.cast(patches_host, _VP), n, r))


def mc_status_get(ctx):
    v = ctypes.c_int32()
    _check("mc_status_get", lib().mc_status_get(ctx, ctypes.byref(v)))
    return v.value


def state(q0, q1, cur=0):
    s = mc_state()
    s.q[0] = _ptr(q0)
    s.q[1] = _ptr(q1)
    s.cur = cur
    s.bufs = (q0, q1)  # for the binding's checks (and kept alive with the state)
    return s


def clock_from_tensor(t):
    """interpret a device tensor (uint8, at least sizeof(mc_clock) = 72
    bytes) as an mc_clock on the host"""
    raw = bytes(t.cpu().numpy().tobytes())
    return mc_clock.from_buffer_copy(raw)


def cfl_from_tensor(t):
    raw = bytes(t.cpu().numpy().tobytes())
    return mc_cfl.from_buffer_copy(raw)


# ------------------------------------------------------------ surrogate
def mc_sur_dims(model):
    """(nparams, nin, nout, ystride) of MC_SW_SURROGATE or MC_EULER_SURROGATE"""
    v = [ctypes.c_int32(0) for _ in range(4)]
    _check("mc_sur_dims", lib().mc_sur_dims(model, *[ctypes.byref(x) for x in v]))
    return tuple(x.value for x in v)


_SUR = {}   # network handle -> its model, for the buffer checks


def _sur_dims(sur):
    """(nparams, nin, nout, ystride) of a handle's model, or None if unknown"""
    model = _SUR.get(getattr(sur, "value", None))
    if model == MC_EULER_SURROGATE:
        return MC_SUR_EU_NPARAMS, MC_SUR_EU_NIN, MC_SUR_EU_NOUT, 16
    if model == MC_SW_SURROGATE:
        return MC_SUR_NPARAMS, MC_SUR_NIN, MC_SUR_NOUT, 8
    return None


def _check_rows(fn, sur, n, X=None, Y=None, out=None):
    """X [n][8], Y and out [n][ystride], FP32"""
    d = _sur_dims(sur)
    ys = d[3] if d else 0
    n = max(int(n), 0)
    _arg(fn, X, n * 8 * 4, "float32")
    _arg(fn, Y, n * ys * 4, "float32")
    _arg(fn, out, n * ys * 4, "float32")


def mc_sur_create(max_batch, model=MC_SW_SURROGATE, stream=None):
    h = _VP()
    _check("mc_sur_create", lib().mc_sur_create(ctypes.byref(h), model, max_batch,
                                                _stream_handle(stream)))
    _SUR[h.value] = model
    return h


def mc_sur_destroy(sur):
    _SUR.pop(getattr(sur, "value", sur), None)
    lib().mc_sur_destroy(sur)


def _nparams(sur):
    d = _sur_dims(sur)
    return d[0] if d else 0


def mc_sur_set_params(sur, params):
    _arg("mc_sur_set_params", params, _nparams(sur) * 4, "float32")
    return _check("mc_sur_set_params", lib().mc_sur_set_params(sur, _ptr(params)))


def mc_sur_get_params(sur, params):
    _arg("mc_sur_get_params", params, _nparams(sur) * 4, "float32")
    return _check("mc_sur_get_params", lib().mc_sur_get_params(sur, _ptr(params)))


def mc_sur_init_params(sur, uniforms):
    _arg("mc_sur_init_params", uniforms, _nparams(sur) * 8, "float64")
    return _check("mc_sur_init_params", lib().mc_sur_init_params(sur, _ptr(uniforms)))


def mc_sur_gen(sur, prm, n, uniforms, X, Y, keep):
    """prm: an mc_params (g for shallow water, gamma for Euler) or a number,
    taken as g"""
    if not isinstance(prm, mc_params):
        prm = params(g=float(prm))
    nu = 8 if _SUR.get(getattr(sur, "value", None)) == MC_EULER_SURROGATE else 6
    _arg("mc_sur_gen", uniforms, nu * max(int(n), 0) * 8, "float64")
    _check_rows("mc_sur_gen", sur, n, X, Y)
    _arg("mc_sur_gen", keep, max(int(n), 0) * 4, "int32")
    return _check("mc_sur_gen", lib().mc_sur_gen(sur, ctypes.byref(prm), n, _ptr(uniforms), _ptr(X),
                                                 _ptr(Y), _ptr(keep)))


def mc_sur_compact(sur, n, X, Y, keep, Xc, Yc):
    _check_rows("mc_sur_compact", sur, n, X, Y)
    _check_rows("mc_sur_compact", sur, n, Xc, Yc)
    _arg("mc_sur_compact", keep, max(int(n), 0) * 4, "int32")
    k = ctypes.c_int64(0)
    _check("mc_sur_compact", lib().mc_sur_compact(sur, n, _ptr(X), _ptr(Y), _ptr(keep), _ptr(Xc),
                                                  _ptr(Yc), ctypes.byref(k)))
    return k.value


def mc_sur_forward(sur, n, X, out):
    _check_rows("mc_sur_forward", sur, n, X, out=out)
    return _check("mc_sur_forward", lib().mc_sur_forward(sur, n, _ptr(X), _ptr(out)))


def mc_sur_loss_grad(sur, n, X, Y, grad=None, loss=None):
    _check_rows("mc_sur_loss_grad", sur, n, X, Y)
    _arg("mc_sur_loss_grad", grad, _nparams(sur) * 4, "float32")
    _arg("mc_sur_loss_grad", loss, 4, "float32")
    return _check("mc_sur_loss_grad", lib().mc_sur_loss_grad(sur, n, _ptr(X), _ptr(Y), _ptr(grad),
                                                             _ptr(loss)))


def mc_sur_adam(sur, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    return _check("mc_sur_adam", lib().mc_sur_adam(sur, lr, beta1, beta2, eps))


def mc_sur_train(sur, n, X, Y, batch, epochs, lr0, order):
    """order: sequence of epochs * (n // batch) batch indices; returns the
    per-epoch mean batch losses"""
    _check_rows("mc_sur_train", sur, n, X, Y)
    nb = n // batch
    if len(order) != epochs * nb:
        raise ValueError("order must hold epochs * (n // batch) batch indices")
    o = (ctypes.c_int32 * max(len(order), 1))(*[int(v) for v in order])
    losses = (ctypes.c_float * max(epochs, 1))()
    _check("mc_sur_train", lib().mc_sur_train(sur, n, _ptr(X), _ptr(Y), batch, epochs, lr0, o, losses))
    return list(losses)[:epochs]


def mc_sur_eval(sur, n, X, Y):
    _check_rows("mc_sur_eval", sur, n, X, Y)
    v = ctypes.c_double(0.0)
    _check("mc_sur_eval", lib().mc_sur_eval(sur, n, _ptr(X), _ptr(Y), ctypes.byref(v)))
    return v.value


def mc_ctx_set_surrogate(ctx, sur):
    return _check("mc_ctx_set_surrogate", lib().mc_ctx_set_surrogate(ctx, sur))


def mc_sur_edge_stats(ctx):
    e, f = ctypes.c_int64(0), ctypes.c_int64(0)
    _check("mc_sur_edge_stats", lib().mc_sur_edge_stats(ctx, ctypes.byref(e), ctypes.byref(f)))
    return e.value, f.value


# ------------------------------------------------------------ refinement
class mc_amr_box(ctypes.Structure):
    _fields_ = [("ci0", ctypes.c_int32), ("cj0", ctypes.c_int32), ("cw", ctypes.c_int32),
                ("ch", ctypes.c_int32)]


def mc_amr_create(ctx, ratio, boxes, bc):
    """boxes: sequence of (ci0, cj0, cw, ch) coarse-cell footprints"""
    n = len(boxes)
    arr = (mc_amr_box * max(n, 1))(*[mc_amr_box(*[int(v) for v in b]) for b in boxes])
    h = _VP()
    _check("mc_amr_create", lib().mc_amr_create(ctypes.byref(h), ctx, ratio, n, arr, bc))
    _AMR[h.value] = _CTX.get(getattr(ctx, "value", None))
    return h


_AMR = {}   # hierarchy -> its context's (solver, dtype, nx, ny), for size checks


def mc_amr_destroy(amr):
    _AMR.pop(getattr(amr, "value", amr), None)
    lib().mc_amr_destroy(amr)


def _check_amr_grid(fn, amr, which, q):
    """q must hold meqn * nx * ny elements of grid `which`"""
    info = _AMR.get(getattr(amr, "value", None))
    if info is None or info[0] not in _MEQN or _nbytes(q) is None:
        _arg(fn, q)
        return
    nx, ny = mc_amr_dims(amr, which)
    _arg(fn, q, _MEQN[info[0]] * nx * ny * (8 if info[1] == MC_F64 else 4), _dtname(info[1]))


def mc_amr_dims(amr, which):
    nx, ny = ctypes.c_int32(0), ctypes.c_int32(0)
    _check("mc_amr_dims", lib().mc_amr_dims(amr, which, ctypes.byref(nx), ctypes.byref(ny)))
    return nx.value, ny.value


def mc_amr_set(amr, which, q):
    _check_amr_grid("mc_amr_set", amr, which, q)
    return _check("mc_amr_set", lib().mc_amr_set(amr, which, _ptr(q)))


def mc_amr_get(amr, which, q):
    _check_amr_grid("mc_amr_get", amr, which, q)
    return _check("mc_amr_get", lib().mc_amr_get(amr, which, _ptr(q)))


def mc_amr_step(amr, dt, limiter, cfl=None):
    return _check("mc_amr_step", lib().mc_amr_step(amr, dt, limiter, _ptr(cfl)))
