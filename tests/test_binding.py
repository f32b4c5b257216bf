"""Host-side argument checks of the Python binding (no GPU).

The C ABI receives bare device addresses, so the binding checks what only it
can see before an address crosses: that a tensor lives on the GPU (a host
address handed to a kernel faults the device), is contiguous, holds the
context's element type, and is large enough.  A CPU tensor stands in for a
device tensor through `OnGpu`, which reports device type "cuda" and nothing
else differs; the checks read only the device, dtype, contiguity and size."""
import ctypes
import types

import pytest
import torch

from paper_1308_1464_amd import inputs
from paper_1308_1464_amd import manyclaw as mc
from paper_1308_1464_amd import patchset


class OnGpu:
    """a CPU tensor presented to the binding's checks as a GPU tensor"""
    device = types.SimpleNamespace(type="cuda")

    def __init__(self, t):
        self.t = t

    @property
    def dtype(self):
        return self.t.dtype

    def is_contiguous(self):
        return self.t.is_contiguous()

    def numel(self):
        return self.t.numel()

    def element_size(self):
        return self.t.element_size()

    def data_ptr(self):
        return self.t.data_ptr()


def g(shape, dtype=torch.float64):
    return OnGpu(torch.zeros(shape, dtype=dtype))


def fake_ctx(key, *info):
    mc._CTX[key] = info
    return types.SimpleNamespace(value=key)


@pytest.fixture
def ctxs():
    keys = []

    def make(key, *info):
        keys.append(key)
        return fake_ctx(key, *info)
    yield make
    for k in keys:
        mc._CTX.pop(k, None)


def test_patch_pools_sized_for_the_solver(ctxs):
    plist = inputs.patch_set(4, seed=2)
    hp, pool, offs = patchset.pack(plist)
    need3 = max(o + 3 * nx * ny for o, (nx, ny, _) in zip(offs, plist))
    sw = ctxs(101, mc.MC_SW_ROE, mc.MC_F64)
    eu = ctxs(102, mc.MC_EULER_ROE, mc.MC_F64)
    f32 = ctxs(103, mc.MC_SW_ROE, mc.MC_F32)
    ok = g(need3)
    mc._check_pools("f", sw, hp, len(plist), (ok, ok))           # exactly large enough
    with pytest.raises(mc.ManyclawError):                         # one element short
        mc._check_pools("f", sw, hp, len(plist), (ok, g(need3 - 1)))
    with pytest.raises(mc.ManyclawError):                         # four fields needed
        mc._check_pools("f", eu, hp, len(plist), (ok, ok))
    mc._check_pools("f", f32, hp, len(plist), (g(need3, torch.float32),) * 2)
    with pytest.raises(mc.ManyclawError):                         # FP64 pool, FP32 context
        mc._check_pools("f", f32, hp, len(plist), (ok, ok))
    with pytest.raises(mc.ManyclawError):                         # a host tensor
        mc._check_pools("f", sw, hp, len(plist), (ok, torch.zeros(need3, dtype=torch.float64)))
    mc._check_pools("f", sw, hp, len(plist), (12345, 67890))      # raw addresses pass through


def test_grid_buffers_sized_for_the_context(ctxs):
    sw = ctxs(201, mc.MC_SW_ROE, mc.MC_F64, 10, 7)
    vc = ctxs(202, mc.MC_ACOUSTICS_VC, mc.MC_F32, 10, 7)
    good, short = g((3, 7, 10)), g((3, 7, 9))
    mc._check_grid("f", sw, mc.state(good, good).bufs)
    with pytest.raises(mc.ManyclawError):
        mc._check_grid("f", sw, mc.state(good, short).bufs)
    q32 = g((3, 7, 10), torch.float32)
    mc._check_grid("f", vc, (q32,), g((2, 7, 10), torch.float32))
    with pytest.raises(mc.ManyclawError):      # aux needs two fields
        mc._check_grid("f", vc, (q32,), g((1, 7, 10), torch.float32))
    with pytest.raises(mc.ManyclawError):      # an FP32 buffer in an FP64 context
        mc._check_grid("f", sw, (g((3, 7, 20), torch.float32),))
    mc._check_grid("f", sw, (None, None))      # raw addresses pass through


def test_host_tensors_refused_before_the_call(ctxs):
    """every entry point that takes device buffers refuses a CPU tensor
    before the library is called"""
    sw = ctxs(301, mc.MC_SW_ROE, mc.MC_F64, 10, 7)
    host = torch.zeros((3, 7, 10), dtype=torch.float64)
    dev = g((3, 7, 10))
    cfl = g(16, torch.uint8)
    with pytest.raises(mc.ManyclawError, match="not on the GPU"):
        mc.mc_step2d(sw, mc.state(dev, host), None, 1e-3, mc.MC_LIM_MC, mc.MC_BC_EXTRAP, cfl)
    with pytest.raises(mc.ManyclawError, match="not on the GPU"):
        mc.mc_step2d_strang(sw, mc.state(host, dev), None, 1e-3, mc.MC_LIM_MC, mc.MC_BC_EXTRAP)
    with pytest.raises(mc.ManyclawError, match="not on the GPU"):
        mc.mc_step2d_unsplit(sw, mc.state(dev, dev), None, 1e-3, mc.MC_LIM_MC, mc.MC_BC_EXTRAP,
                             torch.zeros(16, dtype=torch.uint8))
    with pytest.raises(mc.ManyclawError, match="not on the GPU"):
        mc.mc_max_speed(sw, host, None, mc.MC_BC_EXTRAP, cfl)
    with pytest.raises(mc.ManyclawError, match="not on the GPU"):
        mc.mc_clock_init(sw, torch.zeros(72, dtype=torch.uint8), dev, None, mc.MC_BC_EXTRAP)
    with pytest.raises(mc.ManyclawError, match="not on the GPU"):
        mc.mc_run2d(sw, dev, host, None, g(72, torch.uint8), 1, mc.MC_LIM_MC, mc.MC_BC_EXTRAP)
    n = 5
    with pytest.raises(mc.ManyclawError, match="not on the GPU"):
        mc.mc_rp2(sw, 1, n, torch.zeros((3, n), dtype=torch.float64), g((3, n)), None, g((3, 3, n)),
                  g((3, n)), g((3, n)), g((3, n)))
    with pytest.raises(mc.ManyclawError, match="not on the GPU"):
        mc.mc_copy_probe(sw, g(64, torch.uint8), torch.zeros(64, dtype=torch.uint8), 64)


def test_noncontiguous_and_wrong_dtype_refused(ctxs):
    sw = ctxs(401, mc.MC_SW_ROE, mc.MC_F64, 10, 7)
    f32 = ctxs(402, mc.MC_SW_ROE, mc.MC_F32, 10, 7)
    big = torch.zeros((3, 10, 7), dtype=torch.float64)
    view = OnGpu(big.transpose(1, 2))          # (3, 7, 10), not contiguous
    with pytest.raises(mc.ManyclawError, match="not contiguous"):
        mc._check_grid("f", sw, (view,))
    with pytest.raises(mc.ManyclawError, match="expected torch.float32"):
        mc.mc_step2d(f32, mc.state(g((3, 7, 10)), g((3, 7, 10))), None, 1e-3, mc.MC_LIM_MC,
                     mc.MC_BC_EXTRAP)
    n = 4
    with pytest.raises(mc.ManyclawError, match="expected torch.float64"):
        mc.mc_rp2(sw, 1, n, g((3, n)), g((3, n), torch.float32), None, g((3, 3, n)), g((3, n)),
                  g((3, n)), g((3, n)))
    with pytest.raises(mc.ManyclawError, match="needs"):      # waves hold mwaves * meqn * n
        mc.mc_rp2(sw, 1, n, g((3, n)), g((3, n)), None, g((3, 2, n)), g((3, n)), g((3, n)), g((3, n)))
    with pytest.raises(mc.ManyclawError, match="needs"):      # cfl_out holds 16 bytes
        mc.mc_step2d(sw, mc.state(g((3, 7, 10)), g((3, 7, 10))), None, 1e-3, mc.MC_LIM_MC,
                     mc.MC_BC_EXTRAP, g(8, torch.uint8))
    with pytest.raises(mc.ManyclawError, match="tensor or an int"):
        mc._arg("f", [1, 2, 3])


def test_patch_descriptors_sized_as_the_struct(ctxs):
    """the device descriptors hold n * sizeof(mc_patch) = n * 88 bytes"""
    assert ctypes.sizeof(mc.mc_patch) == 88
    plist = inputs.patch_set(3, seed=1)
    hp, pool, _ = patchset.pack(plist)
    sw = ctxs(501, mc.MC_SW_ROE, mc.MC_F64)
    p0, p1 = OnGpu(torch.from_numpy(pool)), g(pool.size)
    with pytest.raises(mc.ManyclawError, match="needs 264"):
        mc.mc_step2d_patches(sw, hp, g(3 * 80, torch.uint8), 3, p0, p1, 1, mc.MC_LIM_MC)
    with pytest.raises(mc.ManyclawError, match="not on the GPU"):
        mc.mc_step2d_patches(sw, hp, torch.zeros(264, dtype=torch.uint8), 3, p0, p1, 1, mc.MC_LIM_MC)
    with pytest.raises(mc.ManyclawError, match="fewer host descriptors"):
        mc.mc_step2d_patches(sw, hp, g(4 * 88, torch.uint8), 4, p0, p1, 1, mc.MC_LIM_MC)


def test_surrogate_buffers_checked():
    sur = types.SimpleNamespace(value=601)
    mc._SUR[601] = mc.MC_SW_SURROGATE
    try:
        n = 10
        X, out = g((n, 8), torch.float32), g((n, 8), torch.float32)
        mc._check_rows("f", sur, n, X, out=out)
        with pytest.raises(mc.ManyclawError, match="expected torch.float32"):
            mc._check_rows("f", sur, n, g((n, 8)), out=out)
        with pytest.raises(mc.ManyclawError, match="needs"):
            mc._check_rows("f", sur, n, g((n, 6), torch.float32), out=out)
        with pytest.raises(mc.ManyclawError, match="needs"):
            mc.mc_sur_set_params(sur, g(mc.MC_SUR_NPARAMS - 1, torch.float32))
        with pytest.raises(mc.ManyclawError, match="expected torch.float64"):
            mc.mc_sur_init_params(sur, g(mc.MC_SUR_NPARAMS, torch.float32))
        with pytest.raises(mc.ManyclawError, match="expected torch.int32"):
            mc.mc_sur_gen(sur, 9.81, n, g((6, n)), X, g((n, 8), torch.float32), g(n, torch.int64))
        mc._SUR[601] = mc.MC_EULER_SURROGATE        # Euler rows are 16 floats wide
        with pytest.raises(mc.ManyclawError, match="needs"):
            mc._check_rows("f", sur, n, X, out=out)
    finally:
        mc._SUR.pop(601, None)
