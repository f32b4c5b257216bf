"""Helpers for the GPU tests: device arrays via torch, contexts via the C ABI."""
import contextlib

import numpy as np

from paper_1308_1464_amd import manyclaw as mc


def torch():
    import torch as _t
    return _t


def dev(a, dtype=np.float64):
    t = torch()
    arr = np.ascontiguousarray(np.asarray(a, dtype=dtype))
    return t.from_numpy(arr).to("cuda")


def empty(shape, dtype=np.float64):
    t = torch()
    td = t.float64 if dtype == np.float64 else t.float32
    return t.empty(tuple(shape), dtype=td, device="cuda")


def host(t):
    torch().cuda.synchronize()
    return t.detach().cpu().numpy()


def struct_buf(nbytes):
    t = torch()
    return t.zeros(nbytes, dtype=t.uint8, device="cuda")


@contextlib.contextmanager
def context(solver, dtype, prm, nx, ny, dx, dy):
    h = mc.mc_ctx_create(solver, dtype, prm, nx, ny, dx, dy)
    try:
        yield h
    finally:
        torch().cuda.synchronize()
        mc.mc_ctx_destroy(h)


def npdt(dtype):
    return np.float64 if dtype == mc.MC_F64 else np.float32


def run_steps(solver, dtype, prm, q0, dx, dy, dts, limiter, bc, rows=None, aux=None):
    """Host-dt steps through mc_step2d; returns (q_final, list of smax)."""
    m, ny, nx = q0.shape
    T = npdt(dtype)
    a = dev(q0, T)
    b = empty(q0.shape, T)
    auxd = dev(aux, T) if aux is not None else None
    out = struct_buf(16)
    smaxes = []
    with context(solver, dtype, prm, nx, ny, dx, dy) as h:
        if rows is not None:
            mc.mc_ctx_set_tile(h, rows)
        st = mc.state(a, b)
        for dt in dts:
            mc.mc_step2d(h, st, auxd, float(dt), limiter, bc, out)
            smaxes.append(mc.cfl_from_tensor(out).smax)
        res = host(a if st.cur == 0 else b)
        status = mc.mc_status_get(h)
    return res, smaxes, status


def rel_inf(a, b):
    """per-field max-norm error relative to the field's max norm"""
    out = []
    for m in range(b.shape[0]):
        den = np.abs(b[m]).max()
        out.append(np.abs(a[m] - b[m]).max() / (den if den > 0 else 1.0))
    return np.array(out)


def rel_l1(a, b):
    out = []
    for m in range(b.shape[0]):
        den = np.abs(b[m]).sum()
        out.append(np.abs(a[m] - b[m]).sum() / (den if den > 0 else 1.0))
    return np.array(out)


def pack_patches(plist, dtype=np.float64, align=64, bc=1, cur=0):
    from paper_1308_1464_amd import patchset
    return patchset.pack(plist, dtype=dtype, align=align, bc=bc)


def patches_to_dev(host_arr):
    from paper_1308_1464_amd import patchset
    return torch().from_numpy(patchset.descriptors_bytes(host_arr)).to("cuda")


def patches_from_dev(dev_buf, n):
    from paper_1308_1464_amd import patchset
    return patchset.descriptors_from_bytes(host(dev_buf), n)


def unpack_patch(pool0, pool1, desc, dtype=np.float64, meqn=3):
    from paper_1308_1464_amd import patchset
    return patchset.unpack(pool0, pool1, desc, meqn).astype(np.float64)
