"""Packing of a patch batch into the two pools and the descriptor array
that mc_step2d_patches takes (layout only; no arithmetic of the method)."""
import numpy as np

from . import manyclaw as mc


def pack(plist, dtype=np.float64, align=64, bc=mc.MC_BC_EXTRAP):
    """plist: list of (nx, ny, q[meqn][ny][nx]) on the unit square (one meqn
    for the whole batch).  Returns (host mc_patch array, pool numpy array,
    offsets); each patch's fields are contiguous [meqn][ny][nx] starting at
    a multiple of `align` elements."""
    offs = []
    o = 0
    for nx, ny, q in plist:
        offs.append(o)
        o += np.shape(q)[0] * nx * ny
        o = (o + align - 1) // align * align
    pool = np.zeros(max(o, 1), dtype=dtype)
    descs = []
    for (nx, ny, q), off in zip(plist, offs):
        pool[off:off + np.shape(q)[0] * nx * ny] = np.asarray(q, dtype=dtype).ravel()
        descs.append(dict(nx=nx, ny=ny, offset=off, dx=1.0 / nx, dy=1.0 / ny, t=0.0, dt=-1.0,
                          cfl=0.0, smax=0.0, bc=bc, status=0, n_acc=0, n_rej=0, cur=0))
    return mc.patch_array(descs), pool, offs


def descriptors_bytes(host_arr):
    return np.frombuffer(bytes(host_arr), dtype=np.uint8).copy()


def descriptors_from_bytes(raw, n):
    return (mc.mc_patch * n).from_buffer_copy(bytes(raw))


def unpack(pool0, pool1, desc, meqn=3):
    """current state [meqn][ny][nx] of one patch from the two host pools"""
    src = pool1 if desc.cur else pool0
    n = meqn * desc.nx * desc.ny
    return src[desc.offset:desc.offset + n].reshape(meqn, desc.ny, desc.nx)


def edges_per_step(plist):
    """counted edges of one step of every patch: (nx+1) ny + nx (ny+1)"""
    return sum((nx + 1) * ny + nx * (ny + 1) for nx, ny, _ in plist)
