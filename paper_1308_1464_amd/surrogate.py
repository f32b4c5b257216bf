"""Training driver of the learned edge solvers (shallow water, Euler).

Marshalling only: device buffers come from torch, random draws from
``inputs``, and every step (pair generation, compaction, initialisation,
forward, backward, Adam, evaluation) is a call into libmanyclaw.so
(``mc_sur_*``).  Recipe (defaults): 2^24 pairs; shallow water h
log-uniform in [1e-3, 10], u, v uniform in [-5, 5]; Euler rho and p
log-uniform in [0.05, 10], u, v uniform in [-2, 2], gamma 1.4; the pairs the
loss keeps are compacted; batches of 8192, 20 epochs, Adam with a
cosine-decayed step size from 2e-3; a held-out set of 2^20 pairs from
another seed gives the validation loss.
"""
import time

from . import inputs
from . import manyclaw as mc

G = 9.81
GAMMA = 1.4


def _torch():
    import torch
    return torch


def _uniforms(model, n, seed):
    if model == mc.MC_EULER_SURROGATE:
        return inputs.euler_surrogate_uniforms(n, seed)
    return inputs.surrogate_uniforms(n, seed)


def _params(model, g, gamma):
    return mc.params(g=g, gamma=gamma)


def make_pairs(sur, n, seed, g=G, model=mc.MC_SW_SURROGATE, gamma=GAMMA):
    """Kept training pairs (Xc, Yc, n_kept) of n draws; tensors on cuda."""
    t = _torch()
    ys = mc.mc_sur_dims(model)[3]
    U = t.from_numpy(_uniforms(model, n, seed)).to("cuda")
    X = t.empty((n, 8), dtype=t.float32, device="cuda")
    Y = t.empty((n, ys), dtype=t.float32, device="cuda")
    keep = t.empty(n, dtype=t.int32, device="cuda")
    mc.mc_sur_gen(sur, _params(model, g, gamma), n, U, X, Y, keep)
    Xc = t.empty_like(X)
    Yc = t.empty_like(Y)
    nk = mc.mc_sur_compact(sur, n, X, Y, keep, Xc, Yc)
    del U, X, Y, keep
    return Xc[:nk], Yc[:nk], nk


def init(sur, seed, model=mc.MC_SW_SURROGATE):
    t = _torch()
    U = t.from_numpy(inputs.param_uniforms(mc.mc_sur_dims(model)[0], seed)).to("cuda")
    mc.mc_sur_init_params(sur, U)
    t.cuda.synchronize()


def train(seed=0, n_pairs=1 << 24, epochs=20, batch=8192, lr0=2e-3, n_val=1 << 20, g=G,
          log=None, model=mc.MC_SW_SURROGATE, gamma=GAMMA):
    """Trains a network of the given model on the GPU; returns (handle,
    info).  The caller owns the handle (mc_sur_destroy)."""
    t = _torch()
    sur = mc.mc_sur_create(batch, model)
    t0 = time.perf_counter()
    Xc, Yc, nk = make_pairs(sur, n_pairs, seed, g, model, gamma)
    init(sur, seed + 1, model)
    nb = nk // batch
    order = inputs.batch_orders(epochs, nb, seed + 2)
    t1 = time.perf_counter()
    losses = mc.mc_sur_train(sur, nk, Xc, Yc, batch, epochs, lr0, order)
    t.cuda.synchronize()
    t2 = time.perf_counter()
    Xv, Yv, nv = make_pairs(sur, n_val, seed + 100, g, model, gamma)
    val = mc.mc_sur_eval(sur, nv, Xv, Yv)
    info = {"model": "euler" if model == mc.MC_EULER_SURROGATE else "shallow_water",
            "n_pairs": n_pairs, "n_kept": nk, "epochs": epochs, "batch": batch, "lr0": lr0,
            "train_loss": losses, "val_loss": val, "val_kept": nv,
            "gen_seconds": t1 - t0, "train_seconds": t2 - t1}
    if log:
        log(info)
    return sur, info
