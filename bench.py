"""Benchmark of the fused 2D wave-propagation step on one MI355X.

Workload: shallow water (g = 9.81), Roe solver with the Harten-Hyman entropy
fix, MC limiter, zero-order extrapolation boundaries, 4096 x 4096 cells on
the unit square, radial dam break (h = 2 inside r < 0.3, 1 outside) plus
seeded uniform noise of amplitude 1e-3 on h, zero momentum; CFL 0.9 with the
variable time-step rule applied on the device.  A step is one dimensionally
split step (Riemann solves, limiter, correction flux, update and CFL
reduction) over the whole grid; the timed steps are replayed as one captured
HIP graph with the state resident in HBM.

Prints one JSON line.  Throughput is cell-edge Riemann updates per second:
2 (n + 1) n edges per step of an n x n grid.
"""
import argparse
import ctypes
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "cell-edge Riemann updates/s + HBM GB/s; surrogate vs Roe at L1<=1e-3"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def run_gpu(n, dtype_name, steps, warmup, rows, seed=0, problem="sw", reps=1):
    """Time `steps` graph-replayed steps of the device dt rule on an n x n grid,
    MC limiter.  The first timed replay gives the result; with reps > 1 the
    same graph is replayed and timed reps - 1 more times (the run goes on from
    where it stands) and every replay's time per step is returned as well.  problem "sw": shallow-water dam break (CFL 0.9, extrapolation
    boundaries); "euler": four-quadrant Euler problem (CFL 0.8, extrapolation);
    "advection": the Gaussian pulse advected with velocity (1, 0.5); "acoustics":
    the pressure pulse, rho = K = 1; "acoustics_vc": the pulse in the layered
    medium (aux rho, c per cell); the last three CFL 0.9, periodic."""
    import torch

    from paper_1308_1464_amd import inputs
    from paper_1308_1464_amd import manyclaw as mc

    dtype = mc.MC_F64 if dtype_name == "f64" else mc.MC_F32
    tdt = torch.float64 if dtype == mc.MC_F64 else torch.float32
    aux, bc = None, mc.MC_BC_EXTRAP
    if problem == "sw":
        q0 = inputs.sw_dam_break(n, seed=seed)
        solver, cfl, meqn = mc.MC_SW_ROE, 0.9, 3
    elif problem == "euler":
        q0, _ = inputs.euler_quadrants(n, seed=seed)
        solver, cfl, meqn = mc.MC_EULER_ROE, 0.8, 4
    elif problem == "advection":
        q0 = inputs.acoustics_pulse(n)[:1]
        solver, cfl, meqn, bc = mc.MC_ADVECTION, 0.9, 1, mc.MC_BC_PERIODIC
    elif problem == "acoustics":
        q0 = inputs.acoustics_pulse(n)
        solver, cfl, meqn, bc = mc.MC_ACOUSTICS, 0.9, 3, mc.MC_BC_PERIODIC
    elif problem == "acoustics_vc":
        q0 = inputs.acoustics_pulse(n)
        aux = torch.from_numpy(inputs.layered_medium(n)).to("cuda", tdt)
        solver, cfl, meqn, bc = mc.MC_ACOUSTICS_VC, 0.9, 3, mc.MC_BC_PERIODIC
    else:
        raise ValueError(problem)
    maux = 0 if aux is None else aux.shape[0]
    a = torch.from_numpy(q0).to("cuda", tdt)
    b = torch.empty_like(a)
    clk = torch.zeros(ctypes.sizeof(mc.mc_clock), dtype=torch.uint8, device="cuda")
    prm = mc.params(g=9.81, gamma=1.4, rho=1.0, K=1.0, u=1.0, v=0.5, cfl_target=cfl, cfl_max=1.0)
    h = mc.mc_ctx_create(solver, dtype, prm, n, n, 1.0 / n, 1.0 / n)
    try:
        mc.mc_clock_init(h, clk, a, aux, bc)
        if rows:
            mc.mc_ctx_set_tile(h, rows)
            rows_used = rows
        else:
            # rows per work item timed on this machine (setup, outside the timed
            # region; it writes only the state's other buffer)
            dt0 = mc.clock_from_tensor(clk).dt
            rows_used = mc.mc_tune_rows(h, mc.state(a, b), aux, dt0, mc.MC_LIM_MC, bc)
        if warmup > 0:
            mc.mc_run2d(h, a, b, aux, clk, warmup, mc.MC_LIM_MC, bc, False)
        # capture the K-step graph (first call records and runs it)
        mc.mc_run2d(h, a, b, aux, clk, steps, mc.MC_LIM_MC, bc, True)
        torch.cuda.synchronize()
        c0 = mc.clock_from_tensor(clk)
        stream = torch.cuda.current_stream()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        mc.mc_run2d(h, a, b, aux, clk, steps, mc.MC_LIM_MC, bc, True)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        c1 = mc.clock_from_tensor(clk)
        status = mc.mc_status_get(h)
        qf = (a if c1.cur == 0 else b)
        first_min = float(qf[0].min().item())
        rep_ms = [ms / steps]
        for _ in range(reps - 1):
            torch.cuda.synchronize()
            e0.record(stream)
            mc.mc_run2d(h, a, b, aux, clk, steps, mc.MC_LIM_MC, bc, True)
            e1.record(stream)
            torch.cuda.synchronize()
            rep_ms.append(e0.elapsed_time(e1) / steps)
    finally:
        torch.cuda.synchronize()
        mc.mc_ctx_destroy(h)
    acc = c1.n_acc - c0.n_acc
    rej = c1.n_rej - c0.n_rej
    edges = 2.0 * (n + 1) * n
    esize = 8 if dtype == mc.MC_F64 else 4
    bytes_launch = (2.0 * meqn + maux) * esize * n * n  # read q^n and aux, write q^{n+1}
    per_launch_s = ms * 1e-3 / steps
    return {
        "ms_total": ms, "ms_per_step": ms / steps, "accepted": acc, "rejected": rej,
        "edge_updates_per_s": edges * acc / (ms * 1e-3),
        "bytes_per_launch": bytes_launch,
        "achieved_gbs": bytes_launch / per_launch_s / 1e9,
        "status": status, "first_field_min": first_min, "t": c1.t, "dt": c1.dt,
        "rep_ms_per_step": rep_ms, "rows": rows_used,
    }


def run_paper_kernels(n=2048, steps=50, warmup=5):
    """Advection, constant- and variable-coefficient acoustics and Euler (the
    paper's four kernels) on its 2048 x 2048 grid."""
    out = {}
    for p in ("advection", "acoustics", "acoustics_vc", "euler"):
        r = run_gpu(n, "f64", steps, warmup, 0, problem=p)
        out[p] = {"ms_per_step": r["ms_per_step"], "edge_updates_per_s": r["edge_updates_per_s"],
                  "bytes_per_launch": r["bytes_per_launch"], "achieved_gbs": r["achieved_gbs"],
                  "frac": r["achieved_gbs"] / HBM_PEAK_GBS, "accepted": r["accepted"],
                  "rejected": r["rejected"], "rows": r["rows"]}
        log(f"bench: {p} {out[p]}")
    return out


def run_patches(n_patches=2000, steps=20, seed=0):
    """2,000 dam-break patches (sides log-uniform in [16, 256]), FP64, each
    under its own dt, `steps` accepted steps in one persistent graph-captured
    launch with autotuned rows per chunk."""
    import numpy as np
    import torch

    from paper_1308_1464_amd import inputs, patchset
    from paper_1308_1464_amd import manyclaw as mc

    plist = inputs.patch_set(n_patches, seed=seed)
    hp, pool, _ = patchset.pack(plist)
    p0 = torch.from_numpy(pool).cuda()
    p1 = torch.zeros_like(p0)
    raw = torch.from_numpy(patchset.descriptors_bytes(hp)).cuda()
    dp = raw.clone()
    prm = mc.params(g=9.81, cfl_target=0.9, cfl_max=1.0)
    h = mc.mc_ctx_create(mc.MC_SW_ROE, mc.MC_F64, prm, 1, 1, 1.0, 1.0)
    try:
        rows = mc.mc_patches_tune(h, hp, n_patches, mc.MC_LIM_MC)
        # warm-up launch (captures the graph), then reset and time a fresh run
        mc.mc_step2d_patches(h, hp, dp, n_patches, p0, p1, steps, mc.MC_LIM_MC, True)
        torch.cuda.synchronize()
        dp.copy_(raw)
        p0.copy_(torch.from_numpy(pool).cuda())
        stream = torch.cuda.current_stream()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        mc.mc_step2d_patches(h, hp, dp, n_patches, p0, p1, steps, mc.MC_LIM_MC, True)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1)
        out = patchset.descriptors_from_bytes(dp.cpu().numpy(), n_patches)
    finally:
        torch.cuda.synchronize()
        mc.mc_ctx_destroy(h)
    acc = np.array([out[k].n_acc for k in range(n_patches)])
    rej = int(sum(out[k].n_rej for k in range(n_patches)))
    cells = sum(nx * ny for nx, ny, _ in plist)
    edges = patchset.edges_per_step(plist) * steps
    nbytes = 2.0 * 3 * 8 * cells * steps
    # a rejected attempt reads and writes its patch like an accepted step
    rej_bytes = float(sum(2.0 * 3 * 8 * out[k].nx * out[k].ny * out[k].n_rej for k in range(n_patches)))
    return {"n_patches": n_patches, "cells": cells, "steps": steps, "ms": ms,
            "edge_updates_per_s": edges / (ms * 1e-3), "achieved_gbs": nbytes / (ms * 1e-3) / 1e9,
            "frac": nbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "all_accepted": bool((acc == steps).all()),
            "rejected_total": rej, "bytes_accepted": nbytes, "bytes_rejected": rej_bytes,
            "attempt_gbs": (nbytes + rej_bytes) / (ms * 1e-3) / 1e9, "tuned_rows": rows,
            "tune_cache": os.environ.get("MANYCLAW_TUNE_CACHE") or None}


def profiled(key):
    """A figure from the committed rocprofv3 runs of the fused step at
    4096^2 (calibrated HBM bytes or VALU instructions per dispatch), or None
    when the kernel sources changed since they were taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "step_sw_roe_4096_traffic.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        line = line.strip()
        if line and not line.startswith("#") and "=" in line:
            k, v = line.split("=", 1)
            kv[k.strip()] = v.strip()
    h = hashlib.sha256()
    for f in ("paper_1308_1464_amd/csrc/step.hip", "paper_1308_1464_amd/csrc/solvers.hpp",
              "paper_1308_1464_amd/csrc/common.hpp"):
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    if kv.get("source_sha256") != h.hexdigest():
        return None
    v = kv.get(key)
    return float(v) if v else None


# vector ALU issue peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (lane-operations/s)
VALU_PEAK = 256 * 4 * 16 * 2.4e9


def copy_probe(nbytes=1 << 30, reps=5):
    """Achievable HBM copy bandwidth: mc_copy_probe of nbytes, best of reps
    (GB/s counts bytes read plus bytes written)."""
    import torch
    from paper_1308_1464_amd import manyclaw as mc
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda").fill_(1)
    dst = torch.empty_like(src)
    h = mc.mc_ctx_create(mc.MC_SW_ROE, mc.MC_F64, mc.params(), 8, 8, 1.0, 1.0)
    best = 0.0
    try:
        stream = torch.cuda.current_stream()
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            mc.mc_copy_probe(h, dst, src, nbytes)
            e1.record(stream)
            torch.cuda.synchronize()
            best = max(best, 2.0 * nbytes / (e0.elapsed_time(e1) * 1e-3) / 1e9)
    finally:
        torch.cuda.synchronize()
        mc.mc_ctx_destroy(h)
    return best


def cpu_baseline(n, seed=0, min_seconds=10.0, min_seconds_one=5.0):
    """The oracle as it stands, on the host cores, over whole steps of the
    same grid until at least min_seconds of work (at least one step); then
    on one thread for at least min_seconds_one."""
    import oracle
    from paper_1308_1464_amd import inputs
    hw = host_cores()
    threads = hw["threads_used"]
    q = inputs.sw_dam_break(n, seed=seed)
    P = oracle.params(g=9.81)
    sm, _ = oracle.max_speed(oracle.SW_ROE, P, q, 1.0 / n, 1.0 / n, oracle.BC_EXTRAP,
                             nthreads=threads)
    dt = 0.9 / sm
    t0 = time.perf_counter()
    k = 0
    while True:
        q, sm, _ = oracle.step2d(oracle.SW_ROE, P, q, 1.0 / n, 1.0 / n, dt, oracle.LIM_MC,
                                 oracle.BC_EXTRAP, nthreads=threads)
        dt = 0.9 / sm
        k += 1
        el = time.perf_counter() - t0
        if el >= min_seconds:
            break
    edges = 2.0 * (n + 1) * n * k
    out = {"value": edges / el, "unit": "edge updates/s", "cores": threads, "kind": "oracle",
           "sample": f"{k} full step(s) of the {n}x{n} dam break, FP64, {el:.1f} s"}
    # the same oracle on one thread, over a shorter sample (at least one step)
    q1 = inputs.sw_dam_break(n, seed=seed)
    sm, _ = oracle.max_speed(oracle.SW_ROE, P, q1, 1.0 / n, 1.0 / n, oracle.BC_EXTRAP, nthreads=1)
    dt = 0.9 / sm
    t0 = time.perf_counter()
    k1 = 0
    while True:
        q1, sm, _ = oracle.step2d(oracle.SW_ROE, P, q1, 1.0 / n, 1.0 / n, dt, oracle.LIM_MC,
                                  oracle.BC_EXTRAP, nthreads=1)
        dt = 0.9 / sm
        k1 += 1
        el1 = time.perf_counter() - t0
        if el1 >= min_seconds_one:
            break
    out["one_thread"] = {"value": 2.0 * (n + 1) * n * k1 / el1, "cores": 1,
                         "sample": f"{k1} full step(s), {el1:.1f} s"}
    out["cpu_model"] = hw["model"]
    out["host"] = hw
    return out


def host_cores():
    """What the host offers this process: nproc, the CPUs in its affinity
    mask, the lscpu model and topology, and the threads the oracle uses: every
    CPU in the mask, capped by OMP_NUM_THREADS when that is set (a GPU job's
    share of a shared host)."""
    import subprocess
    info = {"nproc": None, "affinity": None, "model": None, "sockets": None,
            "cores_per_socket": None, "threads_per_core": None}
    try:
        info["nproc"] = int(subprocess.run(["nproc"], capture_output=True, text=True).stdout.strip())
    except (OSError, ValueError):
        pass
    try:
        info["affinity"] = len(os.sched_getaffinity(0))
    except AttributeError:
        info["affinity"] = os.cpu_count()
    try:
        out = subprocess.run(["lscpu"], capture_output=True, text=True).stdout
        keys = {"Model name": "model", "Socket(s)": "sockets", "Core(s) per socket": "cores_per_socket",
                "Thread(s) per core": "threads_per_core"}
        for line in out.splitlines():
            k, _, v = line.partition(":")
            if k.strip() in keys:
                info[keys[k.strip()]] = v.strip()
    except OSError:
        pass
    if not info["model"]:
        try:
            with open("/proc/cpuinfo") as f:
                for line in f:
                    if line.startswith("model name"):
                        info["model"] = line.split(":", 1)[1].strip()
                        break
        except OSError:
            pass
    avail = info["affinity"] or info["nproc"] or 1
    cap = os.environ.get("OMP_NUM_THREADS", "")
    info["omp_num_threads"] = int(cap) if cap.isdigit() else None
    info["threads_used"] = max(1, min(avail, info["omp_num_threads"] or avail))
    return info


def run_surrogate(n=4096, steps=50, epochs=20, seed=0, timed=10, model="sw"):
    """Learned edge solver.  model "sw": shallow-water dam break at CFL 0.9;
    "euler": four-quadrant Euler problem (gamma 1.4) at CFL 0.8.  Reference:
    the plain FP64 Roe step of the same system on the same GPU (held to the
    FP64 oracle by the parity tests) for `steps` accepted steps, recording
    its dt sequence.  The network is trained on the GPU, then the surrogate
    runs the same dt sequence in FP32; reported: relative L1 against the
    reference and the time per step against plain FP32 Roe (both launched
    the same way, one step per call)."""
    import numpy as np
    import torch

    from paper_1308_1464_amd import inputs
    from paper_1308_1464_amd import manyclaw as mc
    from paper_1308_1464_amd import surrogate as sg

    g, gm = 9.81, 1.4
    eu = model == "euler"
    if eu:
        q0, _ = inputs.euler_quadrants(n, seed=seed, gamma=gm)
        plain, learned, cfl_t = mc.MC_EULER_ROE, mc.MC_EULER_SURROGATE, 0.8
    else:
        q0 = inputs.sw_dam_break(n, seed=seed)
        plain, learned, cfl_t = mc.MC_SW_ROE, mc.MC_SW_SURROGATE, 0.9
    prm = mc.params(g=g, gamma=gm)

    # reference run and its dt sequence (host-side rule: reject if cfl > 1)
    ctx = mc.mc_ctx_create(plain, mc.MC_F64, prm, n, n, 1.0 / n, 1.0 / n)
    a = torch.from_numpy(q0).to("cuda")
    b = torch.empty_like(a)
    cfl = torch.zeros(16, dtype=torch.uint8, device="cuda")
    mc.mc_max_speed(ctx, a, None, mc.MC_BC_EXTRAP, cfl)
    dt = cfl_t / mc.cfl_from_tensor(cfl).smax
    st = mc.state(a, b)
    dts = []
    while len(dts) < steps:
        mc.mc_step2d(ctx, st, None, dt, mc.MC_LIM_MC, mc.MC_BC_EXTRAP, cfl)
        sm = mc.cfl_from_tensor(cfl).smax
        if dt * sm > 1.0:
            st.cur ^= 1        # discard the attempt
        else:
            dts.append(dt)
        dt = cfl_t / sm
    torch.cuda.synchronize()
    qo = (a if st.cur == 0 else b).cpu().numpy()
    mc.mc_ctx_destroy(ctx)
    del a, b

    sur, info = sg.train(seed=seed, epochs=epochs, model=learned, g=g, gamma=gm)
    log(f"bench: {model} surrogate trained in {info['train_seconds']:.2f} s, "
        f"val loss {info['val_loss']:.3e}")

    def go(solver, net):
        ctx = mc.mc_ctx_create(solver, mc.MC_F32, prm, n, n, 1.0 / n, 1.0 / n)
        if net is not None:
            mc.mc_ctx_set_surrogate(ctx, net)
        a = torch.from_numpy(q0.astype(np.float32)).to("cuda")
        b = torch.empty_like(a)
        st = mc.state(a, b)
        for dt in dts:
            mc.mc_step2d(ctx, st, None, float(dt), mc.MC_LIM_MC, mc.MC_BC_EXTRAP)
        torch.cuda.synchronize()
        q = (a if st.cur == 0 else b).cpu().numpy().astype(np.float64)
        stats = mc.mc_sur_edge_stats(ctx) if net is not None else (0, 0)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(timed):
            mc.mc_step2d(ctx, st, None, float(dts[-1]), mc.MC_LIM_MC, mc.MC_BC_EXTRAP)
        e1.record()
        torch.cuda.synchronize()
        mc.mc_ctx_destroy(ctx)
        return q, e0.elapsed_time(e1) / timed, stats

    qs, ms_s, (ne, nfb) = go(learned, sur)
    qr, ms_r, _ = go(plain, None)
    mc.mc_sur_destroy(sur)

    def l1(q):
        """relative L1 of the density (depth), the momenta against the sum
        of rho c (h sqrt(g h)), and (Euler) the energy"""
        if eu:
            pr = (gm - 1.0) * (qo[3] - 0.5 * (qo[1] ** 2 + qo[2] ** 2) / qo[0])
            den = np.sqrt(gm * pr * qo[0]).sum()
        else:
            den = np.abs(qo[0] * np.sqrt(g * qo[0])).sum()
        out = {"rho" if eu else "h": float(np.abs(q[0] - qo[0]).sum() / np.abs(qo[0]).sum()),
               "momentum": float((np.abs(q[1] - qo[1]).sum() + np.abs(q[2] - qo[2]).sum()) / den)}
        if eu:
            out["E"] = float(np.abs(q[3] - qo[3]).sum() / np.abs(qo[3]).sum())
        return out

    edges = 2 * (n + 1) * n
    evaluated = 2 * (n + 3) * n          # including the limiter's outer neighbours
    nin, nout = (7, 15) if eu else (6, 8)
    flop_edge = 2 * (nin * 128 + 3 * 128 * 128 + 128 * nout)
    rate = evaluated * flop_edge / (ms_s * 1e-3)
    return {"ms_per_step": ms_s, "edge_updates_per_s": edges / (ms_s * 1e-3),
            "roe_f32_ms_per_step": ms_r, "speed_vs_roe_f32": ms_r / ms_s,
            "l1": l1(qs), "l1_bound": 1e-3, "roe_f32_l1": l1(qr),
            "reference": "plain Roe FP64 on the same GPU, its own dt sequence", "steps": steps,
            "fallback_edges": nfb, "edges_solved": ne,
            "mfma_tflops": rate / 1e12, "mfma_frac_bf16_peak": rate / 2.5e15,
            "train_seconds": info["train_seconds"], "train_pairs": info["n_pairs"],
            "train_kept": info["n_kept"], "epochs": epochs, "val_loss": info["val_loss"]}


def run_methods(n=4096, steps=20, warmup=3, dtype_name="f64", seed=0):
    """The three 2D step forms on the shallow-water dam break (MC limiter,
    extrapolation boundaries, one eager launch sequence per step at a fixed
    dt of Courant number 0.8 from the start): the plain Godunov step
    (mc_step2d), Strang splitting (mc_step2d_strang: x(dt/2), y(dt) and the
    closing x(dt/2) fused in one pass) and the unsplit step with transverse
    solves (mc_step2d_unsplit, one pass).  Each form reads q^n once and
    writes q^{n+1} once."""
    import torch

    from paper_1308_1464_amd import inputs
    from paper_1308_1464_amd import manyclaw as mc

    dtype = mc.MC_F64 if dtype_name == "f64" else mc.MC_F32
    tdt = torch.float64 if dtype == mc.MC_F64 else torch.float32
    esize = 8 if dtype == mc.MC_F64 else 4
    q0 = torch.from_numpy(inputs.sw_dam_break(n, seed=seed)).to("cuda", tdt)
    ctx = mc.mc_ctx_create(mc.MC_SW_ROE, dtype, mc.params(g=9.81), n, n, 1.0 / n, 1.0 / n)
    out = {}
    try:
        cfl = torch.zeros(16, dtype=torch.uint8, device="cuda")
        mc.mc_max_speed(ctx, q0, None, mc.MC_BC_EXTRAP, cfl)
        torch.cuda.synchronize()
        dt = 0.8 / mc.cfl_from_tensor(cfl).smax
        stream = torch.cuda.current_stream()
        for name, fn in (("godunov", mc.mc_step2d), ("strang", mc.mc_step2d_strang),
                         ("unsplit", mc.mc_step2d_unsplit)):
            a = q0.clone()
            b = torch.empty_like(a)
            st = mc.state(a, b)
            for _ in range(warmup):
                fn(ctx, st, None, dt, mc.MC_LIM_MC, mc.MC_BC_EXTRAP, cfl)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(stream)
            for _ in range(steps):
                fn(ctx, st, None, dt, mc.MC_LIM_MC, mc.MC_BC_EXTRAP, cfl)
            e1.record(stream)
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            passes = 1
            bts = 2 * 3 * esize * n * n
            out[name] = {"ms_per_step": ms, "edge_updates_per_s": 2.0 * (n + 1) * n / (ms * 1e-3),
                         "launches": passes, "bytes_per_step": bts,
                         "achieved_gbs": bts / (ms * 1e-3) / 1e9,
                         "cfl": mc.cfl_from_tensor(cfl).cfl}
            del a, b
    finally:
        torch.cuda.synchronize()
        mc.mc_ctx_destroy(ctx)
    return out


def run_amr(n=1024, r=4, steps=20, warmup=2, dtype_name="f64", seed=0):
    """Two-level refinement coupling: the n x n dam break (extrapolation
    boundaries, MC limiter) with refined patches of 64 x 64 coarse cells
    along the circular front, ratio r in space and time.  dt = 0.6 / smax of
    the start (the fine steps dt / r then have the same Courant number).
    Times `steps` coarse steps (each: the coarse step, r ghost fills and
    fine steps, the fix-up and averaging down), launched one call per step
    on the context's stream."""
    import numpy as np
    import torch

    from paper_1308_1464_amd import inputs
    from paper_1308_1464_amd import manyclaw as mc

    dtype = mc.MC_F64 if dtype_name == "f64" else mc.MC_F32
    tdt = torch.float64 if dtype == mc.MC_F64 else torch.float32
    esize = 8 if dtype == mc.MC_F64 else 4
    boxes = inputs.amr_ring_boxes(n)
    qf = inputs.sw_dam_break(n * r, seed=seed)
    qc = qf.reshape(3, n, r, n, r).mean(axis=(2, 4))
    ctx = mc.mc_ctx_create(mc.MC_SW_ROE, dtype, mc.params(g=9.81), n, n, 1.0 / n, 1.0 / n)
    amr = mc.mc_amr_create(ctx, r, boxes, mc.MC_BC_EXTRAP)
    try:
        mc.mc_amr_set(amr, -1, torch.from_numpy(qc).to("cuda", tdt))
        for p, (i0, j0, w, h) in enumerate(boxes):
            mc.mc_amr_set(amr, p, torch.from_numpy(
                np.ascontiguousarray(qf[:, j0 * r:(j0 + h) * r, i0 * r:(i0 + w) * r])).to("cuda", tdt))
        hmax = float(qf[0].max())
        dt = 0.6 / (np.sqrt(9.81 * hmax) * n)     # coarse dt; the fine step dt / r has the same Courant number
        cfl = torch.zeros(16, dtype=torch.uint8, device="cuda")
        for _ in range(warmup):
            mc.mc_amr_step(amr, dt, mc.MC_LIM_MC, cfl)
        stream = torch.cuda.current_stream()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        for _ in range(steps):
            mc.mc_amr_step(amr, dt, mc.MC_LIM_MC, cfl)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        c = mc.cfl_from_tensor(cfl)
        status = mc.mc_status_get(ctx)
    finally:
        torch.cuda.synchronize()
        mc.mc_amr_destroy(amr)
        mc.mc_ctx_destroy(ctx)
    nf = [(w * r, h * r) for (_, _, w, h) in boxes]
    edges = 2.0 * (n + 1) * n + r * sum((x + 1) * y + (y + 1) * x for x, y in nf)
    cells = n * n + r * sum(x * y for x, y in nf)
    # walker traffic: read the padded grid, write its interior, per (sub)step;
    # averaging down reads the fine cells once
    walk_bytes = 3 * esize * ((n + 4) ** 2 + n * n + r * sum((x + 4) * (y + 4) + x * y for x, y in nf))
    avg_bytes = 3 * esize * sum(x * y for x, y in nf)
    bts = walk_bytes + avg_bytes
    return {"ms_per_step": ms, "edge_updates_per_s": edges / (ms * 1e-3),
            "cell_updates_per_s": cells / (ms * 1e-3), "patches": len(boxes), "ratio": r,
            "fine_cells": sum(x * y for x, y in nf), "coarse_cells": n * n,
            "bytes_per_step": bts, "achieved_gbs": bts / (ms * 1e-3) / 1e9,
            "frac": bts / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, "cfl": c.cfl, "status": status}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n", type=int, default=4096)
    ap.add_argument("--dtype", choices=["f64", "f32"], default="f64")
    ap.add_argument("--rows", type=int, default=0, help="rows per work item (0 = library default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the FP32 companion measurement")
    ap.add_argument("--probe-only", action="store_true",
                    help="only run the copy probe (counter calibration) and print its GB/s")
    ap.add_argument("--only", choices=["euler", "patches", "surrogate", "surrogate_euler", "paper", "amr",
                                       "methods"],
                    default=None,
                    help="run one companion workload alone and print its result (for profiling)")
    ap.add_argument("--sur-epochs", type=int, default=20)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}): the slab sharding with "
              "halo exchange over RCCL is not built", file=sys.stderr)
        sys.exit(2)

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.probe_only:
        print(json.dumps({"copy_probe_gbs": copy_probe()}), flush=True)
        return
    if args.only == "euler":
        print(json.dumps(run_gpu(args.n, "f32", args.steps, args.warmup, 0, problem="euler")), flush=True)
        return
    if args.only == "paper":
        print(json.dumps(run_paper_kernels(n=args.n, steps=args.steps, warmup=args.warmup)), flush=True)
        return
    if args.only == "patches":
        print(json.dumps(run_patches(steps=args.steps)), flush=True)
        return
    if args.only == "surrogate":
        print(json.dumps(run_surrogate(args.n, steps=args.steps, epochs=args.sur_epochs)), flush=True)
        return
    if args.only == "amr":
        print(json.dumps(run_amr(dtype_name=args.dtype)), flush=True)
        return
    if args.only == "methods":
        print(json.dumps(run_methods(args.n, dtype_name=args.dtype)), flush=True)
        return
    if args.only == "surrogate_euler":
        print(json.dumps(run_surrogate(1024, steps=args.steps, epochs=args.sur_epochs, model="euler")),
              flush=True)
        return
    log(f"bench: shallow water {args.n}x{args.n} {args.dtype}, {args.warmup} warmup + {args.steps} timed steps")
    r = run_gpu(args.n, args.dtype, args.steps, args.warmup, args.rows, reps=5)
    log(f"bench: {r}")
    extra = None
    if not args.no_extra:
        other = "f32" if args.dtype == "f64" else "f64"
        log(f"bench: companion run shallow water {other}")
        r2 = run_gpu(args.n, other, args.steps, args.warmup, args.rows)
        extra = [{"workload": "shallow water, same grid", "dtype": other,
                  "value": r2["edge_updates_per_s"], "ms_per_step": r2["ms_per_step"],
                  "achieved_gbs": r2["achieved_gbs"], "frac": r2["achieved_gbs"] / HBM_PEAK_GBS,
                  "accepted": r2["accepted"], "rejected": r2["rejected"], "rows_per_item": r2["rows"]}]
        log("bench: companion run Euler four quadrants f32, 100 steps")
        r3 = run_gpu(args.n, "f32", 100, args.warmup, 0, problem="euler")
        extra.append({"workload": f"Euler Roe+HH+HLLE, four quadrants {args.n}x{args.n}, CFL 0.8",
                      "dtype": "f32", "steps": 100, "value": r3["edge_updates_per_s"],
                      "ms_per_step": r3["ms_per_step"], "achieved_gbs": r3["achieved_gbs"],
                      "frac": r3["achieved_gbs"] / HBM_PEAK_GBS, "accepted": r3["accepted"],
                      "rejected": r3["rejected"], "status": r3["status"], "rows_per_item": r3["rows"]})
        log("bench: companion runs, the paper's four kernels at 2048x2048 FP64")
        extra.append({"workload": "the paper's four Riemann kernels, 2048x2048 FP64, MC limiter, "
                                  "50 graph-replayed steps of the device dt rule",
                      "dtype": "f64", "kernels": run_paper_kernels()})
        log("bench: companion runs, the same four kernels at 4096x4096 FP64")
        extra.append({"workload": "the paper's four Riemann kernels, 4096x4096 FP64, MC limiter, "
                                  "50 graph-replayed steps of the device dt rule",
                      "dtype": "f64", "kernels": run_paper_kernels(n=4096)})
        log("bench: companion run 2000 patches")
        r4 = run_patches()
        extra.append(dict(workload="2000 shallow-water patches, sides log-uniform in [16,256], "
                                   "own dt each, 20 steps in one persistent graph launch",
                          dtype="f64", **r4))
        log("bench: companion runs, Godunov / Strang / unsplit step forms")
        r8 = run_methods(args.n, dtype_name=args.dtype)
        log(f"bench: {r8}")
        extra.append({"workload": f"shallow water {args.n}x{args.n} dam break, MC, Courant number 0.8, "
                                  "the three step forms launched one step per call",
                      "dtype": args.dtype, "forms": r8})
        log("bench: companion run two-level refinement")
        r7 = run_amr()
        log(f"bench: {r7}")
        extra.append(dict(workload="two-level refinement: 1024x1024 dam break, ratio 4 patches of 64x64 "
                                   "coarse cells along the front (subcycled, space-time ghost "
                                   "interpolation, refluxing), 20 coarse steps", dtype="f64", **r7))
        log("bench: companion run learned edge solver")
        r5 = run_surrogate(args.n, epochs=args.sur_epochs)
        log(f"bench: {r5}")
        extra.append(dict(workload=f"shallow water {args.n}x{args.n} dam break, learned edge solver "
                                   "(6-128x4-8 GELU, BF16 MFMA, FP32 state), trained on the GPU on "
                                   "2^24 Roe pairs; 50 steps against plain FP64 Roe",
                          dtype="f32 state, bf16 network", **r5))
        log("bench: companion run learned Euler edge solver")
        r6 = run_surrogate(1024, epochs=args.sur_epochs, model="euler")
        log(f"bench: {r6}")
        extra.append(dict(workload="Euler 1024x1024 four quadrants, learned edge solver "
                                   "(7-128x4-15 GELU, BF16 MFMA, FP32 state), trained on the GPU on "
                                   "2^24 Roe pairs; 50 steps against plain FP64 Roe",
                          dtype="f32 state, bf16 network", **r6))
    ceiling = copy_probe()
    log(f"bench: copy probe {ceiling:.0f} GB/s")
    cpu = None
    if not args.no_cpu_baseline:
        log("bench: cpu baseline (oracle)")
        cpu = cpu_baseline(args.n)
    out = {
        "metric": METRIC,
        "value": r["edge_updates_per_s"],
        "unit": "edge updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.dtype,
        "data": "synthetic",
        "config": {"workload": f"shallow-water Roe+HH, MC limiter, extrapolation BC, "
                               f"{args.n}x{args.n} radial dam break + 1e-3 noise, CFL 0.9, "
                               f"device dt rule, graph-captured steps",
                   "nx": args.n, "ny": args.n, "edges_per_step": 2 * (args.n + 1) * args.n,
                   "accepted_steps": r["accepted"], "rejected_steps": r["rejected"],
                   "hbm_gbs": r["achieved_gbs"], "rows_per_item": r["rows"],
                   "replays_ms_per_step": {"median": statistics.median(r["rep_ms_per_step"]),
                                           "min": min(r["rep_ms_per_step"]),
                                           "max": max(r["rep_ms_per_step"]),
                                           "n": len(r["rep_ms_per_step"])}},
        "roofline": {"bound": "hbm", "achieved": r["achieved_gbs"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": r["achieved_gbs"] / HBM_PEAK_GBS,
                     "traffic": (None if args.n != 4096 else profiled(f"{args.dtype}_traffic_bytes")),
                     "copy_ceiling_gbs": ceiling, "frac_of_copy": r["achieved_gbs"] / ceiling},
        "cpu_baseline": cpu,
    }
    valu = None if args.n != 4096 else profiled(f"{args.dtype}_valu_insts")
    if valu:
        # the kernel is bound by vector-ALU issue, not by HBM: VALU instructions
        # per dispatch (counters of the committed profile) x 64 lanes / live time
        rate = valu * 64 / (r["ms_per_step"] * 1e-3)
        out["roofline"]["valu_issue"] = {"insts_per_launch": valu, "achieved": rate,
                                         "peak": VALU_PEAK, "unit": "lane-ops/s",
                                         "frac": rate / VALU_PEAK}
    if extra:
        out["companions"] = extra
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
