"""Benchmark of the k-space-preconditioned PDHG hot path on one MI355X.

Workload: 3D centre-out UTE radial, 160^3 complex64 image, 8 coils,
20000 half-spokes x 128 samples (2.56 M samples per coil), oversampling
1.25, Kaiser-Bessel width 4, l1-wavelet (db4, 4 levels, lambda 5e-3),
multi-channel k-space preconditioner, 30 PDHG iterations.  Seeded synthetic
inputs (random ellipsoids, Gaussian-blob coil maps with unit sum of squares,
Fibonacci-sphere spokes, complex Gaussian noise sigma 1e-3); the k-space data
come from a more accurate NUFFT (alpha 2, W 8) of the phantom plus noise.

A timed step is one PDHG iteration (forward NUFFT with the fused dual
update, adjoint NUFFT with the fused primal update, wavelet prox and
extrapolation); K steps run as one pdhg_solve of K iterations with the
preconditioner and lambda_max prepared beforehand (their build times are
reported separately).  `value` is the NUFFT forward+adjoint throughput those
steps achieve, in Msamples.coil/s: M C K / t.

Prints one JSON line.  `python bench.py --gpus N --steps K --warmup W`.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def byte_model(shape, G, C, M, d):
    """Algorithmic HBM bytes of one forward + adjoint (grid-in-HBM model).

    Forward per coil: read x share and s_c, pruned FFT passes (pass j writes
    the array with axis d-1-j expanded N -> G; every later pass reads it
    back), read grid + coordinates/permutation share, write y.  Adjoint: the
    mirror image.  Returns a dict of per-kernel and total bytes.
    """
    N = list(shape)
    Ntot = int(np.prod(N))
    # forward passes: sizes after each pass (complex64 x C)
    sizes = []
    cur = list(N)
    for p in range(d):
        ax = d - 1 - p
        cur[ax] = G[ax]
        sizes.append(int(np.prod(cur)) * 8 * C)
    fwd_fft = (Ntot * 8 + Ntot * 8 * C) + sizes[0]          # pass 1: read x, s; write
    for p in range(1, d):
        fwd_fft += sizes[p - 1] + sizes[p]
    grid = int(np.prod(G)) * 8 * C
    coords = M * (4 * d + 4)
    interp = grid + coords + M * 8 * C
    spread = M * 8 * C + coords + grid
    adj_fft = fwd_fft                                         # mirror image
    return {"fwd_fft": fwd_fft, "interp": interp, "spread": spread, "adj_fft": adj_fft,
            "total": fwd_fft + interp + spread + adj_fft, "grid": grid}


KERNEL_NAMES = {"interp": "k_interp_tl3<8,8,8,4>", "spread": "k_spread<3,4,4,4,true>"}
# sources whose change invalidates a committed counter measurement
TRAFFIC_SOURCES = ["paper_1902_09657_amd/csrc/grid.hip", "paper_1902_09657_amd/csrc/plan.hip",
                   "paper_1902_09657_amd/csrc/kp_internal.h"]


def source_digest():
    import hashlib
    h = hashlib.sha256()
    for f in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE and WRITE_SIZE scaled by a plain copy's readings), or None when
    there is none or the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_3d-ute-160-8coil.md" % kernel)
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if " = " in line:
                k, v = line.strip().split(" = ", 1)
                vals[k.strip()] = v.strip()
    if vals.get("source_sha256") != source_digest():
        return None
    try:
        return int(float(vals["traffic_bytes_per_launch"]))
    except (KeyError, ValueError):
        return None


_POOL = {}


def _coil_worker(c):
    """One coil of the workload in a forked worker: tap setup (untimed), wait
    for every worker, then the oracle's forward + adjoint (timed)."""
    from oracle import nufft as onufft
    cfg, k, x, maps, barrier = (_POOL[n] for n in ("cfg", "k", "x", "maps", "barrier"))
    op = onufft.Nufft(k, cfg.shape, maps[c:c + 1], cfg.alpha, cfg.width)
    barrier.wait()
    t0 = time.perf_counter()
    y = op.forward(x)
    op.adjoint(y)
    return time.perf_counter() - t0


def cpu_legs(cfg, k, x, maps, pool_workers):
    """The FP64 oracle's NUFFT forward + adjoint on the host, before any GPU
    use (the all-cores leg forks worker processes):
    * one core: coil 0 of the workload (full 200^3 grid, every sample), tap
      setup excluded; its outputs also serve as the parity reference;
    * all cores: the 8 coils in a coil-parallel pool of forked workers, one
      coil each, timed together after every worker's tap setup."""
    import multiprocessing as mp
    from oracle import nufft as onufft
    M, C = k.shape[0], cfg.ncoils
    t0 = time.perf_counter()
    op = onufft.Nufft(k, cfg.shape, maps[:1], cfg.alpha, cfg.width)
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    y0 = op.forward(x)
    t1 = time.perf_counter()
    xa0 = op.adjoint(y0)
    t2 = time.perf_counter()
    del op
    one = {"value": M / (t2 - t0) / 1e6, "unit": "Msamples*coil/s", "cores": 1, "kind": "oracle",
           "sample": "coil 0 of the workload (full 200^3 grid, all %d samples): forward %.1f s + adjoint %.1f s, "
                     "tap setup %.1f s excluded; numpy FFT single-threaded" % (M, t1 - t0, t2 - t1, t_setup)}
    nw = min(C, pool_workers)
    ctx = mp.get_context("fork")
    _POOL.update(cfg=cfg, k=k, x=x, maps=maps, barrier=ctx.Barrier(nw))
    t0 = time.perf_counter()
    with ctx.Pool(nw) as pool:
        times = pool.map(_coil_worker, list(range(nw)), chunksize=1)
    wall = time.perf_counter() - t0
    _POOL.clear()
    t_max = max(times)
    allc = {"value": M * nw / t_max / 1e6, "unit": "Msamples*coil/s", "cores": nw, "kind": "oracle",
            "sample": "%d of the %d coils of the workload, one per forked worker (full grid, all samples), forward + "
                      "adjoint timed together after every worker's tap setup: slowest worker %.1f s (pool wall %.1f s "
                      "incl. setup)" % (nw, C, t_max, wall),
            "one_core": one}
    return allc, (y0, xa0)


def oracle_small_timings():
    """The oracle on the two 2D workloads: NUFFT forward + adjoint,
    preconditioner build (efficient algorithm at 2N) and the whole PDHG solve
    (30 power-method iterations and the workload's iterations), one process."""
    import synth
    from oracle import nufft as onufft
    from oracle import pdhg as opdhg
    from oracle import precond as oprecond
    out = {}
    for cid, iters, pits in ((1, 20, 30), (2, 30, 30)):
        cfg = synth.config(cid)
        x, maps, k, w = cfg.inputs(seed=cid)
        op = onufft.Nufft(k, cfg.shape, maps, cfg.alpha, cfg.width)
        t0 = time.perf_counter()
        y = op.forward(x)
        op.adjoint(y)
        t_pair = time.perf_counter() - t0
        y = y + w
        t0 = time.perf_counter()
        p = oprecond.efficient_nufft(maps if cfg.precond == "mc" else None, k, cfg.shape, cfg.alpha, cfg.width)
        t_pre = time.perf_counter() - t0
        t0 = time.perf_counter()
        opdhg.pdhg(op.forward, op.adjoint, y, p, cfg.shape, cfg.reg, cfg.lam, iters, power_iters=pits, levels=4)
        t_solve = time.perf_counter() - t0
        out[cfg.name] = {"nufft_pair_s": round(t_pair, 3), "precond_%s_s" % cfg.precond: round(t_pre, 3),
                         "solve_s": round(t_solve, 3), "solve_iters": iters, "power_iters": pits,
                         "msamples_coil_per_s": round(k.shape[0] * cfg.ncoils / t_pair / 1e6, 4), "cores": 1}
    return out


def _events():
    import torch
    return torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)


def _rel(a, b):
    import torch
    return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))


def bench_small_configs(kp, dev, reps=20):
    """The two 2D workloads at their full sizes on the GPU (absolute numbers:
    their grids sit in L2 / Infinity Cache, so they are launch and latency
    bound): NUFFT forward + adjoint through the C ABI and the PDHG solve of the
    workload (its regulariser, preconditioner and iteration count)."""
    import torch
    import synth
    out = {}
    s = torch.cuda.current_stream()
    e0, e1 = _events()
    for cid in (1, 2):
        cfg = synth.config(cid)
        x, maps, k, w = cfg.inputs(seed=cid)
        M, C = k.shape[0], cfg.ncoils
        kt = torch.from_numpy(k).to(dev)
        mt = None if maps is None else torch.from_numpy(maps.astype(np.complex64)).to(dev)
        xt = torch.from_numpy(x.astype(np.complex64)).to(dev)
        hi = kp.nufft_plan(kt, cfg.shape, mt, oversamp=2.0, kb_width=8)
        y = kp.nufft_forward(hi, xt) + torch.from_numpy(w.astype(np.complex64)).to(dev)
        hi.close()
        plan = kp.nufft_plan(kt, cfg.shape, mt, oversamp=cfg.alpha, kb_width=cfg.width)
        kind = kp.KP_PRECOND_MC if cfg.precond == "mc" else kp.KP_PRECOND_SC
        p = kp.precond_build(plan, kind)
        lmax = float(kp.pdhg_lambda_max(plan, p, 30).item())
        ya, xa = torch.empty_like(y), torch.empty_like(xt)
        for _ in range(3):
            kp.nufft_forward(plan, xt, ya)
            kp.nufft_adjoint(plan, ya, xa)
        torch.cuda.synchronize()
        e0.record(s)
        for _ in range(reps):
            kp.nufft_forward(plan, xt, ya)
            kp.nufft_adjoint(plan, ya, xa)
        e1.record(s)
        torch.cuda.synchronize()
        t_pair = e0.elapsed_time(e1) / 1e3 / reps
        kw = dict(reg=cfg.reg, lam=cfg.lam, iters=cfg.iters, wavelet_levels=4, lambda_max=lmax)
        kp.pdhg_solve(plan, y, p, **kw)
        torch.cuda.synchronize()
        e0.record(s)
        for _ in range(5):
            kp.pdhg_solve(plan, y, p, **kw)
        e1.record(s)
        torch.cuda.synchronize()
        t_solve = e0.elapsed_time(e1) / 1e3 / 5
        info = plan.info()
        bm = byte_model(cfg.shape, info["grid"], C, M, cfg.ndim)
        plan.close()
        out[cfg.name] = {
            "nufft_pair_us": round(t_pair * 1e6, 1),
            "nufft_pair_msamples_coil_per_s": round(M * C / t_pair / 1e6, 1),
            "nufft_pair_byte_model_frac": round(bm["total"] / t_pair / 1e9 / HBM_PEAK_GBS, 4),
            "pdhg_iters": cfg.iters, "pdhg_solve_ms": round(t_solve * 1e3, 3),
            "pdhg_iters_per_s": round(cfg.iters / t_solve, 1),
            "reg": cfg.reg, "precond": cfg.precond,
        }
    return out


def copy_bandwidth(dev, nbytes=1 << 30, reps=10):
    """Device-to-device copy of `nbytes` (read + write) timed with HIP events."""
    import torch
    a = torch.ones(nbytes // 8, dtype=torch.float64, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    s = torch.cuda.current_stream()
    e0, e1 = _events()
    torch.cuda.synchronize()
    e0.record(s)
    for _ in range(reps):
        b.copy_(a)
    e1.record(s)
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / reps
    del a, b
    return 2 * nbytes / t / 1e9


def gpu_clock():
    """Current and top shader clock (MHz) from sysfs, best effort."""
    import glob
    for path in sorted(glob.glob("/sys/class/drm/card*/device/pp_dpm_sclk")):
        try:
            lines = open(path).read().split("\n")
        except OSError:
            continue
        mhz = []
        cur = None
        for ln in lines:
            parts = ln.replace("Mhz", "").replace("MHz", "").split()
            if len(parts) >= 2 and parts[1].isdigit():
                mhz.append(int(parts[1]))
                if "*" in ln:
                    cur = int(parts[1])
        if mhz:
            return {"sclk_mhz_current": cur, "sclk_mhz_max": max(mhz), "source": path}
    return None


def precond_comparison_3d(kp, plan, y, p_mc, cfg, lmax_mc, dev):
    """P = I vs SC vs MC vs the Pipe-Menon DCF on the timed 3D UTE workload
    (l1-db4, lambda 5e-3):
    the normalised objective gap (f_k - f*) / (f_0 - f*) at k = 5, 10, 20, 30,
    f* the least objective of 300 MC-preconditioned iterations, and the time
    per iteration of each preconditioner (lambda_max by 30 power iterations
    each, built beforehand; the timed solves have no objective syncs)."""
    import torch
    s = torch.cuda.current_stream()
    e0, e1 = _events()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    p_dcf = kp.precond_build(plan, kp.KP_PRECOND_DCF)
    torch.cuda.synchronize()
    dcf_s = time.perf_counter() - t0
    ps = {"none": None, "sc": kp.precond_build(plan, kp.KP_PRECOND_SC), "mc": p_mc, "dcf": p_dcf}
    lm = {"none": float(kp.pdhg_lambda_max(plan, None, 30).item()),
          "sc": float(kp.pdhg_lambda_max(plan, ps["sc"], 30).item()), "mc": lmax_mc,
          "dcf": float(kp.pdhg_lambda_max(plan, ps["dcf"], 30).item())}
    kw = dict(reg=cfg.reg, lam=cfg.lam, wavelet_levels=4)
    _, ref = kp.pdhg_solve(plan, y, p_mc, iters=300, lambda_max=lm["mc"], objective=True, **kw)
    fstar = min(ref)
    comp = {}
    for name, p in ps.items():
        _, hist = kp.pdhg_solve(plan, y, p, iters=30, lambda_max=lm[name], objective=True, **kw)
        torch.cuda.synchronize()
        e0.record(s)
        kp.pdhg_solve(plan, y, p, iters=30, lambda_max=lm[name], **kw)
        e1.record(s)
        torch.cuda.synchronize()
        gap = [(h - fstar) / (hist[0] - fstar) for h in hist]
        comp[name] = {"gap_at": {str(i): float("%.4g" % gap[i]) for i in (5, 10, 20, 30)},
                      "ms_per_iter": round(e0.elapsed_time(e1) / 30, 4), "lambda_max": round(lm[name], 6)}
    return {"workload": cfg.name + ", l1-db4 lambda 5e-3, 30 iterations",
            "reference": "f* = least objective of 300 MC-preconditioned iterations", "gap": comp,
            "dcf_build_s": round(dcf_s, 4)}


def bench_batched(kp, dev, reps=3):
    """64 uneven 2D 12-coil radial slices, l2 PDHG, 20 iterations each: one
    pdhg_solve_batch (one launch per phase over all slices, iterations in a
    HIP graph, autotuned tiles) against pdhg_solve slice after slice."""
    import torch
    import synth
    K, C, lam = 20, 12, 1e-3
    sl = synth.slice_config4(64, seed=4, ncoils=C)
    log("batched: inputs and data for", len(sl), "slices")
    coords, maps, ys, xs_true = [], [], [], []
    for i, (shape, k) in enumerate(sl):
        rp, rm, _, rn = synth.streams(4000 + i)
        x = synth.phantom(shape, rp)
        m = synth.coil_maps(shape, C, rm)
        kt = torch.from_numpy(k).to(dev)
        mt = torch.from_numpy(m.astype(np.complex64)).to(dev)
        hi = kp.nufft_plan(kt, shape, mt, oversamp=2.0, kb_width=8)
        w = torch.from_numpy(synth.noise((C, k.shape[0]), 1e-3, rn).astype(np.complex64)).to(dev)
        ys.append(kp.nufft_forward(hi, torch.from_numpy(x.astype(np.complex64)).to(dev)) + w)
        hi.close()
        coords.append(kt)
        maps.append(mt)
    torch.cuda.synchronize()
    log("batched: plain plans, preconditioners, lambda_max")
    plans, ps, lms = [], [], []
    for (shape, _), kt, mt in zip(sl, coords, maps):
        pl = kp.nufft_plan(kt, shape, mt, oversamp=1.25, kb_width=4)
        p = kp.precond_build(pl, kp.KP_PRECOND_MC)
        lms.append(float(kp.pdhg_lambda_max(pl, p, 30).item()))
        plans.append(pl)
        ps.append(p)
    log("batched: batch plan (autotuned)")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b = kp.nufft_plan_batch(coords, [s for s, _ in sl], maps, oversamp=1.25, kb_width=4, tune=True)
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    fast = all(kp.nufft_batch_info(b, i)["fast"] for i in range(len(sl)))
    tiles = sorted({kp.nufft_batch_info(b, i)["bin_size"] for i in range(len(sl))})
    spread_tiles = sorted({kp.nufft_batch_info(b, i)["spread_bin_size"] for i in range(len(sl))})
    s = torch.cuda.current_stream()
    e0, e1 = _events()
    xb = kp.pdhg_solve_batch(b, ys, ps, lam=lam, iters=K, lambda_max=lms)    # captures the graph
    torch.cuda.synchronize()
    e0.record(s)
    for _ in range(reps):
        xb = kp.pdhg_solve_batch(b, ys, ps, lam=lam, iters=K, lambda_max=lms)
    e1.record(s)
    torch.cuda.synchronize()
    t_b = e0.elapsed_time(e1) / 1e3 / reps
    for i, pl in enumerate(plans):
        kp.pdhg_solve(pl, ys[i], ps[i], reg="l2", lam=lam, iters=2, lambda_max=lms[i])
    torch.cuda.synchronize()
    e0.record(s)
    xp = [kp.pdhg_solve(pl, ys[i], ps[i], reg="l2", lam=lam, iters=K, lambda_max=lms[i]) for i, pl in enumerate(plans)]
    e1.record(s)
    torch.cuda.synchronize()
    t_p = e0.elapsed_time(e1) / 1e3
    diff = max(_rel(a, c) for a, c in zip(xb, xp))
    MC = sum(int(k.shape[0]) for _, k in sl) * C
    for pl in plans:
        pl.close()
    b.close()
    return {
        "workload": "64 uneven 2D radial slices, N in {128,192,256,320}, 32-256 spokes x 2N, 12 coils, "
                    "alpha 1.25, W 4, l2 lambda 1e-3, mc precond, 20 iters",
        "slices": len(sl), "iters": K, "samples_coil_total": MC, "one_launch_per_phase": fast,
        "tiles": [list(t) for t in tiles], "spread_tiles": [list(t) for t in spread_tiles],
        "plan_s_incl_autotune": round(t_plan, 3),
        "batched_ms": round(t_b * 1e3, 3), "plain_ms": round(t_p * 1e3, 3),
        "speedup_vs_plain": round(t_p / t_b, 3),
        "batched_msamples_coil_per_s": round(MC * K / t_b / 1e6, 1),
        "plain_msamples_coil_per_s": round(MC * K / t_p / 1e6, 1),
        "batched_slice_iters_per_s": round(len(sl) * K / t_b, 1),
        "max_rel_diff_vs_plain": diff,
    }


def bench_differentiable(kp, dev, reps=3):
    """8 2D 12-coil spiral slices 256^2, 10-step unrolled l2 PDHG with
    learnable step sizes and lambda, loss 1/2||x_K - x_true||^2, forward and
    backward through the autograd Function (checkpoints every 4 steps),
    against the plain 10-iteration pdhg_solve of the same slices."""
    import torch
    import synth
    from paper_1902_09657_amd.autograd import schedule_params, unrolled_pdhg, unrolled_pdhg_batch
    cfg = synth.config(5)
    K, C, nb = cfg.iters, cfg.ncoils, cfg.extra["batch"]
    log("differentiable: inputs for", nb, "slices")
    plans, ys, ps, xt, lms = [], [], [], [], []
    for i in range(nb):
        x, m, k, w = cfg.inputs(seed=5000 + i)
        kt = torch.from_numpy(k).to(dev)
        mt = torch.from_numpy(m.astype(np.complex64)).to(dev)
        xg = torch.from_numpy(x.astype(np.complex64)).to(dev)
        hi = kp.nufft_plan(kt, cfg.shape, mt, oversamp=2.0, kb_width=8)
        ys.append(kp.nufft_forward(hi, xg) + torch.from_numpy(w.astype(np.complex64)).to(dev))
        hi.close()
        pl = kp.nufft_plan(kt, cfg.shape, mt, oversamp=cfg.alpha, kb_width=cfg.width)
        p = kp.precond_build(pl, kp.KP_PRECOND_MC)
        lms.append(float(kp.pdhg_lambda_max(pl, p, 30).item()))
        plans.append(pl)
        ps.append(p)
        xt.append(xg)
    params = [schedule_params(pl, ps[i], K, lam=cfg.lam, lambda_max=lms[i]) for i, pl in enumerate(plans)]

    def step():
        # one forward + backward over the 8 slices as one batch (slices run
        # concurrently on side streams); loss = sum of the slices' losses
        ths = [pr.detach().clone().requires_grad_(True) for pr in params]
        xks = unrolled_pdhg_batch(ys, ths, plans, ps, K)
        loss = 0.0
        for i, xk in enumerate(xks):
            r = xk - xt[i]
            loss = loss + 0.5 * (r.real ** 2 + r.imag ** 2).sum()
        loss.backward()
        return [xk.detach() for xk in xks], loss.detach(), [th.grad for th in ths]

    def step_sequential():
        # the same, slice after slice through the single-slice Function
        out = []
        for i, pl in enumerate(plans):
            th = params[i].detach().clone().requires_grad_(True)
            xk = unrolled_pdhg(ys[i], th, pl, ps[i], K)
            r = xk - xt[i]
            (0.5 * (r.real ** 2 + r.imag ** 2).sum()).backward()
            out.append(th.grad)
        return out

    s = torch.cuda.current_stream()
    e0, e1 = _events()
    step()
    torch.cuda.synchronize()
    e0.record(s)
    for _ in range(reps):
        xs, loss, grads = step()
    e1.record(s)
    torch.cuda.synchronize()
    t_fb = e0.elapsed_time(e1) / 1e3 / reps
    step_sequential()
    torch.cuda.synchronize()
    e0.record(s)
    for _ in range(reps):
        grads_seq = step_sequential()
    e1.record(s)
    torch.cuda.synchronize()
    t_seq = e0.elapsed_time(e1) / 1e3 / reps
    gdiff = max(_rel(a, b) for a, b in zip(grads, grads_seq))
    xp = [kp.pdhg_solve(pl, ys[i], ps[i], reg="l2", lam=cfg.lam, iters=K, lambda_max=lms[i])
          for i, pl in enumerate(plans)]
    torch.cuda.synchronize()
    e0.record(s)
    for _ in range(reps):
        xp = [kp.pdhg_solve(pl, ys[i], ps[i], reg="l2", lam=cfg.lam, iters=K, lambda_max=lms[i])
              for i, pl in enumerate(plans)]
    e1.record(s)
    torch.cuda.synchronize()
    t_p = e0.elapsed_time(e1) / 1e3 / reps
    diff = max(_rel(a, c) for a, c in zip(xs, xp))
    ck = kp._lib.load().pdhg_unrolled_ckpt_bytes(plans[0].handle, K, 4)
    for pl in plans:
        pl.close()
    return {
        "workload": cfg.name + " x%d slices, %d-step unrolled l2 PDHG, learnable steps and lambda" % (nb, K),
        "fwd_bwd_ms": round(t_fb * 1e3, 3), "plain_solve_ms": round(t_p * 1e3, 3),
        "fwd_bwd_over_plain": round(t_fb / t_p, 3), "fwd_bwd_ms_slice_after_slice": round(t_seq * 1e3, 3),
        "loss": float(loss.item()), "ckpt_bytes_per_slice": int(ck), "max_rel_diff_forward_vs_plain": diff,
        "max_rel_diff_grad_batch_vs_slice_after_slice": gdiff,
    }


def bench_context(kp, dev):
    """Context runs (not the headline): (1) P = I vs SC vs MC on the 2D spiral
    workload (256^2, 8 coils, l1-db4, 30 iterations): normalised objective gap
    (f_k - f*) / (f_0 - f*) with f* from 300 MC-preconditioned iterations, and
    the time per iteration; (2) the l2 problem (lambda 1e-2) solved through
    its dual by CG preconditioned with P = I, SC, MC against the SC / MC
    preconditioned PDHG, as the distance to x* per iteration; (3)
    preconditioner build time at the two fully
    specified shapes of the paper's Table I (synthetic trajectories and maps;
    the 255 x 200 brain matrix is taken as 256 x 200 since image extents must be
    even here), beside the paper's Titan Xp figures."""
    import torch
    import synth
    out = {}
    cfg = synth.config(2)
    x, maps, k, w = cfg.inputs(seed=2)
    kt = torch.from_numpy(k).to(dev)
    mt = torch.from_numpy(maps.astype(np.complex64)).to(dev)
    hi = kp.nufft_plan(kt, cfg.shape, mt, oversamp=2.0, kb_width=8)
    y = kp.nufft_forward(hi, torch.from_numpy(x.astype(np.complex64)).to(dev)) + \
        torch.from_numpy(w.astype(np.complex64)).to(dev)
    hi.close()
    plan = kp.nufft_plan(kt, cfg.shape, mt, oversamp=cfg.alpha, kb_width=cfg.width)
    ps = {"none": None, "sc": kp.precond_build(plan, kp.KP_PRECOND_SC), "mc": kp.precond_build(plan, kp.KP_PRECOND_MC),
          "dcf": kp.precond_build(plan, kp.KP_PRECOND_DCF)}
    _, ref = kp.pdhg_solve(plan, y, ps["mc"], reg=cfg.reg, lam=cfg.lam, iters=300, wavelet_levels=4, objective=True)
    fstar = min(ref)
    s = torch.cuda.current_stream()
    e0, e1 = _events()
    comp = {}
    for name, p in ps.items():
        _, hist = kp.pdhg_solve(plan, y, p, reg=cfg.reg, lam=cfg.lam, iters=30, wavelet_levels=4, objective=True)
        torch.cuda.synchronize()
        e0.record(s)
        kp.pdhg_solve(plan, y, p, reg=cfg.reg, lam=cfg.lam, iters=30, wavelet_levels=4)
        e1.record(s)
        torch.cuda.synchronize()
        gap = [(h - fstar) / (hist[0] - fstar) for h in hist]
        comp[name] = {"gap_at": {str(i): float("%.4g" % gap[i]) for i in (5, 10, 20, 30)},
                      "ms_per_iter_incl_power_method": round(e0.elapsed_time(e1) / 30, 4)}
    out["precond_comparison"] = {"workload": cfg.name + ", l1-db4 lambda 5e-3, 30 iterations",
                                 "reference": "f* = min objective of 300 MC iterations", "gap": comp}
    # the same comparison for the Experiments' other two regularisers at their
    # lambda (l2 1e-2, anisotropic TV 1e-3)
    for reg, lam_r in (("l2", 1e-2), ("tv", 1e-3)):
        _, ref = kp.pdhg_solve(plan, y, ps["mc"], reg=reg, lam=lam_r, iters=300, objective=True)
        fstar = min(ref)
        comp_r = {}
        for name, p in ps.items():
            _, hist = kp.pdhg_solve(plan, y, p, reg=reg, lam=lam_r, iters=30, objective=True)
            gap = [(h - fstar) / (hist[0] - fstar) for h in hist]
            comp_r[name] = {"gap_at": {str(i): float("%.4g" % gap[i]) for i in (5, 10, 20, 30)}}
        out["precond_comparison_" + reg] = {"workload": "%s, %s lambda %g, 30 iterations" % (cfg.name, reg, lam_r),
                                            "reference": "f* = min objective of 300 MC iterations", "gap": comp_r}
    # (3) l2 (lambda 1e-2, the paper's l2 value): the dual solve by k-space
    # preconditioned CG vs the preconditioned PDHG, relative distance to x*
    lam2 = 1e-2
    xs = kp.pdhg_solve(plan, y, ps["mc"], reg="l2", lam=lam2, iters=500)
    nrm = float(torch.linalg.vector_norm(xs))
    l2 = {}
    for name in ("none", "sc", "mc"):
        row = {}
        for it in (5, 10, 20, 30):
            xk = kp.l2_dual_cg(plan, y, ps[name], lam=lam2, iters=it)
            row[str(it)] = float("%.4g" % (float(torch.linalg.vector_norm(xk - xs)) / nrm))
        torch.cuda.synchronize()
        e0.record(s)
        kp.l2_dual_cg(plan, y, ps[name], lam=lam2, iters=30)
        e1.record(s)
        torch.cuda.synchronize()
        l2["dual_pcg_" + name] = {"rel_err_at": row, "ms_per_iter": round(e0.elapsed_time(e1) / 30, 4)}
    for name in ("sc", "mc"):
        row = {}
        for it in (5, 10, 20, 30):
            xk = kp.pdhg_solve(plan, y, ps[name], reg="l2", lam=lam2, iters=it)
            row[str(it)] = float("%.4g" % (float(torch.linalg.vector_norm(xk - xs)) / nrm))
        torch.cuda.synchronize()
        e0.record(s)
        kp.pdhg_solve(plan, y, ps[name], reg="l2", lam=lam2, iters=30)
        e1.record(s)
        torch.cuda.synchronize()
        l2["pdhg_" + name] = {"rel_err_at": row, "ms_per_iter_incl_power_method": round(e0.elapsed_time(e1) / 30, 4)}
    plan.close()
    out["l2_dual_cg_vs_pdhg"] = {"workload": cfg.name + ", l2 lambda 1e-2",
                                 "reference": "x* = 500 MC-preconditioned PDHG iterations",
                                 "rel_err = |x_k - x*| / |x*|": l2}
    # Table I shapes
    rows = []
    rng = np.random.default_rng(7)
    th = 2 * np.pi * np.arange(754) / 754
    r = np.pi * np.arange(256) / 256
    brain = np.stack([np.outer(np.cos(th), r).ravel(), np.outer(np.sin(th), r).ravel()], axis=1).astype(np.float32)
    for name, shape, coords, paper_s in (("cardiac", (320, 320), synth.spiral_2d(3, 3996, 320 / 6), 0.117),
                                         ("brain", (256, 200), brain, 0.0334)):
        m = torch.from_numpy(synth.coil_maps(shape, 8, rng).astype(np.complex64)).to(dev)
        ct = torch.from_numpy(coords).to(dev)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        pl = kp.nufft_plan(ct, shape, m, oversamp=1.25, kb_width=4)
        torch.cuda.synchronize()
        t_plan = time.perf_counter() - t0
        kp.precond_build(pl, kp.KP_PRECOND_MC)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        kp.precond_build(pl, kp.KP_PRECOND_MC)
        torch.cuda.synchronize()
        t_mc = time.perf_counter() - t0
        pl.close()
        rows.append({"dataset_shape": name, "image": list(shape), "coils": 8, "samples": int(coords.shape[0]),
                     "plan_ms": round(t_plan * 1e3, 2), "mc_precond_ms": round(t_mc * 1e3, 2),
                     "paper_mc_precond_ms_titan_xp": paper_s * 1e3})
    out["table1_precond_build"] = rows
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true",
                    help="skip the oracle legs (cpu_baseline, the parity gate and the oracle timings)")
    ap.add_argument("--pool-workers", type=int, default=16, help="processes of the all-cores oracle leg (at most)")
    ap.add_argument("--kernel-reps", type=int, default=20)
    ap.add_argument("--no-forms", action="store_true", help="skip the batched and differentiable forms")
    ap.add_argument("--profile-stages", type=int, default=0, metavar="R",
                    help="counter-collection mode: build the plan, run the wavelet prox and each NUFFT stage R "
                         "times and a plain copy of 512 MiB (read) + 512 MiB (write) for calibration, then exit "
                         "without a JSON line")
    ap.add_argument("--form-only", choices=["batched", "differentiable"], default=None,
                    help="profiling mode: run only that form's measurement and print its JSON object (no headline "
                         "line)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (the per-GPU share is the "
              "single-GPU workload); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import synth
    cfg = synth.config(3)
    cpu, ref, oracle_t = None, None, None
    if not args.form_only and not args.profile_stages:
        log("generating inputs", cfg.name)
        x, maps, k, w = cfg.inputs(seed=3)
        if not args.no_cpu_baseline:
            # the oracle legs run before anything touches the GPU (the
            # all-cores leg forks worker processes)
            log("cpu baseline: oracle, one core and a coil-parallel pool")
            workers = max(1, min(args.pool_workers, len(os.sched_getaffinity(0))))
            cpu, ref = cpu_legs(cfg, k, x, maps, workers)
            log("oracle timings of the 2D workloads")
            oracle_t = oracle_small_timings()

    import torch
    import paper_1902_09657_amd as kp
    from paper_1902_09657_amd import _lib

    dev = torch.device("cuda:0")
    if args.form_only:
        fn = bench_batched if args.form_only == "batched" else bench_differentiable
        print(json.dumps(fn(kp, dev)), flush=True)
        return
    d = cfg.ndim
    if args.profile_stages:
        x, maps, k, w = cfg.inputs(seed=3)
    M, C = k.shape[0], cfg.ncoils
    xt = torch.from_numpy(x.astype(np.complex64)).to(dev)
    mt = torch.from_numpy(maps.astype(np.complex64)).to(dev)
    kt = torch.from_numpy(k).to(dev)
    wt = torch.from_numpy(w.astype(np.complex64)).to(dev)
    torch.cuda.synchronize()

    if args.profile_stages > 0:
        plan = kp.nufft_plan(kt, cfg.shape, mt, oversamp=cfg.alpha, kb_width=cfg.width)
        L = _lib.load()
        sp = ctypes_stream(torch.cuda.current_stream())
        for st in (_lib.KP_STAGE_PROX, _lib.KP_STAGE_FWD_FFT, _lib.KP_STAGE_INTERP, _lib.KP_STAGE_SPREAD,
                   _lib.KP_STAGE_ADJ_FFT):
            _lib.check(L.nufft_stage(plan.handle, st, args.profile_stages, sp))
        a = torch.ones(64 * 1024 * 1024, dtype=torch.float64, device=dev)
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        plan.close()
        log("profile stages done")
        return

    # data: a more accurate NUFFT of the phantom plus noise
    log("data")
    hi = kp.nufft_plan(kt, cfg.shape, mt, oversamp=2.0, kb_width=8)
    y = kp.nufft_forward(hi, xt) + wt
    torch.cuda.synchronize()
    hi.close()
    del hi

    log("plan")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = kp.nufft_plan(kt, cfg.shape, mt, oversamp=cfg.alpha, kb_width=cfg.width)
    torch.cuda.synchronize()
    t_plan = time.perf_counter() - t0
    info = plan.info()
    log("plan info", info)

    # accuracy gate: coil 0 of the timed plan's forward, and its adjoint of
    # coil-0 data, against the oracle outputs of the one-core leg
    parity = None
    if ref is not None:
        log("parity gate")
        y0, xa0 = ref
        yg = kp.nufft_forward(plan, xt)[0].cpu().numpy()
        yin = torch.zeros((C, M), dtype=torch.complex64, device=dev)
        yin[0] = torch.from_numpy(y0[0].astype(np.complex64)).to(dev)
        xg = kp.nufft_adjoint(plan, yin).cpu().numpy()
        e_f = float(np.linalg.norm(yg - y0[0]) / np.linalg.norm(y0[0]))
        e_a = float(np.linalg.norm(xg - xa0) / np.linalg.norm(xa0))
        parity = {"forward_coil0_rel_l2": e_f, "adjoint_coil0_rel_l2": e_a, "gate": 1e-4,
                  "reference": "FP64 oracle (one-core leg)"}
        del yin
        if not (e_f <= 1e-4 and e_a <= 1e-4):
            print("bench.py: parity gate failed (forward %.3e, adjoint %.3e > 1e-4): no result" % (e_f, e_a),
                  file=sys.stderr, flush=True)
            sys.exit(3)

    log("precond")
    t0 = time.perf_counter()
    p = kp.precond_build(plan, kp.KP_PRECOND_MC)
    torch.cuda.synchronize()
    t_pre = time.perf_counter() - t0

    log("lambda_max")
    t0 = time.perf_counter()
    lmax = kp.pdhg_lambda_max(plan, p, 30)
    torch.cuda.synchronize()
    t_lmax = time.perf_counter() - t0
    lmax_v = float(lmax.item())

    solve_kw = dict(reg=cfg.reg, lam=cfg.lam, wavelet_levels=4, lambda_max=lmax_v)
    log("warmup")
    if args.warmup > 0:
        kp.pdhg_solve(plan, y, p, iters=args.warmup, **solve_kw)
    torch.cuda.synchronize()

    log("timed solve")
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(s)
    xr = kp.pdhg_solve(plan, y, p, iters=args.steps, **solve_kw)
    e1.record(s)
    torch.cuda.synchronize()
    t_wall = time.perf_counter() - t0
    t_solve = e0.elapsed_time(e1) / 1e3
    assert torch.isfinite(xr).all().item()

    # the same workload with the TV regulariser (constant steps), timed alike
    log("timed TV solve")
    kp.pdhg_solve(plan, y, p, reg="tv", lam=cfg.lam, lambda_max=lmax_v, iters=2)
    torch.cuda.synchronize()
    e0.record(s)
    kp.pdhg_solve(plan, y, p, reg="tv", lam=cfg.lam, lambda_max=lmax_v, iters=args.steps)
    e1.record(s)
    torch.cuda.synchronize()
    t_tv = e0.elapsed_time(e1) / 1e3

    # plain NUFFT forward + adjoint pairs through the C ABI
    log("nufft pairs")
    xa = torch.empty_like(xt)
    for _ in range(2):
        kp.nufft_forward(plan, xt, y)
        kp.nufft_adjoint(plan, y, xa)
    R = 10
    torch.cuda.synchronize()
    e0.record(s)
    for _ in range(R):
        kp.nufft_forward(plan, xt, y)
        kp.nufft_adjoint(plan, y, xa)
    e1.record(s)
    torch.cuda.synchronize()
    t_pair = e0.elapsed_time(e1) / 1e3 / R

    # per-stage timings (HIP events around launches of one stage on this stream)
    L = _lib.load()
    sp = ctypes_stream(s)
    stage_ms = {}
    for name, st in [("fwd_fft", _lib.KP_STAGE_FWD_FFT), ("interp", _lib.KP_STAGE_INTERP),
                     ("spread", _lib.KP_STAGE_SPREAD), ("adj_fft", _lib.KP_STAGE_ADJ_FFT),
                     ("wavelet_prox", _lib.KP_STAGE_PROX)]:
        _lib.check(L.nufft_stage(plan.handle, st, 2, sp))
        torch.cuda.synchronize()
        e0.record(s)
        _lib.check(L.nufft_stage(plan.handle, st, args.kernel_reps, sp))
        e1.record(s)
        torch.cuda.synchronize()
        stage_ms[name] = e0.elapsed_time(e1) / args.kernel_reps
    bm = byte_model(cfg.shape, info["grid"], C, M, d)
    # the dominant gridding kernel, timed alone (the spreading stage's tile
    # kernel without the partial-tile reduction)
    _lib.check(L.nufft_stage(plan.handle, _lib.KP_STAGE_SPREAD_TILES, 2, sp))
    torch.cuda.synchronize()
    e0.record(s)
    _lib.check(L.nufft_stage(plan.handle, _lib.KP_STAGE_SPREAD_TILES, args.kernel_reps, sp))
    e1.record(s)
    torch.cuda.synchronize()
    kernel_ms = {"interp": stage_ms["interp"], "spread": e0.elapsed_time(e1) / args.kernel_reps}
    dom = max(kernel_ms, key=lambda n: kernel_ms[n])
    achieved = bm[dom] / (kernel_ms[dom] / 1e3) / 1e9
    traffic = measured_traffic(dom)

    # the box's own copy bandwidth and shader clock, for context
    bw_copy = copy_bandwidth(dev)
    clock = gpu_clock()

    K = args.steps
    value = M * C * K / t_solve / 1e6
    result = {
        "metric": "NUFFT fwd+adj Msamples*coil/s; PDHG iters/s; % HBM roofline vs plain form",
        "value": round(value, 2),
        "unit": "Msamples*coil/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(t_solve / K * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": cfg.name, "image": list(cfg.shape), "coils": C, "samples_per_coil": M,
                   "oversamp": cfg.alpha, "kb_width": cfg.width, "reg": "l1-db4-4lev", "lambda": cfg.lam,
                   "precond": "mc", "iters": cfg.iters, "timed_iterations": K},
        "pdhg_iters_per_s": round(K / t_solve, 2),
        "tv_ms_per_step": round(t_tv / K * 1e3, 4),
        "nufft_pair_ms": round(t_pair * 1e3, 4),
        "nufft_pair_msamples_coil_per_s": round(M * C / t_pair / 1e6, 2),
        "nufft_pair_hbm_roofline_frac": round(bm["total"] / t_pair / 1e9 / HBM_PEAK_GBS, 4),
        "nufft_pair_byte_model_bytes": int(bm["total"]),
        "copy_bandwidth_gbs": round(bw_copy, 1),
        "nufft_pair_frac_of_copy_bandwidth": round(bm["total"] / t_pair / 1e9 / bw_copy, 4),
        "gpu_clock": clock,
        "parity": parity,
        "stage_ms": {k2: round(v, 4) for k2, v in stage_ms.items()},
        "setup_s": {"plan": round(t_plan, 4), "precond_mc": round(t_pre, 4), "lambda_max_30": round(t_lmax, 4)},
        "lambda_max": lmax_v,
        "wall_s_timed": round(t_wall, 4),
        "roofline": {"bound": "hbm", "kernel": KERNEL_NAMES[dom], "launch_ms": round(kernel_ms[dom], 4),
                     "algorithmic_bytes": int(bm[dom]), "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic},
    }
    ctx3 = None
    if not args.no_forms:
        log("3D preconditioner comparison")
        ctx3 = precond_comparison_3d(kp, plan, y, p, cfg, lmax_v, dev)
    plan.close()
    del plan
    if not args.no_forms:
        log("2D workloads")
        result["small_configs"] = bench_small_configs(kp, dev)
        result["batched"] = bench_batched(kp, dev)
        result["differentiable"] = bench_differentiable(kp, dev)
        result["context"] = bench_context(kp, dev)
        result["context"]["precond_comparison_3d"] = ctx3
    if oracle_t is not None:
        result.setdefault("context", {})["oracle_timings_2d"] = oracle_t
    if cpu is not None:
        result["cpu_baseline"] = cpu
    print(json.dumps(result), flush=True)


def ctypes_stream(s):
    import ctypes
    return ctypes.c_void_p(s.cuda_stream)


if __name__ == "__main__":
    main()
