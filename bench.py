"""Throughput of the RBM-1 step (arXiv:1812.10575, Sec. 2.1, Algorithm 1) on
one MI355X.

Workload: 3-D attraction-repulsion, K(x) = x/(|x|^2 + 0.01) - x, V = 0,
sigma = 0.1, dt = 1e-3, N = 2^24 particles, batch size p = 8, FP32 positions,
X0 ~ N(0, I3).  A "step" is one full RBM-1 step: random division, batch
forces and the Euler-Maruyama update of every particle.

Prints ONE JSON line.  `value` is particle-steps/s with the state already
resident in HBM.  `roofline` is for the kernel that takes the most time per
step, from HIP events recorded between the kernels in a second timed run of
the same steps (`events_ms_per_step`: that run's time per step; the events
add to it, so `value` and `ms_per_step` come from the first run, without
them).
`cpu_baseline` is the FP64 oracle timed on this host on whole steps of the
same workload, on all the host threads the process may use and on one.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-steps/s at N=2^24,p=8; force MSE vs direct sum, plain vs control-variate"
HBM_PEAK_GBS = 8000.0
WORKLOAD = "attrep3d-n2^24-p8"
FIELDS = ("d", "kernel", "n", "p", "kparam", "beta", "sigma", "dt", "seed")
CALIB_COPY_BYTES = 256 << 20


def phase_bytes(w: dict) -> dict:
    """Algorithmic HBM bytes per step of each kernel phase: the bucket scatter
    and the sort/force/update kernel each must read and write every particle
    record (d floats + id); the key-counting and scan phases read no particle
    data."""
    rec = 4 * (w["d"] + 1)
    n = w["n"]
    return {"scatter": 2 * rec * n, "split": 2 * rec * n, "sort": 2 * rec * n}


TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "rbm_step_traffic_attrep3d_n2e24_p8.md")
STEP_SOURCES = ("rbm_kernels.hip", "rbm_device.hpp", "rbm_plan.hpp")


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE, calibrated by a plain copy), or None when the
    step kernel sources have changed since the counters were taken."""
    import hashlib
    import re
    if not os.path.exists(TRAFFIC_SUMMARY):
        return None
    h = hashlib.sha256()
    for fn in STEP_SOURCES:
        with open(os.path.join(ROOT, "paper_1812_10575_amd", "csrc", fn), "rb") as f:
            h.update(f.read())
    with open(TRAFFIC_SUMMARY) as f:
        for line in f:
            m = re.match(r"traffic-record: kernel=(\S+) bytes_per_launch=(\d+) source_sha256=([0-9a-f]+)", line)
            if m and m.group(1) == kernel and m.group(3) == h.hexdigest():
                return int(m.group(2))
    return None


def p_sweep(args, w, x0) -> dict:
    """Throughput of the same workload at other batch sizes (10 timed steps each)."""
    import torch
    import paper_1812_10575_amd as rbm
    out = {}
    xt = torch.from_numpy(x0).cuda()
    for p in (2, 4, 8, 16, 32):
        prm = rbm.Params(**{**{k: w[k] for k in FIELDS}, "p": p})
        ctx = rbm.rbm_init(prm, xt)
        rbm.rbm_run(ctx, 3)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rbm.rbm_run(ctx, 10)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        rbm.rbm_check(ctx)
        out[str(p)] = round(w["n"] * 10 / dt, -6)
        del ctx
    return {"unit": "particle-steps/s", "steps": 10, "value": out}


# FP32 operations per ordered pair of the attraction-repulsion kernel in 3-D:
# difference 3, squared norm 3 FMA (6), + a 1, reciprocal 1, - 1 1,
# scaled accumulation 3 FMA (6)
DIRECT_FLOPS_PER_PAIR = 18
FP32_PEAK_TFLOPS = 157.3


def direct_rate(w, x0) -> dict:
    """The exact O(N^2) force (direct_forces) at N = 2^20 for a subset of
    2^16 target particles: pair evaluations per second and FP32 FLOP/s."""
    import numpy as np
    import torch
    import paper_1812_10575_amd as rbm
    n = 1 << 20
    prm = rbm.Params(**{**{k: w[k] for k in FIELDS}, "n": n})
    x = torch.from_numpy(np.ascontiguousarray(x0[:n])).cuda()
    ids = torch.arange(0, n, 16, dtype=torch.int32, device="cuda")
    rbm.direct_forces(prm, x, ids)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    reps = 3
    for _ in range(reps):
        rbm.direct_forces(prm, x, ids)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    pairs = ids.numel() * (n - 1)
    tf = pairs * DIRECT_FLOPS_PER_PAIR / dt / 1e12
    return {"n": n, "targets": ids.numel(), "seconds": round(dt, 5), "pairs_per_s": pairs / dt,
            "roofline": {"bound": "fp32", "achieved": round(tf, 2), "peak": FP32_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": round(tf / FP32_PEAK_TFLOPS, 4), "flops_per_pair": DIRECT_FLOPS_PER_PAIR}}


def host_threads() -> int:
    """Host threads this process may use: the CPUs it is allowed to run on,
    capped by OMP_NUM_THREADS when that is set (the GPU machine sets it to its
    CPU share)."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


def cpu_baseline(w: dict, x0) -> dict:
    """The FP64 oracle on this host: whole steps of the same workload on all
    the host threads this process may use (the value), then on one thread,
    each repeated until a few seconds have passed.  The oracle's results do
    not depend on the thread count."""
    import numpy as np
    import oracle as ora
    o = ora.Params(d=w["d"], kernel=w["kernel"], kparam=w["kparam"], beta=w["beta"],
                   sigma=w["sigma"], dt=w["dt"], seed=w["seed"])

    def timed(threads: int, min_s: float):
        used = ora.set_threads(threads)
        x = x0.astype(np.float64)
        slots = np.arange(w["n"], dtype=np.uint32)
        steps = 0
        t0 = time.perf_counter()
        while True:
            x, slots = ora.rbm_step(o, w["p"], steps, x, slots)
            steps += 1
            t = time.perf_counter() - t0
            if t >= min_s:
                return w["n"] * steps / t, steps, t, used

    nt = host_threads()
    v_all, s_all, t_all, used = timed(nt, 8.0)
    v_one, s_one, t_one, _ = timed(1, 8.0)
    # the direct sum of eq. (1.2) on the same kernel at N = 2^20: 2^12 of the
    # targets on all threads, the whole step extrapolated from them
    import rbm_inputs
    nd, nt_ids = 1 << 20, 1 << 12
    xd = rbm_inputs.workload(w["init"], nd, w["seed"]).astype(np.float64)
    ora.set_threads(nt)
    t0 = time.perf_counter()
    ora.direct_forces(o, xd, np.arange(nt_ids, dtype=np.uint32))
    td = time.perf_counter() - t0
    return {"value": v_all, "unit": "particle-steps/s", "cores": used, "kind": "oracle",
            "sample": f"{s_all} full steps of the same workload (N={w['n']}, p={w['p']}) on {used} threads "
                      f"(OpenMP over particles, parallel merge sort of the keys), {t_all:.1f} s; "
                      f"single thread: {s_one} steps, {t_one:.1f} s",
            "single_thread": {"value": v_one, "cores": 1, "steps": s_one, "seconds": round(t_one, 2)},
            "os_cpu_count": os.cpu_count(),
            "direct_sum": {"n": nd, "targets": nt_ids, "seconds": round(td, 3), "cores": used,
                           "pairs_per_s": nt_ids * (nd - 1) / td,
                           "step_seconds_extrapolated": round(td * nd / nt_ids, 1)}}


def force_mse(args) -> dict:
    """Force MSE against the direct sum, plain RBM-1 vs the learned control
    variate, on the Gaussian workload at N = 2^22, p = 2.  The networks are
    trained on pairs drawn from 16 snapshots of the run's own plain
    trajectory; the MSE is averaged over 16 divisions on a fixed subset of
    2^16 particles whose exact forces come from the direct sum."""
    import numpy as np
    import torch

    import paper_1812_10575_amd as rbm
    import rbm_inputs

    w = rbm_inputs.params_of("gauss2d-n2^22-p2")
    n = w["n"]
    mk = lambda **o: rbm.Params(**{k: o.get(k, w[k]) for k in FIELDS}, cv=o.get("cv", 0))
    x0 = torch.from_numpy(rbm_inputs.workload(w["init"], n, w["seed"])).cuda()
    plain = rbm.rbm_init(mk(), x0)
    snaps = []
    for _ in range(16):
        rbm.rbm_run(plain, args.mse_snap_every)
        snaps.append(rbm.rbm_positions(plain).clone())
    snap = torch.stack(snaps)
    x = snaps[-1]
    cvctx = rbm.rbm_init(mk(cv=1), x)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    losses = rbm.cv_train(cvctx, snap, args.train_steps, args.train_batch, lr=args.lr)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    ids = torch.from_numpy(np.random.default_rng(7).choice(n, 1 << 16, replace=False).astype(np.int32)).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fdir, m2 = rbm.direct_moments(mk(), x, ids)
    torch.cuda.synchronize()
    pair_rate = ids.numel() * (n - 1) / (time.perf_counter() - t0)  # Gaussian pairs per second, d = 2
    # Lemma 3.1: E|F^RBM - F|^2 = (1/(p-1) - 1/(N-1)) Lambda_i,
    # Lambda_i = (N-1)/(N-2) (m2_i - |F_i|^2)
    f64 = fdir.double()
    lam = (n - 1) / (n - 2) * (m2.double() - (f64 * f64).sum(dim=1))
    pred_plain = float(((1.0 / (w["p"] - 1) - 1.0 / (n - 1)) * lam).mean())

    def mse_of(ctx):
        acc = 0.0
        for m in range(16):
            f = rbm.rbm_forces(ctx, 100000 + m)
            acc += float(rbm.rbm_force_sqerr(f, ids, fdir).cpu()[0])
        return acc / (16 * ids.numel())

    def rate_of(ctx, steps=20):
        rbm.rbm_run(ctx, 3)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        rbm.rbm_run(ctx, steps)
        e1.record()
        torch.cuda.synchronize()
        return n * steps / (e0.elapsed_time(e1) * 1e-3)

    mse_plain = mse_of(rbm.rbm_init(mk(), x))
    mse_cv = mse_of(cvctx)
    gain = mse_plain / mse_cv
    # Lemma 3.1: MSE(p) = (1/(p-1) - 1/(N-1)) Lambda, so equal MSE needs
    # 1/(p'-1) - 1/(N-1) = (1 - 1/(N-1)) / gain
    pp_equal = int(math.ceil(1.0 + 1.0 / ((1.0 - 1.0 / (n - 1)) / gain + 1.0 / (n - 1))))
    pp = max(2, min(pp_equal, 64))
    plain_pp = rbm.rbm_init(mk(p=pp), x)
    mse_pp = mse_of(plain_pp)
    out = {"workload": "gauss2d-n2^22-p2", "n": n, "p": 2, "subset": int(ids.numel()), "divisions": 16,
           "mse_plain": mse_plain, "mse_plain_lemma_3_1": pred_plain, "mse_cv": mse_cv, "gain": gain,
           "train": {"pairs": args.train_steps * args.train_batch, "adam_steps": args.train_steps,
                     "batch": args.train_batch, "seconds": round(t_train, 3),
                     "loss_first": float(losses[:16].mean().cpu()), "loss_last": float(losses[-16:].mean().cpu())},
           "equal_mse": {"p_equal": pp_equal,
                         # plain RBM-1 at p_equal needs (p_equal - 1) / 2 pair evaluations per
                         # particle at the very least; at the direct sum's pair rate on this
                         # GPU that bounds its throughput from above
                         "plain_bound_at_p_equal": 2.0 * pair_rate / max(pp_equal - 1, 1),
                         "pair_rate": pair_rate,
                         "p_plain": pp, "mse_plain": mse_pp,
                         "plain_particle_steps_per_s": rate_of(plain_pp),
                         "cv_particle_steps_per_s": rate_of(cvctx),
                         "plain_p2_particle_steps_per_s": rate_of(rbm.rbm_init(mk(), x))}}
    return out


def mse_sweep(args) -> dict:
    """Force MSE of plain RBM-1 against the direct sum on the headline
    system's kernel (3-D attraction-repulsion, a = 0.01) at N = 2^20, for
    p = 2 .. 32: the mean over 16 divisions and a fixed subset of 2^14
    particles of |F^RBM - F|^2, beside the Lemma 3.1 prediction
    (1/(p-1) - 1/(N-1)) Lambda_i from the direct sum's moments at the same
    positions (the headline's initial law, X0 ~ N(0, I3))."""
    import numpy as np
    import torch
    import paper_1812_10575_amd as rbm
    from paper_1812_10575_amd import measure
    import rbm_inputs
    w = rbm_inputs.params_of("attrep3d-n2^24-p8", n=1 << 20)
    n = w["n"]
    x = torch.from_numpy(rbm_inputs.workload(w["init"], n, w["seed"])).cuda()
    ids = torch.from_numpy(np.random.default_rng(9).choice(n, 1 << 14, replace=False).astype(np.int32)).cuda()
    prm = rbm.Params(**{k: w[k] for k in FIELDS})
    fdir, m2 = rbm.direct_moments(prm, x, ids)
    f64 = fdir.double()
    lam = ((n - 1) / (n - 2) * (m2.double() - (f64 * f64).sum(dim=1))).cpu().numpy()
    out = {}
    for p in (2, 4, 8, 16, 32):
        ctx = rbm.rbm_init(rbm.Params(**{**{k: w[k] for k in FIELDS}, "n": n, "p": p}), x)
        acc = 0.0
        for m in range(16):
            acc += float(rbm.rbm_force_sqerr(rbm.rbm_forces(ctx, 1000 + m), ids, fdir).cpu()[0])
        mse = acc / (16 * ids.numel())
        pred = float(np.mean(measure.lemma_3_1_mse(p, n, lam)))
        out[str(p)] = {"mse": mse, "lemma_3_1": pred, "ratio": mse / pred}
    return {"workload": "attrep3d-n2^20", "n": n, "subset": int(ids.numel()), "divisions": 16, "p": out}


def ensemble_rate(args) -> dict:
    """The batched ensemble: 4096 independent 2-D Gaussian systems, N_s
    log-uniform on [64, 65536], p = 4, 500 steps in one persistent launch
    with the tile from the autotuner.

    The value is the direct launch timed with HIP events on its stream.  The
    same call in graph form (recorded, instantiated, replayed once) is timed
    beside it and reported as a cost, not a gain: the graph holds one node.
    Roofline: a streamed system (N_s > lds_max) moves each particle's 12-byte
    record and 4-byte PERM word in and out of HBM once per step (32 B per
    particle-step, plus 8 B of positions in and out per call); an LDS-resident
    system touches HBM only to load and store its positions once per call
    (16 B per particle and call).  Each class is also run alone, as an
    ensemble of its own systems, for its own rate."""
    import numpy as np
    import torch
    import paper_1812_10575_amd as rbm
    from paper_1812_10575_amd import autotune
    import rbm_inputs
    E = rbm_inputs.ENSEMBLE
    n, keys, x0 = rbm_inputs.ensemble()
    steps = E["steps"]

    def make(sizes, seeds):
        return rbm.Ensemble(d=E["d"], kernel=E["kernel"], p=E["p"], sizes=sizes, seeds=seeds, kparam=E["kparam"],
                            beta=E["beta"], sigma=E["sigma"], dt=E["dt"])

    ens = make(n, keys)
    x = torch.from_numpy(x0).cuda()
    t0 = time.perf_counter()
    tile = autotune.tune(ens, x, retune=args.retune)
    t_tune = time.perf_counter() - t0
    stream = torch.cuda.current_stream()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)

    def timed(e, xs, graph):
        ws = torch.empty(rbm.ensemble_workspace_size(e), dtype=torch.uint8, device=xs.device)
        xr = xs.clone()
        rbm.ensemble_run(e, xr, 0, 5, ws=ws, graph=graph, **tile)  # warm-up
        xr.copy_(xs)
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        ev0.record(stream)
        rbm.ensemble_run(e, xr, 0, steps, ws=ws, graph=graph, **tile)
        ev1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - w0
        assert bool(torch.isfinite(xr).all())
        return ev0.elapsed_time(ev1) * 1e-3, wall

    sec, wall = timed(ens, x, False)
    sec_g, wall_g = timed(ens, x, True)
    tot = int(n.sum())
    lds_max = int(tile.get("lds_max") or 0) or 4 * int(tile.get("wg") or 1024)
    streamed = n > lds_max
    n_str, n_res = int(n[streamed].sum()), int(n[~streamed].sum())
    bytes_str = n_str * (16 + 32 * steps)
    bytes_res = n_res * 16
    ach = (bytes_str + bytes_res) / sec / 1e9
    off = np.concatenate([[0], np.cumsum(n)])
    classes = {}
    for name, mask, bps in (("streamed", streamed, 32.0), ("lds_resident", ~streamed, 16.0 / steps)):
        idx = np.nonzero(mask)[0]
        rows = np.concatenate([np.arange(off[i], off[i + 1]) for i in idx])
        xs = torch.from_numpy(np.ascontiguousarray(x0[rows])).cuda()
        s_c, _ = timed(make(n[idx], keys[idx]), xs, False)
        pc = int(n[idx].sum())
        c = {"systems": int(len(idx)), "particles": pc, "seconds_alone": round(s_c, 4),
             "particle_steps_per_s_alone": pc * steps / s_c, "hbm_bytes_per_particle_step": round(bps, 4)}
        if name == "streamed":
            a_c = pc * (16 + 32 * steps) / s_c / 1e9
            c.update({"achieved_GBps_alone": round(a_c, 1), "frac_alone": round(a_c / HBM_PEAK_GBS, 4)})
        classes[name] = c
    return {"workload": E["name"], "systems": int(len(n)), "particles": tot, "steps": steps, "p": E["p"],
            "seconds": round(sec, 4), "value": tot * steps / sec, "unit": "particle-steps/s",
            "roofline": {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(ach / HBM_PEAK_GBS, 4), "algorithmic_bytes": bytes_str + bytes_res},
            "classes": classes,
            "graph": {"seconds": round(sec_g, 4), "wall_seconds": round(wall_g, 4),
                      "direct_wall_seconds": round(wall, 4)},
            "tile": tile, "tune_seconds": round(t_tune, 2),
            "launch": "one persistent kernel, direct launch, HIP events on its stream"}


def dyson_split(args) -> dict:
    """Sec. 4.2's Dyson Brownian motion by the splitting with the exact pair
    flow (K = 1/x, p = 2, beta = 1, sigma = 1/sqrt(N), tau = 1e-3), N = 2^20
    from the radius-2 semicircle to t = 5: throughput and the KS distance to
    the analytic density at the end."""
    import numpy as np
    import torch
    import paper_1812_10575_amd as rbm
    from paper_1812_10575_amd import measure
    import rbm_inputs
    w = rbm_inputs.params_of("dysonsplit1d-n2^20-p2")
    prm = rbm.Params(**{k: w[k] for k in FIELDS})
    ctx = rbm.rbm_init(prm, torch.from_numpy(rbm_inputs.workload(w["init"], w["n"], w["seed"])).cuda())
    rbm.rbm_run(ctx, 10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rbm.rbm_run(ctx, w["steps"] - 10)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    rbm.rbm_check(ctx)
    x = rbm.rbm_positions(ctx).cpu().numpy()[:, 0].astype(np.float64)
    t_end = w["steps"] * w["dt"]
    radius = measure.dyson_radius(t_end)
    ks = measure.ks_distance(x, lambda v: measure.semicircle_cdf(v, radius))
    return {"workload": "dysonsplit1d-n2^20-p2", "n": w["n"], "steps": w["steps"], "t": t_end,
            "value": w["n"] * (w["steps"] - 10) / dt, "unit": "particle-steps/s",
            "ks_vs_analytic": ks, "m2": measure.second_moment(x), "m2_analytic": radius * radius / 4}


def wealth(args) -> dict:
    """Sec. 5's wealth model (kappa = D = 1, quadratic trading, p = 2, exact
    pair flow and exact multiplicative noise, tau = 1e-3), N = 2^20 from
    |N(0,1)| to T = 3: throughput and the KS distance to the inverse Gamma
    law of shape 2 and scale the mean wealth."""
    import numpy as np
    import torch
    import paper_1812_10575_amd as rbm
    from paper_1812_10575_amd import measure
    import rbm_inputs
    w = rbm_inputs.params_of("wealth1d-n2^20-p2")
    prm = rbm.Params(**{k: w[k] for k in FIELDS})
    ctx = rbm.rbm_init(prm, torch.from_numpy(rbm_inputs.workload(w["init"], w["n"], w["seed"])).cuda())
    rbm.rbm_run(ctx, 10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rbm.rbm_run(ctx, w["steps"] - 10)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    rbm.rbm_check(ctx)
    y = rbm.rbm_positions(ctx).cpu().numpy()[:, 0].astype(np.float64)
    eta = float(y.mean())
    return {"workload": "wealth1d-n2^20-p2", "n": w["n"], "steps": w["steps"], "t": w["steps"] * w["dt"],
            "value": w["n"] * (w["steps"] - 10) / dt, "unit": "particle-steps/s",
            "mean_wealth": eta, "ks_vs_inverse_gamma": measure.ks_distance(y, lambda v: measure.inverse_gamma_cdf(v, 2.0, eta))}


def rbmr(args) -> dict:
    """Sec. 4.2's Dyson Brownian motion by RBM-r (Sec. 2.2): one random pair
    per iteration, N/2 iterations per dt = 1e-3, exact pair flow, N = 2^20
    from the radius-2 semicircle to t = 5: throughput in particle updates
    per second (p per iteration; N/p iterations make one particle-step each)
    and the KS distance to the analytic density at the end."""
    import numpy as np
    import torch
    import paper_1812_10575_amd as rbm
    from paper_1812_10575_amd import measure
    import rbm_inputs
    w = rbm_inputs.params_of("dysonrbmr1d-n2^20-p2")
    prm = rbm.Params(**{k: w[k] for k in FIELDS})
    x = torch.from_numpy(rbm_inputs.workload(w["init"], w["n"], w["seed"])).cuda()
    ws = torch.empty(rbm.rbmr_workspace_size(prm), dtype=torch.uint8, device="cuda")
    per = w["n"] // w["p"]
    rbm.rbmr_run(prm, x, 0, 10 * per, ws=ws)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rbm.rbmr_run(prm, x, 10 * per, (w["steps"] - 10) * per, ws=ws)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    y = x.cpu().numpy()[:, 0].astype(np.float64)
    t_end = w["steps"] * w["dt"]
    radius = measure.dyson_radius(t_end)
    return {"workload": "dysonrbmr1d-n2^20-p2", "n": w["n"], "iterations": w["steps"] * per, "t": t_end,
            "value": (w["steps"] - 10) * per * w["p"] / dt, "unit": "particle-steps/s",
            "us_per_window": 1e6 * dt / (w["steps"] - 10),
            "ks_vs_analytic": measure.ks_distance(y, lambda v: measure.semicircle_cdf(v, radius)),
            "m2": measure.second_moment(y), "m2_analytic": radius * radius / 4}


def hamilton(args) -> dict:
    """Sec. 4.1's second-order example (x'' = F with K = x/(1+x^2), p = 2,
    Verlet, tau = 2^-7, T = 1) at N = 2^20 from semicircle positions and
    N(0, 1) velocities: throughput.  At N = 2^14: the RMS position error at
    T = 1 against the fully coupled Verlet solution (tau = 2^-11) for
    tau = 2^-4 .. 2^-8 (2 seeds each) and its log-log slope (Theorem A.1
    bounds it by C(T) sqrt(tau/(p-1)))."""
    import numpy as np
    import torch
    import paper_1812_10575_amd as rbm
    from paper_1812_10575_amd import measure
    import rbm_inputs
    w = rbm_inputs.params_of("hamilton1d-n2^20-p2")
    prm = rbm.Params(**{k: w[k] for k in FIELDS})
    ctx = rbm.rbm_init(prm, torch.from_numpy(rbm_inputs.workload(w["init"], w["n"], w["seed"])).cuda())
    rbm.rbm_run(ctx, 10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rbm.rbm_run(ctx, w["steps"] - 10)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    rbm.rbm_check(ctx)
    n = 1 << 14
    ws = dict(w, n=n, dt=2.0 ** -11)
    x0 = rbm_inputs.workload(w["init"], n, w["seed"])
    xr = torch.from_numpy(x0).cuda()
    pr = rbm.Params(**{k: ws[k] for k in FIELDS})
    for m in range(2 ** 11):
        xr = rbm.direct_step(pr, xr, m)
    xr = xr.cpu().numpy()[:, 0].astype(np.float64)
    taus = [2.0 ** -k for k in (4, 5, 6, 7, 8)]
    errs = []
    for tau in taus:
        e2 = []
        for seed in (1, 2):
            c = rbm.rbm_init(rbm.Params(**{k: dict(ws, dt=tau, seed=seed)[k] for k in FIELDS}),
                             torch.from_numpy(x0).cuda())
            rbm.rbm_run(c, int(round(1.0 / tau)))
            e2.append(measure.rms_error(rbm.rbm_positions(c).cpu().numpy()[:, 0], xr) ** 2)
        errs.append(math.sqrt(float(np.mean(e2))))
    slope = measure.loglog_slope(taus, errs)
    return {"workload": "hamilton1d-n2^20-p2", "n": w["n"], "steps": w["steps"], "t": w["steps"] * w["dt"],
            "value": w["n"] * (w["steps"] - 10) / dt, "unit": "particle-steps/s",
            "error_n": n, "error_taus": taus, "rms_position_error": errs, "slope": slope}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--repeats", type=int, default=5, help="timed calls of --steps steps; the median is the value")
    ap.add_argument("--workload", default=WORKLOAD)
    ap.add_argument("--p", type=int, default=None, help="override the batch size")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mse", action="store_true", help="skip the force MSE parts (control variate, p sweep)")
    ap.add_argument("--train-steps", type=int, default=4096)
    ap.add_argument("--train-batch", type=int, default=16384)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--mse-snap-every", type=int, default=25)
    ap.add_argument("--no-ensemble", action="store_true", help="skip the batched-ensemble part")
    ap.add_argument("--no-sweep", action="store_true", help="skip the p sweep and the direct-sum rate")
    ap.add_argument("--retune", action="store_true", help="ignore the ensemble autotune cache")
    ap.add_argument("--calib-copy", action="store_true",
                    help="run one plain 256 MiB device-to-device copy first (a reference for HBM byte counters)")
    ap.add_argument("--only", choices=("dyson_split", "wealth", "hamilton", "rbmr", "ensemble", "force_mse",
                                        "mse_sweep"),
                    default=None,
                    help="run one extra workload alone and print its JSON object (for profiling it)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported "
              "(the path has no multi-GPU mode)", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_1812_10575_amd as rbm
    import rbm_inputs

    if not os.path.exists(rbm.LIB_PATH):
        from paper_1812_10575_amd import build as hip_build
        hip_build.build()

    if args.calib_copy:
        torch.cuda.set_device(torch.device("cuda:0"))
        a = torch.ones(CALIB_COPY_BYTES // 4, dtype=torch.float32, device="cuda:0")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    if args.only is not None:
        torch.cuda.set_device(torch.device("cuda:0"))
        fn = {"dyson_split": dyson_split, "wealth": wealth, "hamilton": hamilton, "rbmr": rbmr,
              "ensemble": ensemble_rate, "force_mse": force_mse, "mse_sweep": mse_sweep}[args.only]
        print(json.dumps({args.only: fn(args)}), flush=True)
        return 0

    over = {} if args.p is None else {"p": args.p}
    w = rbm_inputs.params_of(args.workload, **over)
    prm = rbm.Params(**{k: w[k] for k in FIELDS})
    x0 = rbm_inputs.workload(w["init"], w["n"], w["seed"])
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ctx = rbm.rbm_init(prm, torch.from_numpy(x0).to(dev))
    stream = torch.cuda.current_stream()

    rbm.rbm_run(ctx, args.warmup)
    rbm.rbm_check(ctx)
    torch.cuda.synchronize()

    # the timed steps: one rbm_run call of K steps, repeated (the run goes
    # on from where the last call stopped); the median call is the value
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)

    def timed_call(k):
        torch.cuda.synchronize()
        t_start.record(stream)
        rbm.rbm_run(ctx, k)
        t_end.record(stream)
        torch.cuda.synchronize()
        return t_start.elapsed_time(t_end)

    runs = [timed_call(args.steps) for _ in range(args.repeats)]
    ms_total = sorted(runs)[len(runs) // 2]
    # a call's first step also scatters the records into their first coarse
    # buckets (later steps find them there): the cost of a one-step call,
    # and the per-step cost inside a call without it
    one = sorted(timed_call(1) for _ in range(5))[2]
    rbm.rbm_check(ctx)

    # the same K steps again with the library's HIP events between its
    # kernels: the per-kernel durations of the roofline (the events
    # themselves add to the step, so `value` comes from the run above)
    rbm.rbm_timing(ctx, args.steps)
    torch.cuda.synchronize()
    t_start.record(stream)
    rbm.rbm_run(ctx, args.steps)
    t_end.record(stream)
    torch.cuda.synchronize()
    ms_total_ev = t_start.elapsed_time(t_end)
    phase_ms, nrec = rbm.rbm_phase_times(ctx)
    rbm.rbm_timing(ctx, 0)
    rbm.rbm_check(ctx)

    ms_step = ms_total / args.steps
    value = w["n"] * args.steps / (ms_total * 1e-3)
    pb = phase_bytes(w)
    dom = max(phase_ms, key=phase_ms.get)
    if dom in pb:
        ach = pb[dom] / (phase_ms[dom] * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": measured_traffic(dom), "kernel": dom,
                "algorithmic_bytes_per_launch": pb[dom]}
    else:
        roof = {"bound": "alu", "achieved": None, "peak": None, "unit": None, "frac": None,
                "traffic": None, "kernel": dom}
    # every data pass against the same peak (the split and the fused sort
    # are the two memory passes of a fused step)
    roof["passes"] = {k: {"achieved": round(pb[k] / (phase_ms[k] * 1e-3) / 1e9, 1),
                          "frac": round(pb[k] / (phase_ms[k] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                          "traffic": measured_traffic(k)}
                      for k in ("split", "sort") if k in pb and phase_ms.get(k, 0.0) > 0.0}
    roof["phase_ms"] = {k: round(v, 5) for k, v in phase_ms.items()}
    roof["events_ms_per_step"] = round(ms_total_ev / args.steps, 5)
    rec = 4 * (w["d"] + 1)
    roof["step_floor_frac"] = round(2 * rec * value / (HBM_PEAK_GBS * 1e9), 4)
    timing = {"repeats": args.repeats, "ms_per_call": [round(v, 4) for v in runs],
              "ms_per_step_min": round(min(runs) / args.steps, 5), "ms_per_step_max": round(max(runs) / args.steps, 5),
              "ms_one_step_call": round(one, 5)}
    if args.steps > 1:
        timing["ms_per_step_after_first"] = round((ms_total - one) / (args.steps - 1), 5)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "particle-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic: X0 ~ N(0, I3) (numpy Philox, seed 1); method randomness from Philox4x32-10",
        "config": {"workload": args.workload, "d": w["d"], "n": w["n"], "p": w["p"],
                   "kernel": ["-x exp(-|x|^2)", "x/(|x|^2+a)", "x/(|x|^2+a)-x"][w["kernel"]],
                   "a": w["kparam"], "beta": w["beta"], "sigma": w["sigma"], "dt": w["dt"]},
        "roofline": roof,
        "timing": timing,
    }
    if not args.no_sweep:
        out["p_sweep"] = p_sweep(args, w, x0)
        out["direct"] = direct_rate(w, x0)
    if not args.no_mse:
        out["force_mse"] = force_mse(args)
        out["mse_sweep"] = mse_sweep(args)
    if not args.no_ensemble:
        out["ensemble"] = ensemble_rate(args)
    if not args.no_sweep:
        out["dyson_split"] = dyson_split(args)
        out["wealth"] = wealth(args)
        out["hamilton"] = hamilton(args)
        out["rbmr"] = rbmr(args)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, x0)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
