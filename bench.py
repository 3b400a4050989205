"""Throughput of the RBM-1 step (arXiv:1812.10575, Sec. 2.1, Algorithm 1) on
one MI355X.

Workload: 3-D attraction-repulsion, K(x) = x/(|x|^2 + 0.01) - x, V = 0,
sigma = 0.1, dt = 1e-3, N = 2^24 particles, batch size p = 8, FP32 positions,
X0 ~ N(0, I3).  A "step" is one full RBM-1 step: random division, batch
forces and the Euler-Maruyama update of every particle.

Prints ONE JSON line.  `value` is particle-steps/s with the state already
resident in HBM.  `roofline` is for the kernel that takes the most time per
step, from HIP events recorded between the kernels inside the timed region.
`cpu_baseline` is the FP64 oracle timed on this host on one step of the same
workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "particle-steps/s at N=2^24,p=8; force MSE vs direct sum, plain vs control-variate"
HBM_PEAK_GBS = 8000.0
WORKLOAD = "attrep3d-n2^24-p8"
FIELDS = ("d", "kernel", "n", "p", "kparam", "beta", "sigma", "dt", "seed")


def phase_bytes(w: dict) -> dict:
    """Algorithmic HBM bytes per step of each kernel phase: the bucket scatter
    and the sort/force/update kernel each must read and write every particle
    record (d floats + id); the key-counting and scan phases read no particle
    data."""
    rec = 4 * (w["d"] + 1)
    n = w["n"]
    return {"scatter": 2 * rec * n, "split": 2 * rec * n, "sort": 2 * rec * n}


def cpu_baseline(w: dict, x0) -> dict:
    import numpy as np
    import oracle as ora
    o = ora.Params(d=w["d"], kernel=w["kernel"], kparam=w["kparam"], beta=w["beta"],
                   sigma=w["sigma"], dt=w["dt"], seed=w["seed"])
    x = x0.astype(np.float64)
    slots = np.arange(w["n"], dtype=np.uint32)
    t0 = time.perf_counter()
    ora.rbm_step(o, w["p"], 0, x, slots)
    t = time.perf_counter() - t0
    return {"value": w["n"] / t, "unit": "particle-steps/s", "cores": 1, "kind": "oracle",
            "sample": f"one full step of the same workload (N={w['n']}, p={w['p']}), "
                      f"single-threaded FP64 C oracle, {t:.1f} s"}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default=WORKLOAD)
    ap.add_argument("--p", type=int, default=None, help="override the batch size")
    ap.add_argument("--no-cpu-baseline", action="store_true")
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

    rbm.rbm_timing(ctx, args.steps)
    t_start = torch.cuda.Event(enable_timing=True)
    t_end = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t_start.record(stream)
    rbm.rbm_run(ctx, args.steps)
    t_end.record(stream)
    torch.cuda.synchronize()
    ms_total = t_start.elapsed_time(t_end)
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
                "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None, "kernel": dom,
                "algorithmic_bytes_per_launch": pb[dom]}
    else:
        roof = {"bound": "alu", "achieved": None, "peak": None, "unit": None, "frac": None,
                "traffic": None, "kernel": dom}
    roof["phase_ms"] = {k: round(v, 5) for k, v in phase_ms.items()}
    rec = 4 * (w["d"] + 1)
    roof["step_floor_frac"] = round(2 * rec * value / (HBM_PEAK_GBS * 1e9), 4)

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
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, x0)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
