"""Launch-shape autotuner of the batched ensemble (ensemble_run).

The tile of an ensemble launch has a workgroup shape (1024 threads with 4096
records of LDS, or 512 threads with 2048 records and two workgroups per
compute unit) and three knobs, each acting on one size class of systems:
  team    threads per system for systems of at most 4 team particles, which
          run 1024 / team to a workgroup;
  lds_max whole-workgroup systems up to this size stay in LDS for all steps;
  bucket  mean bucket of the systems streamed through global memory.
The tuner times every candidate tile on a copy of the positions for a few
steps (the result of a launch does not depend on the tile) and keeps the
fastest.  Results are cached in a JSON file keyed by the device
architecture, d, p, the kernel and the histogram of log2 N_s.
"""
from __future__ import annotations

import json
import os
import time

import numpy as np

from . import Ensemble, ensemble_run, ensemble_workspace_size

WGS = (1024, 512)  # threads per workgroup (4096 or 2048 records of LDS)
DEFAULT_CACHE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "autotune_cache.json")


def key_of(ens: Ensemble, arch: str) -> str:
    n = np.asarray(ens.sizes, np.int64)
    hist = np.bincount(np.floor(np.log2(n)).astype(np.int64), minlength=19)
    cls = ",".join(str(int(v)) for v in hist)
    return f"{arch}|d{ens.d}|p{ens.p}|k{ens.kernel}|n{len(n)}|{cls}"


def candidates(ens: Ensemble):
    nmax = int(np.max(ens.sizes))
    for wg in WGS:
        for team in (64, 128, 256, 512, 1024):
            if team > wg:
                continue
            for bucket in (wg, 2 * wg, 3 * wg):
                if (nmax + bucket - 1) // bucket > 256:
                    continue
                for lds_max in (2 * wg, 4 * wg):
                    yield dict(wg=wg, team=team, bucket=bucket, lds_max=lds_max)


def _arch():
    import torch
    p = torch.cuda.get_device_properties(0)
    return getattr(p, "gcnArchName", p.name).split(":")[0]


def tune(ens: Ensemble, x, probe_steps: int = 20, cache: str | None = DEFAULT_CACHE, retune: bool = False,
         log=None):
    """Fastest tile for this ensemble (dict of ensemble_run keyword
    arguments).  x: the positions a run would start from (not modified)."""
    import torch
    key = key_of(ens, _arch())
    table = {}
    if cache and os.path.exists(cache):
        with open(cache) as f:
            table = json.load(f)
        if key in table and not retune:
            return dict(table[key]["tile"])
    ws = torch.empty(max(ensemble_workspace_size(ens), 1), dtype=torch.uint8, device=x.device)
    xt = torch.empty_like(x)
    best, best_t, rows = None, float("inf"), []
    for tile in candidates(ens):
        xt.copy_(x)
        ensemble_run(ens, xt, 0, 2, ws=ws, graph=False, **tile)  # warm-up
        xt.copy_(x)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ensemble_run(ens, xt, 0, probe_steps, ws=ws, graph=False, **tile)
        dt = time.perf_counter() - t0
        rows.append((tile, dt))
        if log:
            log(f"tile {tile}: {dt * 1e3:.3f} ms for {probe_steps} steps")
        if dt < best_t:
            best, best_t = tile, dt
    if cache:
        table[key] = dict(tile=best, ms_per_step=best_t * 1e3 / probe_steps, probe_steps=probe_steps,
                          candidates=len(rows))
        tmp = cache + ".tmp"
        with open(tmp, "w") as f:
            json.dump(table, f, indent=1, sort_keys=True)
        os.replace(tmp, cache)
    return dict(best)
