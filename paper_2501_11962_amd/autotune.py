"""Autotuner for the neighbour-search geometry of a plan.

The pair kernels' cost depends on the x-y column width (it sets the cluster shape, the
candidate count and the in-cutoff fraction) and on the waves per workgroup.  `autotune`
times veff_grad on the caller's own system and path for each candidate setting (HIP
events on the library stream, median of a few calls) and caches the winner in a JSON
file keyed by the system's shape, so later plans for similar systems reuse it.

    opts = autotune(ctx, system_dict, R)          # R: (N, Q, 3) float64 CUDA tensor
    plan = Plan(System(ctx, system_dict), N, **opts)
"""
from __future__ import annotations

import json
import os

import numpy as np

DEFAULT_CANDIDATES = [dict(col_width=cw, waves=w) for cw in (0.35, 0.4, 0.45, 0.5)
                      for w in (2, 4)]
DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "mop_autotune.json")


def shape_key(system, N):
    """Cache key: atom count bucket, density, cutoff, box aspect and bead count."""
    box = np.asarray(system["box"], np.float64)
    Q = int(system["Q"])
    rho = Q / float(np.prod(box))
    qb = int(round(np.log2(max(Q, 1)) * 2))          # half-octave buckets of Q
    aspect = "x".join(f"{b / box.min():.2f}" for b in box)
    return f"q{qb}_rho{rho:.0f}_rc{float(system['rc']):.2f}_box{aspect}_n{int(N)}"


def load_cache(path=DEFAULT_CACHE):
    try:
        with open(path) as f:
            d = json.load(f)
        return d if isinstance(d, dict) else {}
    except (OSError, ValueError):
        return {}


def save_cache(d, path=DEFAULT_CACHE):
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = f"{path}.tmp{os.getpid()}"
    with open(tmp, "w") as f:
        json.dump(d, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def autotune(ctx, system, R, candidates=None, repeats=3, cache=DEFAULT_CACHE, force=False,
             log=None):
    """Best plan options (col_width, waves) for `system` with path R (CUDA tensor)."""
    import torch

    from . import Plan, System, veff_grad

    N = int(R.shape[0])
    key = shape_key(system, N)
    table = load_cache(cache) if cache else {}
    if not force and key in table:
        return dict(table[key]["opts"])
    cands = candidates or DEFAULT_CANDIDATES
    sysh = System(ctx, system)
    G = torch.empty_like(R)
    v = torch.empty(1, dtype=torch.float64, device=R.device)
    results = []
    for c in cands:
        plan = Plan(sysh, N, **c)
        veff_grad(plan, R, 0, 0.0, G, v)  # warm-up
        times = []
        for _ in range(repeats):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            veff_grad(plan, R, 0, 0.0, G, v)
            e1.record()
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1))
        ms = float(np.median(times))
        results.append((ms, c))
        if log:
            log(f"[autotune] {c}: {ms:.3f} ms")
        del plan
    ms, best = min(results, key=lambda t: t[0])
    if cache:
        table = load_cache(cache)
        table[key] = dict(opts=best, ms=ms, tried=[dict(c, ms=t) for t, c in results])
        save_cache(table, cache)
    return dict(best)
