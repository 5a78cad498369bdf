"""Schedule autotuner of the batched persistent launch.

The rollout tile of the kernels is fixed by the matrix instruction (32 rollouts
per wave); what varies with the workload is how work is handed to the
persistent workgroups: waves per workgroup (the tile units a workgroup runs
together and the LDS copy of the network they share), resident workgroups per
CU, and whether workgroups pull cost-sorted items from an atomic queue or walk
a static stride.  ``tune`` times every candidate schedule on the caller's own
instances with HIP events and returns the fastest; results are cached in a
JSON file keyed by the batch signature (network shape, precision, GPU
architecture, number of instances and coarse size totals).
"""
from __future__ import annotations

import json
import os
import time

import torch

from . import Batch, VOILA_BATCH_PLAN, VOILA_BATCH_UPDATE

CANDIDATES = [
    {"waves_per_block": 4, "blocks_per_cu": 0, "dynamic": True},
    {"waves_per_block": 8, "blocks_per_cu": 0, "dynamic": True},
    {"waves_per_block": 2, "blocks_per_cu": 0, "dynamic": True},
    {"waves_per_block": 4, "blocks_per_cu": 0, "dynamic": False},
    {"waves_per_block": 8, "blocks_per_cu": 0, "dynamic": False},
    {"waves_per_block": 4, "blocks_per_cu": 2, "dynamic": True},
    {"waves_per_block": 8, "blocks_per_cu": 1, "dynamic": True},
]


def cache_path() -> str:
    return os.environ.get("VOILA_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "voila", "autotune.json"))


def signature(instances, with_update: bool) -> str:
    m = instances[0]["model"]
    d = m.desc
    arch = torch.cuda.get_device_properties(m.device).gcnArchName.split(":")[0]
    nkh = sum(int(i["states"].shape[0]) * int(i["cands"].shape[0]) * int(i["cands"].shape[1]) for i in instances)
    n = sum(int(i["states"].shape[0]) for i in instances)
    bucket = lambda x: int(round(float(x) ** 0.25)) if x > 0 else 0  # noqa: E731  coarse size class
    return (f"{arch}|ds{d.d_s}-na{d.n_actions}-da{d.d_a}-dw{d.d_w}-w{int(d.trans[0][0].shape[0])}-"
            f"l{len(d.trans)}|{m.compute}|n{len(instances)}|nkh{bucket(nkh)}|N{bucket(n)}|u{int(with_update)}")


def _load_cache(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store_cache(path, cache):
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + f".tmp{os.getpid()}"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass


def time_schedule(instances, schedule, what, run_args, reps=3, warmup=1):
    """Mean milliseconds of one batch run under `schedule`."""
    b = Batch(instances, with_update=bool(what & VOILA_BATCH_UPDATE), **schedule)
    stream = torch.cuda.current_stream()
    for _ in range(warmup):
        b.run(what, **run_args)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        b.run(what, **run_args)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    b.close()
    return ms


def tune(instances, what=VOILA_BATCH_PLAN | VOILA_BATCH_UPDATE, run_args=None, reps=3, use_cache=True,
         candidates=None, verbose=False):
    """Fastest schedule for these instances: dict(schedule=..., ms=..., timings=[...], cached=bool)."""
    run_args = run_args or {}
    key = signature(instances, bool(what & VOILA_BATCH_UPDATE))
    path = cache_path()
    cache = _load_cache(path) if use_cache else {}
    if use_cache and key in cache:
        hit = dict(cache[key])
        hit["cached"] = True
        return hit
    timings = []
    for sch in candidates or CANDIDATES:
        t0 = time.perf_counter()
        ms = time_schedule(instances, sch, what, run_args, reps=reps)
        timings.append({"schedule": sch, "ms": ms})
        if verbose:
            print(f"[autotune] {sch} -> {ms:.3f} ms ({time.perf_counter() - t0:.1f} s)", flush=True)
    best = min(timings, key=lambda r: r["ms"])
    result = {"schedule": best["schedule"], "ms": best["ms"], "timings": timings, "key": key}
    if use_cache:
        cache[key] = result
        _store_cache(path, cache)
    result["cached"] = False
    return result
