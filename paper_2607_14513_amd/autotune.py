"""Autotuner for the batched encoder's work distribution.

Searches the gsbc_batch_tuning knobs -- 256-block rounds per work item,
persistent workgroups per compute unit, BC1 workgroup size, how the BC7
candidate groups are split over search kernels, and whether BC1 runs beside
BC7 on a second stream -- by timing replays of the captured batch on the
workload itself.  No setting changes the bits (every block is coded on its
own with fixed integer decisions), so the tuner only compares times.

The search is coordinate descent from the defaults: each knob in turn is
set to the value with the least median time while the others stay fixed;
two sweeps.  Results are cached in a JSON file keyed by device name,
compute-unit count and a hash of the workload shape (block counts and band
formats per scene).
"""
import hashlib
import json
import os
import time

import torch

from . import gsbc

SPACE = {
    "item_rounds": [1, 2, 4, 8],
    "wgs_per_cu": [0, 2, 4, 8, 12],
    "bc1_lanes": [64, 128, 256],
    "bc7_split": [0, 1, 2, 3],
    "concurrent": [0, 1],
}


def cache_path():
    return os.environ.get("GSBC_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "gsbc", "autotune.json"))


def workload_key(descs, params=None):
    p = params if params is not None else gsbc.default_params()
    h = hashlib.sha1()
    h.update(f"{p.refine_steps},{p.bc7_mode_mask}".encode())
    for d in descs:
        h.update(f"{d.blocks_per_stream}:{''.join(str(int(f)) for f in d.formats())};".encode())
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    return f"{props.name}|{props.multi_processor_count}|{h.hexdigest()[:16]}"


def _load_cache(path):
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(path, key, entry):
    data = _load_cache(path)
    data[key] = entry
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def time_batch(ctx, textures, descs, blocks, tuning, params=None, repeats=3):
    """Median device time (ms) of `repeats` replays of the captured batch."""
    ctx.encode_batch(textures, descs, blocks, params=params, tuning=tuning)   # capture (and warm)
    ts = []
    for _ in range(repeats):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(ctx.stream)
        ctx.encode_batch(textures, descs, blocks, params=params, tuning=tuning)
        e1.record(ctx.stream)
        e1.synchronize()
        ts.append(e0.elapsed_time(e1))
    ts.sort()
    return ts[len(ts) // 2]


def tune(ctx, textures, descs, blocks, params=None, repeats=3, sweeps=2, use_cache=True, log=None):
    """Best gsbc.BatchTuning for this batch (cached).  Returns (tuning, info)."""
    key = workload_key(descs, params)
    path = cache_path()
    if use_cache:
        hit = _load_cache(path).get(key)
        if hit:
            return gsbc.default_batch_tuning(**hit["tuning"]), dict(hit, cached=True)
    cur = gsbc.default_batch_tuning().as_dict()
    seen = {}

    def measure(cfg):
        k = tuple(sorted(cfg.items()))
        if k not in seen:
            seen[k] = time_batch(ctx, textures, descs, blocks, gsbc.default_batch_tuning(**cfg), params, repeats)
            if log:
                log(f"autotune {cfg} -> {seen[k]:.3f} ms")
        return seen[k]

    t0 = time.perf_counter()
    base = measure(cur)
    best = base
    for _ in range(sweeps):
        changed = False
        for knob, values in SPACE.items():
            for v in values:
                if v == cur[knob]:
                    continue
                cand = dict(cur, **{knob: v})
                t = measure(cand)
                if t < best:
                    best, cur, changed = t, cand, True
        if not changed:
            break
    info = {"tuning": cur, "ms": best, "default_ms": base, "configs_timed": len(seen),
            "search_s": round(time.perf_counter() - t0, 2), "key": key}
    if use_cache:
        _store(path, key, info)
    return gsbc.default_batch_tuning(**cur), dict(info, cached=False)
