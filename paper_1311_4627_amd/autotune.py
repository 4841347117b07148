"""Autotuner front end: cached launch configurations for plans.

The timing itself runs natively (hsd_autotune_plan in the C ABI: each
candidate configuration — per bin-count class the slot-group size and lane
layout, and the contraction's workgroup size — is timed as a whole
concurrent plan replay on the caller's batch, first replay discarded, the
rest averaged, one class at a time).  This module caches the winners as
JSON, keyed by the tuner, the device, the wavelength count, the bin counts of
the grains in each class and the batch size, so that a later run on the same
kind of batch applies them without timing again.
"""

from __future__ import annotations

import json
import os
from typing import Dict, List, Optional, Sequence

from . import hsd


def batch_key(ctx: "hsd.Context", grain_ids: Sequence[int], n_cells: int, device_name: str) -> str:
    bins = sorted(ctx.n_bins[g] for g in grain_ids)
    per_class = []
    for lo, hi in hsd.CLASS_BINS:
        per_class.append([b for b in bins if lo <= b <= hi])
    return json.dumps({"tuner": "plan", "device": device_name, "L": ctx.L, "n_cells": int(n_cells),
                       "bins": per_class}, sort_keys=True)


def _load(path: str) -> Dict[str, dict]:
    if path and os.path.exists(path):
        with open(path) as f:
            return json.load(f)
    return {}


MAX_TUNE_CELLS = 16384


def device_id(dev) -> str:
    """Architecture and compute-unit count of the device (the marketing name
    is not always reported, e.g. under a profiler)."""
    import torch
    p = torch.cuda.get_device_properties(dev)
    arch = getattr(p, "gcnArchName", "") or "unknown"
    return f"{arch.split(':')[0]}/{p.multi_processor_count}cu"


def tune(ctx: "hsd.Context", u, grain_ids: Sequence[int], cache_path: Optional[str] = None,
         runs: int = 4, force: bool = False) -> dict:
    """Apply the cached configuration of this batch's key, or time and cache
    it.  Batches larger than MAX_TUNE_CELLS cells are timed (and keyed) on
    their first MAX_TUNE_CELLS cells: by then every class has thousands of
    work items and the ranking of configurations no longer changes.
    Returns {"key", "cached", "cfg": [per class], "contract_waves", "records": [...]}."""
    if int(u.shape[0]) > MAX_TUNE_CELLS:
        u = u[:MAX_TUNE_CELLS]
    key = batch_key(ctx, grain_ids, int(u.shape[0]), device_id(u.device))
    cache = _load(cache_path) if cache_path else {}
    if not force and key in cache:
        entry = cache[key]
        for cls, cfg in enumerate(entry["cfg"]):
            ctx.hsd_set_class_cfg(cls, **cfg)
        ctx.hsd_set_contract_waves(entry.get("contract_waves", 4))
        return {"key": key, "cached": True, "cfg": entry["cfg"], "contract_waves": ctx.hsd_get_contract_waves(),
                "records": entry.get("records", [])}
    records: List[dict] = ctx.hsd_autotune_plan(u, grain_ids, runs=runs)
    cfg = [ctx.hsd_get_class_cfg(c) for c in range(hsd.N_CLASSES)]
    waves = ctx.hsd_get_contract_waves()
    if cache_path:
        cache[key] = {"cfg": cfg, "contract_waves": waves, "records": records}
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, cache_path)
    return {"key": key, "cached": False, "cfg": cfg, "contract_waves": waves, "records": records}
