"""Autotuning driver: pick tile shapes per dims class and the launch
schedule, and remember them.

The library's autotuner (mt_autotune) times every compiled tile shape of each
dims class present in a batch and checks that all of them give bit-identical
triplets.  This driver keeps the winners in a JSON cache keyed by GPU
architecture and dims class (path: $MT_AUTOTUNE_CACHE, default
~/.cache/mt_autotune.json), and re-applies cached choices without timing.
"""
from __future__ import annotations

import json
import os
from typing import Sequence

import torch

from . import mt

CLASS_NAMES = {0: "3d", 1: "2d", 2: "1d"}


def cache_path() -> str:
    return os.environ.get("MT_AUTOTUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "mt_autotune.json"))


def _arch(device) -> str:
    props = torch.cuda.get_device_properties(device)
    return getattr(props, "gcnArchName", props.name).split(":")[0]


def _load() -> dict:
    try:
        with open(cache_path()) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _shape_id(entry: dict, dims_class: int):
    for s in mt.tile_shapes():
        if s["dims_class"] == dims_class and [s["tx"], s["ty"], s["tz"]] == entry["tile"]:
            return s["id"]
    return None


def tune(fields: Sequence[torch.Tensor], reps: int = 3, force: bool = False) -> dict:
    """Select tile shapes for the classes in `fields` (cached per arch/class)."""
    dev = fields[0].device
    arch = _arch(dev)
    cache = _load()
    classes = {0 if len(f.shape) == 3 and f.shape[0] > 1 else 1 if len(f.shape) >= 2 and f.shape[-2] > 1 else 2
               for f in fields}
    pending = []
    for c in sorted(classes):
        key = f"{arch}|{CLASS_NAMES[c]}"
        sid = _shape_id(cache[key], c) if (key in cache and not force) else None
        if sid is None:
            pending.append(c)
        else:
            mt.set_tile_shape(c, sid)
    if pending:
        result = mt.autotune(fields, reps=reps)
        shapes = {s["id"]: s for s in mt.tile_shapes()}
        for c, (sid, ms) in result.items():
            s = shapes[sid]
            cache[f"{arch}|{CLASS_NAMES[c]}"] = {"tile": [s["tx"], s["ty"], s["tz"]], "threads": s["threads"],
                                                 "ms": ms}
        os.makedirs(os.path.dirname(cache_path()), exist_ok=True)
        with open(cache_path(), "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)
    return {CLASS_NAMES[c]: mt.get_tile_shape(c) for c in sorted(classes)}


def tune_schedule(fields: Sequence[torch.Tensor], reps: int = 3, force: bool = False) -> dict:
    """Select the launch schedule (XCD-aware tile order, merge workgroups per
    XCD) for this batch with the tile shapes in force; cached per arch and
    the batch's set of dims classes."""
    dev = fields[0].device
    classes = sorted({0 if len(f.shape) == 3 and f.shape[0] > 1 else 1 if len(f.shape) >= 2 and f.shape[-2] > 1
                      else 2 for f in fields})
    key = f"{_arch(dev)}|schedule|{'+'.join(CLASS_NAMES[c] for c in classes)}"
    cache = _load()
    if key in cache and not force:
        e = cache[key]
        mt.set_schedule(e["xcd_remap"], e["merge_groups"])
    else:
        r, g, ms = mt.autotune_schedule(fields, reps=reps)
        cache[key] = {"xcd_remap": r, "merge_groups": g, "ms": ms}
        os.makedirs(os.path.dirname(cache_path()), exist_ok=True)
        with open(cache_path(), "w") as fh:
            json.dump(cache, fh, indent=1, sort_keys=True)
    r, g = mt.get_schedule()
    return {"xcd_remap": r, "merge_groups": g}
