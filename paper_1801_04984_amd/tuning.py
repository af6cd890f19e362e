"""Tile-shape cache for the operator apply.

`biot_autotune` (C ABI) times every tile variant of the apply on the handle's
own problem and selects the fastest per precision; all variants produce
bitwise the same result, so the choice only affects speed.  This module keeps
the selections in a JSON file per GPU architecture, keyed by dimension, dG
order, batch size and a size class (power of two of the slab length), so a
later handle of the same shape reuses the choice without timing again.
"""
from __future__ import annotations

import json
import math
import os
from typing import Optional

DEFAULT_PATH = os.path.join(os.environ.get("XDG_CACHE_HOME", os.path.expanduser("~/.cache")),
                            "biotst", "apply_tiles.json")


def _arch() -> str:
    import torch
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    return getattr(props, "gcnArchName", props.name).split(":")[0]


def cache_key(h) -> str:
    wl = h.wls[0]
    size_class = int(math.log2(max(h.slab_len, 1)))
    return f"dim{wl.dim}-r{wl.r}-count{h.count}-slab2^{size_class}"


def tune(h, path: Optional[str] = DEFAULT_PATH, reps: int = 20, refresh: bool = False) -> dict:
    """Select the apply tile variants of handle `h` (a BiotSlab), from the
    cache when it holds this shape, else by timing; returns the selection."""
    arch = _arch()
    key = cache_key(h)
    cache = {}
    if path and os.path.exists(path):
        try:
            with open(path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
    entry = cache.get(arch, {}).get(key)
    if entry is not None and not refresh:
        h.set_tuning(entry["apply_variant"])
        return dict(entry, source="cache")
    res = h.autotune(reps=reps)
    entry = {"apply_variant": res["apply_variant"], "apply_us": res["apply_us"]}
    if path:
        cache.setdefault(arch, {})[key] = entry
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(cache, f, indent=1, sort_keys=True)
        os.replace(tmp, path)
    return dict(entry, source="timed")
