"""Autotuner cache for the spreading work-group shape.

The spreading kernel has a few work-group shapes (waves per group x coils per
lane); all give bit-identical grids, and the fastest depends on the grid, the
sample count and the coil chunk.  ``tune`` times every shape once per
geometry through ``Context.autotune_spread`` and keeps the choice in a JSON
file, so later contexts of the same geometry reuse it without timing.
"""
from __future__ import annotations

import json
import os
import tempfile


def cache_path() -> str:
    return os.environ.get("CS_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "coilsketch",
                                       "spread_shapes.json"))


def geometry_key(ndim: int, grid, nsamp: int, ncoil: int) -> str:
    """Cache key: dimension, oversampled grid, samples per coil, coil chunk."""
    chunk = min(int(ncoil), 16)
    return f"{ndim}d/{'x'.join(str(int(g)) for g in grid)}/N{int(nsamp)}/c{chunk}"


def load_cache(path: str) -> dict:
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def store_cache(path: str, cache: dict) -> None:
    """Write the cache atomically (temporary file, then rename)."""
    d = os.path.dirname(path) or "."
    os.makedirs(d, exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=d, prefix=".spread_shapes")
    with os.fdopen(fd, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune(ctx, maps, reps: int = 3, path: str | None = None):
    """Select the spreading shape of `ctx` for normal applies with `maps`:
    from the cache if this geometry was tuned before, else by timing every
    shape.  Returns (shape index, per-shape ms per apply or None, from_cache)."""
    path = path or cache_path()
    key = geometry_key(ctx.ndim, ctx.grid_shape(), ctx.N, maps.shape[-1])
    cache = load_cache(path)
    hit = cache.get(key)
    if isinstance(hit, dict) and isinstance(hit.get("shape"), int):
        ctx.set_spread_cfg(hit["shape"])
        return hit["shape"], hit.get("ms"), True
    best, ms = ctx.autotune_spread(maps, reps)
    cache[key] = {"shape": best, "ms": ms}
    store_cache(path, cache)
    return best, ms, False
