"""Autotuner of the tile-wavefront sweep's launch shape.

The free parameter is the number of 64-lane waves per sweep workgroup (1 .. min(R, 10),
R = rays per octant; with fewer waves than rays each wave runs several rays in turn).
The best count depends on the grid size (how many tiles a stage offers against the
CUs), on R, on the precision and on the segment order, so it is tuned per shape class:
the device times a few formal solutions of the problem at hand for every count
(rt_problem_tune) and the winner is kept in a JSON file keyed by the class, so later
problems of the same class only look it up.  The cache path is RTSC_TUNE_CACHE, or
~/.cache/rtsc/tune.json.
"""
from __future__ import annotations

import json
import os


def _pow2(n: int) -> int:
    p = 1
    while p < n:
        p *= 2
    return p


def shape_class(desc) -> str:
    """Key of a problem's shape class: precision, segment order, rays per octant, bins
    (up to powers of two) and the grid edges rounded up to powers of two."""
    na = desc.na if getattr(desc, "mu", None) else desc.n_mu * (desc.n_mu + 2)
    return (f"p{desc.precision}-o{desc.order}-R{na // 8}-nf{_pow2(desc.nf)}-"
            f"{_pow2(desc.nx)}x{_pow2(desc.ny)}x{_pow2(desc.nz)}")


def cache_path() -> str:
    return os.environ.get("RTSC_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "rtsc", "tune.json"))


def load_cache(path: str | None = None) -> dict:
    path = path or cache_path()
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def store(key: str, entry: dict, path: str | None = None) -> None:
    path = path or cache_path()
    data = load_cache(path)
    data[key] = entry
    os.makedirs(os.path.dirname(os.path.abspath(path)), exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        json.dump(data, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def autotune(problem, S, path: str | None = None, reps: int = 3, retune: bool = False, stream=None) -> dict:
    """Set the problem's wave count from the cache, or tune it on the device (S: the
    source function to sweep, device FP64 [nf][cells]) and record it.  Returns the
    cache entry {"waves": w, "ms": {w: ms per sweep}}."""
    key = shape_class(problem.desc)
    entry = None if retune else load_cache(path).get(key)
    if entry is not None:
        problem.set_waves(int(entry["waves"]))
        return entry
    best, ms = problem.tune(S, reps=reps, stream=stream)
    entry = {"waves": int(best), "ms": {str(w): float(t) for w, t in ms.items()}}
    store(key, entry, path)
    return entry
