"""Autotuner of the Gauss-point launch: lanes per point and persistent waves.

For every DMN depth of a workload it times each compiled lane variant
(``dmn_gp_lane_variants``) at a few persistent-wave counts on the workload
itself, keeps the fastest with ``dmn_gp_set_tuning`` and records the choice
in a JSON cache, keyed by device, library version, depth and point count
(rounded to a power of two), so later processes set it without timing.  A
workload whose fixed-normal groups differ in depth runs in one mixed-depth
launch; there the wave count of that launch is tuned on the whole workload.

The update is functional (inputs are never written), so timing repeated calls
on the caller's groups leaves their inputs intact; their outputs end up as
one call would leave them.  Tuning never changes what a call computes per
point, only how fast.
"""
import ctypes
import json
import math
import os
import tempfile
from typing import Callable, Dict, List, Optional, Sequence, Tuple

from . import _lib as L

WAVES_PER_CU = (4, 8, 16)


def default_cache_path() -> str:
    return os.environ.get("DMN_AUTOTUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "libdmn",
                                       "autotune.json"))


def lane_variants(depth: int) -> List[int]:
    """Lane counts per point compiled for a depth."""
    lib = L.lib()
    n = lib.dmn_gp_lane_variants(depth, None, 0)
    buf = (ctypes.c_int32 * max(n, 1))()
    lib.dmn_gp_lane_variants(depth, buf, n)
    return list(buf[:n])


def get_tuning(depth: int) -> Tuple[int, int]:
    t = L.DmnGpTuning()
    L.check(L.lib().dmn_gp_get_tuning(depth, ctypes.byref(t)), "dmn_gp_get_tuning")
    return t.lanes_per_point, t.waves_per_cu


def set_tuning(depth: int, lanes_per_point: int = 0, waves_per_cu: int = 0):
    """Set the tuning of a depth (0 = default for either field)."""
    t = L.DmnGpTuning(lanes_per_point, waves_per_cu)
    L.check(L.lib().dmn_gp_set_tuning(depth, ctypes.byref(t)), "dmn_gp_set_tuning")


def reset_tuning():
    for k in range(1, 11):
        L.check(L.lib().dmn_gp_set_tuning(k, None), "dmn_gp_set_tuning")


def device_tag(device=None) -> str:
    import torch
    p = torch.cuda.get_device_properties(device if device is not None else 0)
    return f"{p.name}|{p.multi_processor_count}CU|{L.lib().dmn_version().decode()}"


def cache_key(tag: str, depth: int, n_points: int) -> str:
    bucket = 2 ** int(round(math.log2(max(n_points, 1))))
    return f"{tag}|K{depth}|P{bucket}"


def load_cache(path: str) -> Dict[str, dict]:
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def save_cache(path: str, cache: Dict[str, dict]):
    """Write atomically (rename of a temporary file in the same folder)."""
    folder = os.path.dirname(os.path.abspath(path))
    os.makedirs(folder, exist_ok=True)
    fd, tmp = tempfile.mkstemp(dir=folder, suffix=".tmp")
    with os.fdopen(fd, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def _gpu_timer(groups, fiber, matrix, reps: int, newton: dict) -> float:
    """Median milliseconds of one dmn_update_gauss_points call on the groups."""
    import torch
    from .api import dmn_update_gauss_points
    ws = dmn_update_gauss_points(groups, fiber, matrix, **newton)  # warm-up
    times = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        dmn_update_gauss_points(groups, fiber, matrix, ws=ws, **newton)
        b.record()
        b.synchronize()
        times.append(a.elapsed_time(b))
    times.sort()
    return times[len(times) // 2]


def mixed_cache_key(tag: str, depths: Sequence[int], n_points: int) -> str:
    bucket = 2 ** int(round(math.log2(max(n_points, 1))))
    return f"{tag}|mixed|K{','.join(str(k) for k in sorted(depths))}|P{bucket}"


# the library runs fixed-normal groups of several depths (or of depth 9) in one
# mixed-depth launch for depths >= MIXED_MIN_DEPTH; only the persistent wave
# count of that launch is a choice (lane splits are fixed there)
MIXED_MIN_DEPTH = 2
SPLIT_DEPTH = 9


def _depth_of(g) -> int:
    return int(round(math.log2(g.w.numel())))


def tune_gauss_points(groups: Sequence, fiber: dict, matrix: dict,
                      cache_path: Optional[str] = None, reps: int = 3,
                      waves: Sequence[int] = WAVES_PER_CU, retune: bool = False,
                      timer: Optional[Callable] = None, tag: Optional[str] = None,
                      **newton) -> Dict[int, dict]:
    """Tune the launches of a workload like ``groups`` and set the winners.

    Groups of one depth: every compiled lane variant at each wave count, per
    depth.  Fixed-normal groups of several depths (or with depth 9), which the
    library runs in one mixed-depth launch: the wave count of that launch,
    timed on all those groups together (depths 2-9), and depth 1 on its own.

    Returns {depth: {"lanes_per_point", "waves_per_cu", "ms", "cached"}, with
    "launch": "mixed" for the depths of a mixed launch}.  ``timer(groups,
    fiber, matrix, reps, newton) -> ms`` and ``tag`` replace the GPU timing and
    device tag (for tests of the cache logic).
    """
    timer = timer or _gpu_timer
    path = cache_path or default_cache_path()
    tag = tag or device_tag()
    by_depth: Dict[int, list] = {}
    for g in groups:
        if getattr(g, "ori", None) is not None:
            continue  # orientation-interpolated groups always use the default split
        if g.E.shape[0] > 0:
            by_depth.setdefault(_depth_of(g), []).append(g)
    cache = load_cache(path)
    chosen: Dict[int, dict] = {}
    dirty = False

    mixed = sorted(K for K in by_depth if K >= MIXED_MIN_DEPTH)
    if len(by_depth) > 1 or SPLIT_DEPTH in by_depth:
        gs = [g for K in mixed for g in by_depth[K]]
        key = mixed_cache_key(tag, mixed, sum(g.E.shape[0] for g in gs))
        hit = cache.get(key)
        if hit and not retune:
            best, cached = (hit["ms"], hit["waves_per_cu"]), True
        else:
            best, cached = None, False
            for w in waves:
                for K in mixed:
                    set_tuning(K, 0, w)
                ms = float(timer(gs, fiber, matrix, reps, newton))
                if best is None or ms < best[0]:
                    best = (ms, w)
            cache[key] = dict(waves_per_cu=best[1], ms=best[0])
            dirty = True
        for K in mixed:
            set_tuning(K, 0, best[1])
            lanes, _ = get_tuning(K)
            chosen[K] = dict(lanes_per_point=lanes, waves_per_cu=best[1], ms=best[0],
                             cached=cached, launch="mixed")
        single = [K for K in by_depth if K < MIXED_MIN_DEPTH]
    else:
        single = list(by_depth)

    for K in sorted(single, reverse=True):
        gs = by_depth[K]
        P = sum(g.E.shape[0] for g in gs)
        key = cache_key(tag, K, P)
        hit = cache.get(key)
        if hit and not retune and hit.get("lanes_per_point") in lane_variants(K):
            set_tuning(K, hit["lanes_per_point"], hit["waves_per_cu"])
            chosen[K] = dict(hit, cached=True)
            continue
        best = None
        for lanes in lane_variants(K):
            for w in waves:
                set_tuning(K, lanes, w)
                ms = float(timer(gs, fiber, matrix, reps, newton))
                if best is None or ms < best[0]:
                    best = (ms, lanes, w)
        set_tuning(K, best[1], best[2])
        cache[key] = dict(lanes_per_point=best[1], waves_per_cu=best[2], ms=best[0])
        chosen[K] = dict(cache[key], cached=False)
        dirty = True
    if dirty:
        save_cache(path, cache)
    return chosen
