"""Autotuner of the persistent batched launch.

For every array of a batch it measures a small set of tile codes -- the input
block a work item stages (64, 128 or 256 inputs; smaller blocks only for
arrays that fit) times the number of time ranges per channel (automatic, 1, 2,
4, 8) -- each as one persistent launch on the real inputs, and keeps the
fastest.  Results are cached in a JSON file keyed by device architecture and
array shape, so a later batch with the same shapes skips the search.

The paper fixes its tile shape at compile time for one array (Sec. 3.3.2,
footnote on compile-time parameters); here the shape is chosen per array at
run time.
"""

from __future__ import annotations

import json
import os

import numpy as np
import torch

from . import corrx

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "corrx", "tune.json")
SPLITS = (0, 1, 2, 4, 8)


def cache_path() -> str:
    return os.environ.get("CORRX_TUNE_CACHE", DEFAULT_CACHE)


def _arch() -> str:
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def _key(desc) -> str:
    n, f, t, lay = desc
    return f"{_arch()}|N{n}|F{f}|T{t}|L{lay}"


def candidates(n_inputs: int) -> list[int]:
    units = [corrx.CORRX_TILE_UNIT256]
    if n_inputs <= 128:
        units.append(corrx.CORRX_TILE_UNIT128)
    if n_inputs <= 64:
        units.append(corrx.CORRX_TILE_UNIT64)
    return [u | (s << 8) for u in units for s in SPLITS]


def measure(descs, tile_cfg, ins, accs, reps: int = 3) -> float:
    """Median time (ms) of one persistent launch of the batch."""
    b = corrx.Batch(descs, tile_cfg=tile_cfg)
    stream = torch.cuda.current_stream()
    b.xmac(ins, accs)  # warm-up
    times = []
    for _ in range(reps):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        b.xmac(ins, accs)
        e1.record(stream)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    b.close()
    return float(np.median(times))


def _load_cache(path: str) -> dict:
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _save_cache(path: str, data: dict) -> None:
    os.makedirs(os.path.dirname(path) or ".", exist_ok=True)
    tmp = path + ".tmp"
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def tune_batch(descs, ins, accs, use_cache: bool = True, reps: int = 3, log=None) -> tuple[list[int], dict]:
    """Tile code per array; each array searched alone on its own inputs.

    Returns (codes, report) where report maps each array's key to the times
    (ms) of all candidates.  The accumulators are used as scratch by the
    search; zero them before the real run.
    """
    path = cache_path()
    cache = _load_cache(path) if use_cache else {}
    codes, report = [], {}
    for k, d in enumerate(descs):
        key = _key(d)
        if key in cache:
            codes.append(int(cache[key]["code"]))
            report[key] = cache[key]
            continue
        times = {}
        for code in candidates(d[0]):
            times[str(code)] = measure([d], [code], [ins[k]], [accs[k]], reps)
            if log:
                log(f"tune {key} code {code:#x}: {times[str(code)]:.3f} ms")
        best = min(times, key=times.get)
        cache[key] = {"code": int(best), "ms": times[best], "times": times}
        report[key] = cache[key]
        codes.append(int(best))
    if use_cache:
        _save_cache(path, cache)
    return codes, report
