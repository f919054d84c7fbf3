"""Autotuner of the int8 engine's tiles, for the persistent batched launch
and for one correlator.

A tile code (include/corrx.h) names the input block a work unit stages (64,
128 or 256 inputs; smaller blocks only for arrays that fit), the number of
time ranges per channel (automatic, 1, 2, 4, 8) and the samples a unit stages
at a time (the K-chunk: 64, 128 or 256, where the kernels have that variant).
The tuner measures each candidate on the real inputs and keeps the fastest:
for a batch, every array alone as a one-array persistent launch; for a
correlator, corr_xmac with corr_set_tile.  Results are cached in a JSON file
keyed by device architecture, engine, path and array shape, so a later run
with the same shapes skips the search.

The paper fixes its tile shape at compile time for one array (Sec. 3.3.3,
footnote on compile-time parameters; Sec. 3.4.2 on the tile's arithmetic
intensity); here the shape is chosen per array at run time.
"""

from __future__ import annotations

import json
import os

import numpy as np
import torch

from . import corrx

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "corrx", "tune.json")
SPLITS = (0, 1, 2, 4, 8)

# K-chunk lengths (samples) each unit has kernels for, first the default.
BATCH_CHUNKS = {corrx.CORRX_TILE_UNIT64: (0, 256), corrx.CORRX_TILE_UNIT128: (0, 128),
                corrx.CORRX_TILE_UNIT256: (0,)}
XMAC_CHUNKS = {corrx.CORRX_TILE_UNIT64: (0, 64, 256), corrx.CORRX_TILE_UNIT128: (0, 128),
               corrx.CORRX_TILE_UNIT256: (0,)}


def cache_path() -> str:
    return os.environ.get("CORRX_TUNE_CACHE", DEFAULT_CACHE)


def _arch() -> str:
    return torch.cuda.get_device_properties(0).gcnArchName.split(":")[0]


def _key(desc, engine: str = "mfma_i8", path: str = "batch", arch: str | None = None) -> str:
    n, f, t, lay = desc
    return f"{arch or _arch()}|{engine}|{path}|N{n}|F{f}|T{t}|L{lay}"


def _units(n_inputs: int) -> list[int]:
    units = [corrx.CORRX_TILE_UNIT256]
    if n_inputs <= 128:
        units.append(corrx.CORRX_TILE_UNIT128)
    if n_inputs <= 64:
        units.append(corrx.CORRX_TILE_UNIT64)
    return units


def candidates(n_inputs: int, path: str = "batch") -> list[int]:
    """Tile codes worth measuring for an array of n_inputs inputs."""
    chunks = BATCH_CHUNKS if path == "batch" else XMAC_CHUNKS
    return [corrx.tile_code(u, s, c) for u in _units(n_inputs) for c in chunks[u] for s in SPLITS]


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


def measure_xmac(desc, code: int, inp, acc, reps: int = 3) -> float:
    """Median time (ms) of corr_xmac with tile code `code`."""
    n, f, t, lay = desc
    c = corrx.Correlator(n, f, t, lay, "mfma_i8")
    c.set_tile(code)
    stream = torch.cuda.current_stream()
    c.zero(acc)
    c.xmac(inp, acc)  # warm-up
    times = []
    for _ in range(reps):
        c.zero(acc)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        c.xmac(inp, acc)
        e1.record(stream)
        torch.cuda.synchronize()
        times.append(e0.elapsed_time(e1))
    c.close()
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


def _search(key, cache, codes, timer, log):
    times = {}
    for code in codes:
        try:
            times[str(code)] = timer(code)
        except corrx.CorrxError as e:  # a variant this shape cannot use
            if e.status != corrx.CORRX_EUNSUPPORTED:
                raise
            continue
        if log:
            log(f"tune {key} code {code:#x}: {times[str(code)]:.3f} ms")
    best = min(times, key=times.get)
    cache[key] = {"code": int(best), "ms": times[best], "times": times}
    return cache[key]


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
        key = _key(d, "mfma_i8", "batch")
        if key not in cache:
            _search(key, cache, candidates(d[0], "batch"),
                    lambda code: measure([d], [code], [ins[k]], [accs[k]], reps), log)
        codes.append(int(cache[key]["code"]))
        report[key] = cache[key]
    if use_cache:
        _save_cache(path, cache)
    return codes, report


def tune_correlator(desc, inp, acc, use_cache: bool = True, reps: int = 3, log=None) -> tuple[int, dict]:
    """Tile code for corr_xmac on one array (int8 engine), measured on its
    input; apply it with Correlator.set_tile.  acc is used as scratch."""
    path = cache_path()
    cache = _load_cache(path) if use_cache else {}
    key = _key(desc, "mfma_i8", "xmac")
    if key not in cache:
        _search(key, cache, candidates(desc[0], "xmac"), lambda code: measure_xmac(desc, code, inp, acc, reps), log)
    if use_cache:
        _save_cache(path, cache)
    return int(cache[key]["code"]), cache[key]
