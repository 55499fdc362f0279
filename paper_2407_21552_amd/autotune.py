"""Autotuner for the batched build's launch shape.

The batched build (pdm_batch_build) has four knobs that change its speed
but not its result: three grouped launches or one cooperative launch, the
brick rows per first-phase work item, the number of 64-line groups per y/z
work item, and whether the largest volumes' items come first.
`tune_batch_build` times every candidate on the actual batch (HIP events on
the launch stream, median of a few runs, after one warm-up, checking the
workspace error word) and caches the fastest configuration under a
signature of the batch (volume shapes, dtypes, partition counts) and the
device name.  The brick size is fixed at 4 by the method; only these launch
shapes are tuned.
"""
from __future__ import annotations

import hashlib
import json
import os

from . import _lib

CANDIDATES = [dict(single_launch=sl, rows_per_item=r, lines_mult=m, largest_first=lf)
              for sl in (0, 1) for r in (1, 2, 4) for m in (1, 2, 4) for lf in (0, 1)]

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "pdm_autotune.json")


def signature(items) -> str:
    """Key of a batch: device name plus (shape, dtype, levels, n) of every volume."""
    import torch
    parts = [torch.cuda.get_device_name(0)]
    for desc, _vol, _bmin, _bmax, bounds, _pdms in items:
        parts.append(f"{desc.nx}x{desc.ny}x{desc.nz}:{desc.dtype}:{desc.levels}:{len(bounds) - 1}")
    return hashlib.sha256("|".join(parts).encode()).hexdigest()[:24]


def _load(path: str) -> dict:
    try:
        with open(path) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def cached_config(items, cache_path: str = DEFAULT_CACHE):
    """The cached best configuration of this batch, or None."""
    return _load(cache_path).get(signature(items), {}).get("best")


def time_batch_build(items, workspace, config, reps: int = 3, stream=None) -> float:
    """Median milliseconds of one batched build with `config` (after a warm-up)."""
    import torch
    s = torch.cuda.current_stream() if stream is None else stream
    _lib.batch_build(items, workspace, config, s)
    times = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record(s)
        _lib.batch_build(items, workspace, config, s)
        b.record(s)
        b.synchronize()
        if _lib.batch_error(workspace) != 0:
            raise _lib.PdmError(_lib.PDM_E_DEVICE, "single-launch batched build: a barrier wait gave up")
        times.append(a.elapsed_time(b))
    times.sort()
    return times[len(times) // 2]


def tune_batch_build(items, workspace, candidates=None, reps: int = 3,
                     cache_path: str = DEFAULT_CACHE, stream=None):
    """Time every candidate; return (best config, {config-string: ms}).  The
    winner is stored in the JSON cache at `cache_path` (None: no cache)."""
    cands = CANDIDATES if candidates is None else candidates
    table = {}
    best, best_ms = None, float("inf")
    for cfg in cands:
        ms = time_batch_build(items, workspace, cfg, reps, stream)
        table[json.dumps(cfg, sort_keys=True)] = ms
        if ms < best_ms:
            best, best_ms = dict(cfg), ms
    if cache_path:
        data = _load(cache_path)
        data[signature(items)] = {"best": best, "ms": best_ms}
        os.makedirs(os.path.dirname(cache_path), exist_ok=True)
        tmp = cache_path + ".tmp"
        with open(tmp, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
        os.replace(tmp, cache_path)
    return best, table
