"""Autotuner of launch shapes.

For the batched persistent solve it times every variant of the kernel (rows per wave of
the column chunks, target channels per column group, row-tile size) on the caller's own
problem set,
keeps the fastest, and caches the choice in a JSON file keyed by the device architecture
and a coarse signature of the problem set (instance count, total pixels, widest row,
channel counts), so later solvers of the same kind skip the measurement.

Cache file: $DTS_TUNE_CACHE, else ~/.cache/dts_mi355x/tuning.json.
"""
from __future__ import annotations

import json
import math
import os

import torch

_CACHE_ENV = "DTS_TUNE_CACHE"


def cache_path():
    p = os.environ.get(_CACHE_ENV)
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "dts_mi355x", "tuning.json")


def _load():
    try:
        with open(cache_path()) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _store(db):
    path = cache_path()
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        tmp = path + ".tmp"
        with open(tmp, "w") as fh:
            json.dump(db, fh, indent=1, sort_keys=True)
        os.replace(tmp, path)
    except OSError:
        pass  # a read-only home only costs a re-measurement next time


def _arch():
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    return getattr(props, "gcnArchName", props.name)


def batched_signature(problems):
    n = len(problems)
    px = sum(q["target"].shape[1] * q["target"].shape[2] for q in problems)
    wmax = max(q["target"].shape[2] for q in problems)
    ct = max(q["target"].shape[0] for q in problems)
    cg = max(q["guide"].shape[0] for q in problems)
    return (f"batched|n{2 ** max(0, math.ceil(math.log2(n)))}|px2^{round(math.log2(max(px, 1)))}"
            f"|w{2 ** math.ceil(math.log2(wmax))}|ct{ct}|cg{cg}")


def time_run(fn, iters):
    start, stop = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fn()
    torch.cuda.synchronize()
    start.record()
    for _ in range(iters):
        fn()
    stop.record()
    torch.cuda.synchronize()
    return start.elapsed_time(stop) / iters


def batched_variant(solver, iters=2, use_cache=True, report=None):
    """Index of the fastest batched-kernel variant for ``solver``'s problems.  A variant
    the problem set does not fit (DTS_ENOTSUP from the library, e.g. a strip with more
    chunks than the variant's grid) is skipped; any other failure is raised.  A cached
    choice is used only if that variant accepts the problem set."""
    from . import DTS_ENOTSUP, DTSError, batched_variants

    shapes = batched_variants()
    key = (_arch() + "|" + batched_signature(solver.problems) + "|variants:" +
           ",".join("x".join(str(x) for x in v[1:]) for v in shapes))
    db = _load() if use_cache else {}
    if key in db:
        cached = int(db[key]["variant"])
        try:
            solver._prepare(cached)
            return cached
        except DTSError as e:
            if e.code != DTS_ENOTSUP:
                raise
    timings = {}
    for v, *_ in shapes:
        try:
            solver._prepare(v)
        except DTSError as e:
            if e.code != DTS_ENOTSUP:
                raise
            continue
        timings[v] = time_run(solver.run, iters)
        solver.status()
    if not timings:
        raise DTSError(DTS_ENOTSUP, "no batched-kernel variant accepts this problem set")
    best = min(timings, key=timings.get)
    if report is not None:
        report.update({str(k): t for k, t in timings.items()})
    db = _load()
    db[key] = {"variant": best, "ms": timings}
    _store(db)
    return best
