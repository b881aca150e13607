"""Launch-shape autotuner for plans and batches.

Each candidate shape (samples per lane S, one-shot vs streaming kernel,
persistent blocks per CU) is timed with HIP events on the current stream over
a few launches after a warm-up; the fastest is applied and cached as JSON,
keyed by GPU architecture and workload class:

  plan   (NI, L, ceil(log2 n))         forward kernels of one plan
  batch  (sorted class histogram, ceil(log2 total samples))

The cache file is $DPD_TUNE_CACHE, else ~/.cache/paper_1612_09001_amd/tune.json.
Tuning changes launch shapes only; every candidate computes the same outputs
(bit for bit: the per-output arithmetic order does not depend on the shape).
"""
from __future__ import annotations

import json
import math
import os

import torch

from . import dpd as _dpd

PLAN_CANDIDATES = [dict(samples_per_thread=s, stage_lds=l, grid_mult=g)
                   for s in (2, 4, 8) for l, gs in ((0, (8,)), (1, (4, 8, 16))) for g in gs]
BATCH_CANDIDATES = [dict(samples_per_thread=s, grid_mult=g) for s in (2, 4, 8) for g in (2, 4, 8, 16)]


def cache_path() -> str:
    p = os.environ.get("DPD_TUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "paper_1612_09001_amd", "tune.json")


def _load() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(d: dict):
    p = cache_path()
    try:
        os.makedirs(os.path.dirname(p), exist_ok=True)
        tmp = p + ".tmp%d" % os.getpid()
        with open(tmp, "w") as f:
            json.dump(d, f, indent=1, sort_keys=True)
        os.replace(tmp, p)
    except OSError:
        pass   # a read-only home directory only loses the cache


def arch() -> str:
    props = torch.cuda.get_device_properties(torch.cuda.current_device())
    return getattr(props, "gcnArchName", props.name).split(":")[0]


def time_us(fn, warmup=3, iters=10) -> float:
    """Mean time per call of fn() in microseconds (HIP events, current stream)."""
    for _ in range(warmup):
        fn()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(iters):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) * 1e3 / iters


def _levels(orders) -> int:
    return (max(orders) + 1) // 2


def plan_key(plan, n) -> str:
    ni = _levels(plan.main_orders + plan.conj_orders)
    return "plan|%s|NI%d|L%d|n2^%d" % (arch(), ni, plan.L, max(0, math.ceil(math.log2(max(n, 1)))))


def tune_plan(plan, x, out=None, candidates=None, use_cache=True, iters=10) -> dict:
    """Pick and apply the fastest forward launch shape of `plan` on input x."""
    key = plan_key(plan, x.numel())
    cache = _load() if use_cache else {}
    if use_cache and key in cache:
        best = cache[key]["tune"]
        plan.set_tune(**best)
        return best
    out = torch.empty_like(x) if out is None else out
    st = _dpd.current_stream()
    results = []
    for cand in candidates or PLAN_CANDIDATES:
        plan.set_tune(**cand)
        us = time_us(lambda: _dpd.dpd_apply(plan.handle, st, x.data_ptr(), out.data_ptr(), x.numel()),
                     iters=iters)
        results.append((us, cand))
    results.sort(key=lambda r: r[0])
    best = results[0][1]
    plan.set_tune(**best)
    if use_cache:
        cache = _load()
        cache[key] = {"tune": best, "us": results[0][0]}
        _store(cache)
    return best


def batch_key(specs) -> str:
    hist = {}
    total = 0
    for n, pmax, L in specs:
        k = "%d:%d" % ((pmax + 1) // 2, L)
        hist[k] = hist.get(k, 0) + n
        total += n
    sig = ",".join("%s=%d" % (k, max(0, math.ceil(math.log2(max(v, 1))))) for k, v in sorted(hist.items()))
    return "batch|%s|%s|n2^%d" % (arch(), sig, max(0, math.ceil(math.log2(max(total, 1)))))


def tune_batch(workload, candidates=None, use_cache=True, iters=5):
    """Pick the fastest persistent launch shape for a BatchWorkload; returns
    (tune dict, Batch built with it)."""
    from .batch import Batch

    key = batch_key(workload.specs)
    cache = _load() if use_cache else {}
    if use_cache and key in cache:
        best = cache[key]["tune"]
        return best, Batch(workload.streams(), tune=best)
    results = []
    for cand in candidates or BATCH_CANDIDATES:
        b = Batch(workload.streams(), tune=cand)
        us = time_us(b.apply, iters=iters)
        b.close()
        results.append((us, cand))
    results.sort(key=lambda r: r[0])
    best = results[0][1]
    if use_cache:
        cache = _load()
        cache[key] = {"tune": best, "us": results[0][0]}
        _store(cache)
    return best, Batch(workload.streams(), tune=best)
