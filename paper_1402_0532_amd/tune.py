"""Autotuner for the contraction tile plans.

For a workload (a single surface or a batch of CPIs) it times every tile plan of the
precision (and, for single surfaces, a few split-K counts; for batches, a few chunk
sizes) with hipEvents on the current stream, keeps the fastest, stores it in a JSON cache
(``$NDFT_TUNE_CACHE`` or ``~/.cache/ndft_mi355x/tune.json``) and applies it through
``ndft_set_plan``. Timing only: results are identical across plans up to rounding order.
"""
from __future__ import annotations

import json
import os
import threading

import torch

from . import BatchPlan, caf, caf_workspace_bytes, get_plan, plan_count, plan_name, set_plan, _prec

_LOCK = threading.Lock()


def cache_path() -> str:
    p = os.environ.get("NDFT_TUNE_CACHE")
    if p:
        return p
    return os.path.join(os.path.expanduser("~"), ".cache", "ndft_mi355x", "tune.json")


def _load_cache() -> dict:
    try:
        with open(cache_path()) as f:
            return json.load(f)
    except (OSError, ValueError):
        return {}


def _store(key: str, value: dict) -> None:
    with _LOCK:
        data = _load_cache()
        data[key] = value
        path = cache_path()
        try:
            os.makedirs(os.path.dirname(path), exist_ok=True)
            tmp = path + ".tmp%d" % os.getpid()
            with open(tmp, "w") as f:
                json.dump(data, f, indent=1, sort_keys=True)
            os.replace(tmp, path)
        except OSError:
            pass  # a read-only home still tunes, it just does not persist


def _time(fn, reps: int) -> float:
    fn()
    fn()
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def caf_key(prec, n, tau0, n_tau, p0, n_dop) -> str:
    return "caf:%d:%d:%d:%d:%d:%d" % (_prec(prec), n, tau0, n_tau, p0, n_dop)


def autotune_caf(s: torch.Tensor, r: torch.Tensor, tau0: int, n_tau: int, p0: int, n_dop: int,
                 prec=0, reps: int = 10, splits=None, use_cache: bool = True) -> dict:
    """Best (plan, ksplit) for this surface; applies it with set_plan and returns it."""
    p = _prec(prec)
    n = s.shape[0]
    key = caf_key(p, n, tau0, n_tau, p0, n_dop)
    if use_cache:
        hit = _load_cache().get(key)
        if hit and 0 <= hit.get("plan", -1) < plan_count(p) and plan_name(p, hit["plan"]) == hit.get("name"):
            set_plan(p, hit["plan"], hit["ksplit"])
            return hit
    out = torch.empty((n_tau, n_dop), dtype=torch.complex64, device=s.device)
    results = []
    for plan in range(plan_count(p)):
        set_plan(p, plan, 0)
        _, ks0 = get_plan(p, n, n_tau, p0, n_dop)
        # the library's count (a cost model of the rounds over the compute units), its
        # neighbours and half / double of it
        cands = sorted(set(splits or [ks0, max(1, ks0 - 1), ks0 + 1, max(1, ks0 // 2), 2 * ks0]))
        for ks in cands:
            set_plan(p, plan, ks)
            try:
                ws = torch.empty(caf_workspace_bytes(n, tau0, n_tau, p0, n_dop, p), dtype=torch.uint8,
                                 device=s.device)
                ms = _time(lambda: caf(s, r, tau0, n_tau, p0, n_dop, p, out=out, ws=ws), reps)
            except RuntimeError:
                continue  # a plan that does not fit this shape (e.g. LDS) is skipped
            results.append(dict(plan=plan, name=plan_name(p, plan), ksplit=ks, ms=ms))
    best = min(results, key=lambda d: d["ms"])
    best = dict(best, tried=len(results))
    set_plan(p, best["plan"], best["ksplit"])
    _store(key, best)
    return best


def autotune_batch(descs, surv_pool, ref_pool, out_pool, prec=0, reps: int = 3,
                   chunks=(2048, 4096, 8192)) -> tuple:
    """Best (plan, chunk) for a batch; returns (BatchPlan prepared with it, record)."""
    p = _prec(prec)
    results = []
    seen = set()
    for plan in range(plan_count(p)):
        set_plan(p, plan, 0)
        for ch in chunks:
            try:
                bp = BatchPlan(descs, p, device=surv_pool.device, chunk=ch)
            except RuntimeError:
                continue
            # a plan without a batched kernel falls back to the built-in one: time each
            # (plan actually used, chunk) once
            used = bp.batch.plan
            if (used, ch) in seen:
                del bp
                continue
            seen.add((used, ch))
            ms = _time(lambda: bp.run(surv_pool, ref_pool, out_pool), reps)
            results.append(dict(plan=used, name=plan_name(p, used), chunk=ch, ms=ms))
            del bp
    set_plan(p, -1, 0)
    if not results:
        raise RuntimeError("autotune_batch: no batched plan for this precision")
    best = min(results, key=lambda d: d["ms"])
    set_plan(p, best["plan"], 0)
    bp = BatchPlan(descs, p, device=surv_pool.device, chunk=best["chunk"])
    return bp, dict(best, tried=len(results))


def reset(prec=None) -> None:
    """Back to the library's built-in plan choice."""
    for p in ([0, 1, 2] if prec is None else [_prec(prec)]):
        set_plan(p, -1, 0)
