"""Autotuner for the launch shapes of the stage kernels and the batch kernel.

Single-transform plans: for every axis it times the candidate shapes (lines
per workgroup, threads-per-line divisor, split exchange, padding) that the
library accepts for that stage, using the per-stage timing events, and keeps
the fastest.  Batches: for every (length, layout) present it times the whole
persistent launch with each candidate lines-per-item value, one coordinate at a
time, and keeps the fastest.  The shapes only change how work is mapped onto
threads, never the arithmetic, so results are bitwise identical whatever is
chosen.

Choices are cached in a JSON file (``FFT3D_TUNE_CACHE``, default
``~/.cache/fft3d_tune.json``) keyed by GPU architecture, precision, length,
layout and line stride.
"""
from __future__ import annotations

import json
import os
import threading

import torch

from . import fft3d

_lock = threading.Lock()


def cache_path() -> str:
    return os.environ.get("FFT3D_TUNE_CACHE", os.path.expanduser("~/.cache/fft3d_tune.json"))


def _load():
    try:
        with open(cache_path()) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def _save(d):
    p = cache_path()
    os.makedirs(os.path.dirname(p) or ".", exist_ok=True)
    tmp = p + ".tmp%d" % os.getpid()
    with open(tmp, "w") as fh:
        json.dump(d, fh, indent=1, sort_keys=True)
    os.replace(tmp, p)


def _arch() -> str:
    return torch.cuda.get_device_properties(torch.cuda.current_device()).gcnArchName.split(":")[0]


def _stage_key(plan: fft3d.Plan, axis: int) -> str:
    nz, ny, nx = plan.shape
    n = (nx, ny, nz)[axis]
    nxc = nx // 2 + 1 if plan.r2c else nx
    stride = (1, nxc, nxc * ny)[axis]
    kind = "r2c" if (plan.r2c and axis == 0) else "c2c"
    return f"{_arch()}|{'c64' if plan.code == fft3d.C64 else 'c128'}|{kind}|n{n}|axis{axis}|stride{stride}"


def stage_candidates(axis: int):
    if axis == 0:
        return [(lw, td, sp, pd) for lw in (1, 2, 4, 8, 16) for td in (1, 2) for sp in (0, 1) for pd in (0, 1)]
    return [(lw, td, sp, 0) for lw in (4, 8, 16, 32, 64) for td in (1, 2, 4) for sp in (0, 1)]


def _time_stage(plan, x, out, axis, reps):
    plan.set_timing(True)
    plan.forward(x, out=out)
    plan.stage_times()
    ts = []
    for _ in range(reps):
        plan.forward(x, out=out)
        t = plan.stage_times()
        # forward stages run x, y, z
        ts.append(t[axis])
    plan.set_timing(False)
    ts.sort()
    return ts[len(ts) // 2]


def tune_plan(plan: fft3d.Plan, reps: int = 5, use_cache: bool = True, verbose: bool = False):
    """Pick the fastest launch shape of every forward stage of `plan`; returns {axis: shape}."""
    with _lock:
        cache = _load() if use_cache else {}
    chosen = {}
    nz, ny, nx = plan.shape
    if plan.r2c:
        x = torch.randn(plan.shape, dtype=plan.real_dtype, device="cuda")
        out = torch.empty(plan.half_shape, dtype=plan.complex_dtype, device="cuda")
    else:
        x = torch.randn(plan.shape, dtype=plan.complex_dtype, device="cuda")
        out = torch.empty_like(x)
    for axis in (0, 1, 2):
        key = _stage_key(plan, axis)
        if key in cache:
            shape = tuple(cache[key])
            try:
                plan.set_stage_config(axis, *shape)
                chosen[axis] = shape
                continue
            except RuntimeError:
                pass
        best = None
        plan.set_stage_config(axis, 0)
        t0 = _time_stage(plan, x, out, axis, reps)
        best = (t0, None)
        for cand in stage_candidates(axis):
            try:
                plan.set_stage_config(axis, *cand)
            except RuntimeError:
                continue
            t = _time_stage(plan, x, out, axis, reps)
            if verbose:
                print(f"axis {axis} {cand}: {t:.4f} ms")
            if t < best[0]:
                best = (t, cand)
        if best[1] is None:
            plan.set_stage_config(axis, 0)
        else:
            plan.set_stage_config(axis, *best[1])
            chosen[axis] = best[1]
            cache[key] = list(best[1])
    if use_cache:
        with _lock:
            merged = _load()
            merged.update(cache)
            _save(merged)
    return chosen


def _time_batch(bp, xs, outs, reps):
    for _ in range(2):
        bp.forward(xs, outs)
    torch.cuda.synchronize()
    s = torch.cuda.Event(enable_timing=True)
    e = torch.cuda.Event(enable_timing=True)
    s.record()
    for _ in range(reps):
        bp.forward(xs, outs)
    e.record()
    torch.cuda.synchronize()
    bp.check()
    return s.elapsed_time(e) / reps


def tune_batch(bp: fft3d.BatchPlan, xs, reps: int = 5, use_cache: bool = True, verbose: bool = False):
    """Pick lines per item for every (length, layout) of the batch; returns {(n, strided): lw}."""
    with _lock:
        cache = _load() if use_cache else {}
    outs = [torch.empty_like(x) for x in xs]
    keys = set()
    for nz, ny, nx in bp.shapes:
        keys |= {(nx, 0), (ny, 1), (nz, 1)}
    chosen = {}
    pending = []
    for n, strided in sorted(keys):
        ck = f"{_arch()}|batch|c64|n{n}|strided{strided}"
        if ck in cache:
            bp.set_lines(n, strided, int(cache[ck]))
            chosen[(n, strided)] = int(cache[ck])
        else:
            pending.append((n, strided, ck))
    for n, strided, ck in pending:
        _, tpl = fft3d.query_radix_plan(n)
        best = (_time_batch(bp, xs, outs, reps), 0)
        lw_max = max(1, 256 // tpl)
        cands = sorted({max(1, lw_max // d) for d in (1, 2, 3, 4, 6, 8)})
        for lw in cands:
            try:
                bp.set_lines(n, strided, lw)
            except RuntimeError:
                continue
            t = _time_batch(bp, xs, outs, reps)
            if verbose:
                print(f"n={n} strided={strided} lw={lw}: {t:.4f} ms")
            if t < best[0]:
                best = (t, lw)
        bp.set_lines(n, strided, best[1])
        if best[1]:
            chosen[(n, strided)] = best[1]
            cache[ck] = best[1]
    if use_cache:
        with _lock:
            merged = _load()
            merged.update(cache)
            _save(merged)
    return chosen
