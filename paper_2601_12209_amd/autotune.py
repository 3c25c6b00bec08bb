"""Autotuner for the launch shapes of the stage kernels.

For every axis of a plan it times the candidate shapes (lines per workgroup,
threads-per-line divisor, split exchange, padding) that the library accepts
for that stage, using the per-stage timing events, and keeps the fastest; a
batch is tuned shape by shape the same way, and for shapes that fit the
fused x-y kernel the staging (fused planes or three line stages) is picked
by timing the whole batch.  The shapes only change how work
is mapped onto threads, never the arithmetic, so results are bitwise
identical whatever shape is chosen; for the complex line kernels it also
tries the reverse radix order (fft3d_set_radix_order), which changes the
rounding of the results but not their accuracy class.

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


def _stage_key(plan: fft3d.Plan, axis: int, nstages: int = 3) -> str:
    nz, ny, nx = plan.shape
    n = (nx, ny, nz)[axis]
    nxc = nx // 2 + 1 if plan.r2c else nx
    stride = (1, nxc, nxc * ny)[axis]
    kind = "r2c" if (plan.r2c and axis == 0) else "c2c"
    return (f"{_arch()}|{'c64' if plan.code == fft3d.C64 else 'c128'}|{kind}|n{n}|axis{axis}|stride{stride}"
            f"|stages{nstages}")


def stage_candidates(axis: int):
    if axis == 0:
        return [(lw, td, sp, pd) for lw in (1, 2, 4, 8, 16) for td in (1, 2) for sp in (0, 1) for pd in (0, 1)]
    return [(lw, td, sp, 0) for lw in (4, 8, 16, 32, 64) for td in (1, 2, 4) for sp in (0, 1)]


def _forward_stage_count(plan, x, out):
    plan.set_timing(True)
    plan.forward(x, out=out)
    n = len(plan.stage_times())
    plan.set_timing(False)
    return n


def _time_stage(plan, x, out, index, reps):
    plan.set_timing(True)
    plan.forward(x, out=out)
    plan.stage_times()
    ts = []
    for _ in range(reps):
        plan.forward(x, out=out)
        ts.append(plan.stage_times()[index])
    plan.set_timing(False)
    ts.sort()
    return ts[len(ts) // 2]


def _apply(plan, axis, shape):
    """Set a tuned (lw, tdiv, split, pad[, radix order]) on one axis of a plan or batch shape."""
    plan.set_stage_config(axis, *shape[:4])
    if len(shape) > 4:
        plan.set_radix_order(axis, shape[4])


def tune_plan(plan: fft3d.Plan, reps: int = 5, use_cache: bool = True, verbose: bool = False):
    """Pick the fastest launch shape, and radix order of the line kernels, of
    every forward stage of `plan`; returns {axis: (lw, tdiv, split, pad,
    order)}.  The launch shape never changes the results; the reverse radix
    order changes their rounding."""
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
    # forward stages: x, y, z; with fused x-y planes the plane kernel (a fixed
    # launch shape) and then z, so only the z stage is tuned
    nst = _forward_stage_count(plan, x, out)
    stage_of = {0: 0, 1: 1, 2: 2} if nst == 3 else {2: nst - 1}
    for axis, index in stage_of.items():
        key = _stage_key(plan, axis, nst)
        if key in cache:
            shape = tuple(cache[key])
            try:
                _apply(plan, axis, shape)
                chosen[axis] = shape
                continue
            except RuntimeError:
                plan.set_stage_config(axis, 0)
                plan.set_radix_order(axis, 0)
        plan.set_stage_config(axis, 0)
        plan.set_radix_order(axis, 0)
        t0 = _time_stage(plan, x, out, index, reps)
        best = (t0, None)
        # the reverse radix order runs with one thread per butterfly and the
        # plain exchange; the real x kernels have no such choice
        line_kernels = not (plan.r2c and axis == 0)
        for cand in stage_candidates(axis):
            try:
                plan.set_stage_config(axis, *cand)
            except RuntimeError:
                continue
            for order in ((0, 1) if line_kernels and cand[1] == 1 and cand[2] == 0 else (0,)):
                try:
                    plan.set_radix_order(axis, order)
                except RuntimeError:
                    break
                t = _time_stage(plan, x, out, index, reps)
                if verbose:
                    print(f"axis {axis} {cand} order {order}: {t:.4f} ms")
                if t < best[0]:
                    best = (t, tuple(cand) + (order,))
            plan.set_radix_order(axis, 0)
        if best[1] is None:
            plan.set_stage_config(axis, 0)
        else:
            _apply(plan, axis, best[1])
            chosen[axis] = best[1]
            cache[key] = list(best[1])
    if use_cache:
        with _lock:
            merged = _load()
            merged.update(cache)
            _save(merged)
    return chosen


def _time_batch(bp, xs, outs, reps):
    bp.forward(xs, outs)  # builds the launch tables of this pointer set
    start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ts = []
    for _ in range(reps):
        start.record()
        bp.forward(xs, outs)
        end.record()
        end.synchronize()
        ts.append(start.elapsed_time(end))
    ts.sort()
    return ts[len(ts) // 2]


def tune_batch(bp: fft3d.BatchPlan, reps: int = 5, use_cache: bool = True, verbose: bool = False):
    """Tune every distinct shape of the batch and apply the result: the stage
    launch shapes on a stand-alone plan of that shape, for each staging the
    shape can take, and then, for shapes that fit the fused x-y kernel, the
    staging itself (fused planes or three line stages) by timing the whole
    batch, largest shapes first (the shapes share the GPU, so the better
    staging depends on the rest of the batch).  Returns {shape: (staging,
    {axis: shape})}."""
    dt = fft3d._COMPLEX[bp.code]
    shapes = sorted(set(bp.shapes))
    counts = {sh: bp.shapes.count(sh) for sh in shapes}
    fusable = [sh for sh in shapes if bp.staging(sh) == fft3d.STAGING_FUSED_XY]
    tuned = {}
    for sh in shapes:
        for st in ((fft3d.STAGING_FUSED_XY, fft3d.STAGING_IN_PLACE) if sh in fusable else (fft3d.STAGING_IN_PLACE,)):
            p = fft3d.Plan(sh, dt, staging=st)
            tuned[(sh, st)] = tune_plan(p, reps=reps, use_cache=use_cache, verbose=verbose)
            p.close()

    class _Shape:  # one shape of the batch, with a plan's setter names
        def __init__(self, sh):
            self.sh = sh

        def set_stage_config(self, axis, *cfg):
            bp.set_stage_config(self.sh, axis, *cfg)

        def set_radix_order(self, axis, order):
            bp.set_radix_order(self.sh, axis, order)

    def apply(sh, st):
        bp.set_staging(sh, st)
        for axis in range(3):
            bp.set_stage_config(sh, axis, 0)
            bp.set_radix_order(sh, axis, 0)
        for axis, cfg in tuned[(sh, st)].items():
            _apply(_Shape(sh), axis, cfg)

    choice = {sh: (fft3d.STAGING_FUSED_XY if sh in fusable else fft3d.STAGING_IN_PLACE) for sh in shapes}
    for sh in shapes:
        apply(sh, choice[sh])
    if fusable:
        with _lock:
            cache = _load() if use_cache else {}
        comp = ",".join(f"{a}x{b}x{c}:{counts[(a, b, c)]}" for (a, b, c) in shapes)
        key = f"{_arch()}|{'c64' if bp.code == fft3d.C64 else 'c128'}|batch-staging|{comp}"
        if key in cache:
            picked = {tuple(json.loads(k)): v for k, v in cache[key].items()}
        else:
            xs = [torch.randn(sh, dtype=dt, device="cuda") for sh in bp.shapes]
            outs = [torch.empty_like(t) for t in xs]
            picked = {}
            for sh in sorted(fusable, key=lambda v: -counts[v] * v[0] * v[1] * v[2]):
                best = None
                for st in (fft3d.STAGING_FUSED_XY, fft3d.STAGING_IN_PLACE):
                    apply(sh, st)
                    t = _time_batch(bp, xs, outs, reps)
                    if verbose:
                        print(f"batch staging {sh} {st}: {t:.4f} ms")
                    if best is None or t < best[0]:
                        best = (t, st)
                picked[sh] = best[1]
                apply(sh, best[1])
            del xs, outs
            cache[key] = {json.dumps(list(k)): v for k, v in picked.items()}
            if use_cache:
                with _lock:
                    merged = _load()
                    merged.update(cache)
                    _save(merged)
        for sh, st in picked.items():
            choice[sh] = st
            apply(sh, st)
    return {sh: (choice[sh], tuned[(sh, choice[sh])]) for sh in shapes}
