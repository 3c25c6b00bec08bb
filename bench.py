#!/usr/bin/env python3
"""Benchmark of the pencil 3D FFT on one MI355X.

One step = forward + inverse 3D C2C FFT of a 512^3 complex64 field (the
headline workload): x, y, z stages in both directions (the library's default
staging for this size: the y stage writes a y/z-swapped workspace that the z
stage reads back), every stage a batch of 1D Stockham FFTs over its pencil
tiles.  The input (i.i.d. N(0,1)
real and imaginary parts, seed 0) is resident in HBM before timing starts.

Reported (one JSON line):
  value       GFLOP/s = 2 transforms * 5 N log2 N / (seconds per step), FP32 path
  fp64        the same workload in complex128, and the FP32/FP64 speedup
  stages      per-stage milliseconds and achieved GB/s (2 * elem bytes * N per stage)
  roofline    the slowest stage kernel against the 8 TB/s HBM peak
  cpu_baseline the FP64 oracle on the same field on the host cores, with the
              rel-L2 error of the GPU results against it
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

HBM_PEAK_GBS = 8000.0
ROOT = os.path.dirname(os.path.abspath(__file__))
TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "traffic_c2c_512cubed.json")


def kernel_source_hash() -> str:
    """sha256 over the library sources (kernels and launch shapes); a counter record is
    valid only for the sources it was taken with."""
    import glob
    import hashlib

    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2601_12209_amd", "csrc")
    for p in sorted(glob.glob(os.path.join(csrc, "*.hip")) + glob.glob(os.path.join(csrc, "*.hpp"))
                    + glob.glob(os.path.join(csrc, "*.cpp"))):
        h.update(os.path.basename(p).encode())
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(n_edge):
    """HBM bytes per launch of the dominant stage kernel from the committed
    rocprofv3 counter record, or None if it is absent or the kernels changed."""
    try:
        with open(TRAFFIC_RECORD) as fh:
            rec = json.load(fh)
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != kernel_source_hash() or rec.get("n_edge") != n_edge:
        return None
    return rec["read_bytes_per_launch"] + rec["write_bytes_per_launch"]
DEFAULT_GRID = (1, 1)
DEFAULT_STREAMS = 1
STAGINGS = {"in_place": 0, "swap_yz": 1}
DEFAULT_STAGING = "swap_yz"


def _timed_steps(step, steps, warmup, torch):
    """Mean ms per step over the timed region, its wall time, and the median
    of the per-step times (an event recorded on the stream after each step)."""
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    events = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    t0 = time.perf_counter()
    events[0].record()
    for i in range(steps):
        step()
        events[i + 1].record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per_step = sorted(events[i].elapsed_time(events[i + 1]) for i in range(steps))
    mid = steps // 2
    median = per_step[mid] if steps % 2 else 0.5 * (per_step[mid - 1] + per_step[mid])
    return events[0].elapsed_time(events[-1]) / steps, wall, median


def _stage_profile(plan, x, X, Y, reps, torch):
    """Average per-stage milliseconds of forward and inverse (timing mode)."""
    plan.set_timing(True)
    fwd, inv = None, None
    for _ in range(reps):
        plan.forward(x, out=X)
        f = plan.stage_times()
        plan.inverse(X, out=Y)
        i = plan.stage_times()
        fwd = f if fwd is None else [a + b for a, b in zip(fwd, f)]
        inv = i if inv is None else [a + b for a, b in zip(inv, i)]
    plan.set_timing(False)
    torch.cuda.synchronize()
    return [v / reps for v in fwd], [v / reps for v in inv]


def _measure(dtype, shape, grid, streams, steps, warmup, a_host, torch, fft3d, staging=0):
    x = torch.from_numpy(a_host).to(device="cuda", dtype=dtype)
    X = torch.empty_like(x)
    Y = torch.empty_like(x)
    plan = fft3d.Plan(shape, dtype, grid, streams=streams, staging=staging)

    def step():
        plan.forward(x, out=X)
        plan.inverse(X, out=Y)

    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        ms, wall, ms_median = _timed_steps(step, steps, warmup, torch)
    fwd_st, inv_st = _stage_profile(plan, x, X, Y, max(3, min(steps, 10)), torch)
    plan.forward(x, out=X)
    plan.inverse(X, out=Y)
    torch.cuda.synchronize()
    plan.close()
    return dict(ms=ms, ms_median=ms_median, wall=wall, fwd_stages=fwd_st, inv_stages=inv_st, X=X, Y=Y)


def _time(fn, reps, torch):
    for _ in range(2):
        fn()
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    end = torch.cuda.Event(enable_timing=True)
    start.record()
    for _ in range(reps):
        fn()
    end.record()
    torch.cuda.synchronize()
    return start.elapsed_time(end) / reps


def _progress(msg):
    print(f"# {msg}", file=sys.stderr, flush=True)


EXTRAS = ("r2c512", "grid256", "r2c1024", "c840", "batch", "poisson", "ppb")


def _extras(reps, torch, fft3d, synth, np, only=EXTRAS):
    """The other workloads (those named in `only`), timed on the GPU.  Returns
    (report, checks) where checks holds (name, GPU result on the host, function
    giving the FP64 oracle result) for the CPU-baseline leg."""
    rep, checks = {}, []

    def want(name):
        return name in only

    n = 512
    N = n ** 3
    nh = (n // 2 + 1) * n * n
    side = torch.cuda.Stream()
    if want("r2c512"):
        for dt, tag, sr, npdt in ((torch.float32, "f32", 4, np.float32), (torch.float64, "f64", 8, np.float64)):
            _progress(f"extras: 512^3 r2c {tag}")
            f = synth.real_normal((n, n, n), 10, npdt)
            x = torch.from_numpy(f).cuda()
            p = fft3d.Plan((n, n, n), dt, r2c=True)
            H = p.forward(x)
            y = p.inverse(H)
            ms = _time(lambda: (p.forward(x, out=H), p.inverse(H, out=y)), reps, torch)
            bytes_moved = 2 * N * sr + 10 * nh * 2 * sr  # x stage real in/out, 5 half-spectrum passes each way
            rep[f"r2c_512cubed_fwd_inv_{tag}"] = {
                "ms": round(ms, 4), "GFLOP/s (2.5 N log2 N per transform)": round(2 * 2.5 * N * math.log2(N) / (ms * 1e-3) / 1e9, 1),
                "hbm_frac": round(bytes_moved / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
            Hh, yh = H.cpu().numpy(), y.cpu().numpy()
            checks.append((f"r2c_512cubed_{tag}_forward", Hh, lambda f=f: _oracle().rfftn(f.astype(np.float64))))
            checks.append((f"r2c_512cubed_{tag}_roundtrip", yh, lambda f=f: f.astype(np.float64)))
            p.close()
            del x, H, y
            torch.cuda.empty_cache()
    if want("grid256"):
        # 256^3 C2C on the 4x4 pencil grid of tiles, and 1x1 for comparison
        cfg = synth.CFG2
        m = cfg["shape"][0] ** 3
        a = synth.complex_normal(cfg["shape"], cfg["seed"], np.complex64)
        side = torch.cuda.Stream()
        for dt, tag, es in ((torch.complex64, "c64", 8), (torch.complex128, "c128", 16)):
            _progress(f"extras: 256^3 c2c {tag}")
            x = torch.from_numpy(a).to("cuda", dt)
            g2 = tuple(cfg["grid"])
            for grid, ns, issue, suffix in ((g2, 4, fft3d.ISSUE_STAGES, ""), (g2, 4, fft3d.ISSUE_TILES, "_tiles"),
                                            ((1, 1), 1, fft3d.ISSUE_STAGES, "")):
                p = fft3d.Plan(cfg["shape"], dt, grid, streams=ns, issue=issue)
                X = p.forward(x)
                Y = torch.empty_like(X)
                with torch.cuda.stream(side):
                    ms = _time(lambda: (p.forward(x, out=X), p.inverse(X, out=Y)), reps, torch)
                name = f"c2c_256cubed_{tag}_grid{grid[0]}x{grid[1]}{suffix}"
                rep[name] = {
                    "ms": round(ms, 4), "GFLOP/s": round(2 * 5 * m * math.log2(m) / (ms * 1e-3) / 1e9, 1),
                    "hbm_frac": round(12 * es * m / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                    "issue": (f"tiles on {ns} stream(s)" if issue == fft3d.ISSUE_TILES or grid == (1, 1)
                              else "one grouped launch per stage")}
                if grid != (1, 1) and issue == fft3d.ISSUE_STAGES:
                    torch.cuda.synchronize()
                    checks.append((f"c2c_256cubed_{tag}_forward", X.cpu().numpy(),
                                   lambda: _oracle().fftn(a.astype(np.complex128))))
                p.close()
            del x
            torch.cuda.empty_cache()
    if want("r2c1024"):
        # 1024^3 float32 R2C + C2R on the 8x8 pencil grid of tiles (one grouped
        # launch per stage, and one launch per tile on the plan's streams) and on
        # one tile per stage; the values do not change the
        # timing, so the input is torch's normal generator (parity of the
        # turbulence field at this size is a GPU test)
        c3 = synth.CFG3
        m3 = int(np.prod(c3["shape"]))
        nh3 = (c3["shape"][2] // 2 + 1) * c3["shape"][0] * c3["shape"][1]
        x = torch.randn(c3["shape"], dtype=torch.float32, device="cuda")
        g3 = tuple(c3["grid"])
        for grid, issue, suffix in ((g3, fft3d.ISSUE_STAGES, ""), (g3, fft3d.ISSUE_TILES, "_tiles"),
                                    ((1, 1), fft3d.ISSUE_STAGES, "")):
            _progress(f"extras: 1024^3 r2c grid {grid}{suffix}")
            p = fft3d.Plan(c3["shape"], torch.float32, grid, r2c=True, issue=issue)
            H = p.forward(x)
            y = torch.empty_like(x)
            with torch.cuda.stream(side):
                ms = _time(lambda: (p.forward(x, out=H), p.inverse(H, out=y)), max(3, reps // 2), torch)
            bytes_moved = 2 * m3 * 4 + 10 * nh3 * 2 * 4
            rep[f"r2c_1024cubed_f32_grid{grid[0]}x{grid[1]}{suffix}"] = {
                "ms": round(ms, 4), "GFLOP/s (2.5 N log2 N per transform)": round(2 * 2.5 * m3 * math.log2(m3) / (ms * 1e-3) / 1e9, 1),
                "hbm_frac": round(bytes_moved / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "issue": ("one tile per stage" if grid == (1, 1) else
                          "tiles on 4 streams" if issue == fft3d.ISSUE_TILES else "one grouped launch per stage")}
            p.close()
            del H, y
        del x
        torch.cuda.empty_cache()
    if want("c840"):
        # 840^3 complex64: the largest grid of the paper's GPU runs (lengths with a
        # factor 7), whole on one GPU; parity is covered by the GPU tests
        _progress("extras: 840^3 c2c")
        n8 = 840
        m8 = n8 ** 3
        x = torch.randn((n8, n8, n8), dtype=torch.complex64, device="cuda")
        p = fft3d.Plan((n8, n8, n8), torch.complex64)
        X = p.forward(x)
        Y = torch.empty_like(X)
        with torch.cuda.stream(side):
            ms = _time(lambda: (p.forward(x, out=X), p.inverse(X, out=Y)), max(3, reps // 2), torch)
        rep["c2c_840cubed_c64_grid1x1"] = {
            "ms": round(ms, 4), "GFLOP/s": round(2 * 5 * m8 * math.log2(m8) / (ms * 1e-3) / 1e9, 1),
            "hbm_frac": round(12 * 8 * m8 / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        p.close()
        del x, X, Y
        torch.cuda.empty_cache()
    if want("batch"):
        # 64 uneven transforms, one grouped launch per shape and stage, on a
        # non-default stream
        _progress("extras: 64 uneven transforms")
        shapes = synth.batch_sizes()
        host = synth.batch_inputs(shapes, synth.CFG4["seed"])
        xs = [torch.from_numpy(h).cuda() for h in host]
        outs = [torch.empty_like(t) for t in xs]
        pts = sum(int(np.prod(sh)) for sh in shapes)
        flops = sum(5 * np.prod(sh) * math.log2(np.prod(sh)) for sh in shapes)
        # shapes whose planes fit the fused x-y kernel take two passes over HBM
        # (the batch's default there), the others three
        probe = fft3d.BatchPlan(shapes)
        fused = set()
        for sh in set(shapes):
            try:
                probe.set_staging(sh, fft3d.STAGING_FUSED_XY)
                fused.add(sh)
            except RuntimeError:
                pass
        probe.close()
        brep = {"transforms": len(shapes), "points": pts}
        side = torch.cuda.Stream()
        # launch shapes per transform shape from the autotuner (untimed; measured
        # once, then taken from its cache file, a temporary one here)
        from paper_2601_12209_amd import autotune
        import tempfile
        tune_path = os.path.join(tempfile.gettempdir(), f"fft3d_tune_{os.getpid()}.json")
        own_cache = "FFT3D_TUNE_CACHE" not in os.environ
        if own_cache:
            os.environ["FFT3D_TUNE_CACHE"] = tune_path
        brep["launch_shapes"] = "autotuned (launch shapes per stage, staging per shape)"
        bp = fft3d.BatchPlan(shapes)
        autotune.tune_batch(bp, reps=5)
        # bytes of the passes made: two for shapes in fused x-y planes, three otherwise
        tuned_fused = sorted(sh for sh in set(shapes) if bp.staging(sh) == fft3d.STAGING_FUSED_XY)
        bbytes = sum((2 if sh in tuned_fused else 3) * 2 * 8 * int(np.prod(sh)) for sh in shapes)
        brep["fused_xy_shapes"] = tuned_fused
        brep["hbm_bytes_per_call"] = bbytes
        with torch.cuda.stream(side):
            ms = _time(lambda: bp.forward(xs, outs), reps, torch)
        brep["grouped"] = {"ms": round(ms, 4), "GFLOP/s": round(flops / (ms * 1e-3) / 1e9, 1),
                              "hbm_frac": round(bbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        bp.close()
        # for comparison: the same transforms one after another, each through its own
        # plan (the batch's default staging per shape, default launch shapes) on one
        # stream
        plans = {}
        for sh in set(shapes):
            pl = fft3d.Plan(sh, torch.complex64)
            if sh in fused:
                pl.set_staging(fft3d.STAGING_FUSED_XY)
            else:
                pl.set_staging(fft3d.STAGING_IN_PLACE)
            plans[sh] = pl

        def serial():
            for sh, x_, o_ in zip(shapes, xs, outs):
                plans[sh].forward(x_, out=o_)

        with torch.cuda.stream(side):
            ms = _time(serial, reps, torch)
        sbytes = sum((2 if sh in fused else 3) * 2 * 8 * int(np.prod(sh)) for sh in shapes)
        brep["serial_one_stream"] = {"ms": round(ms, 4), "GFLOP/s": round(flops / (ms * 1e-3) / 1e9, 1),
                                     "hbm_frac": round(sbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        for pl in plans.values():
            pl.close()
        bp = fft3d.BatchPlan(shapes)
        autotune.tune_batch(bp, reps=5)
        with torch.cuda.stream(side):
            bp.forward(xs, outs)
        torch.cuda.synchronize()
        bp.close()
        if own_cache:
            del os.environ["FFT3D_TUNE_CACHE"]
            try:
                os.remove(tune_path)
            except OSError:
                pass
        rep["batched_64_uneven_c64"] = brep
        checks.append(("batched_64_uneven_forward_worst", [o.cpu().numpy() for o in outs],
                       lambda: [_oracle().fftn(h.astype(np.complex128)) for h in host]))
        del xs, outs
        torch.cuda.empty_cache()
    if want("poisson"):
        # differentiable Poisson solve, 256^3 float32: forward solve + adjoint (one gradient step)
        _progress("extras: 256^3 Poisson")
        c5 = synth.CFG5
        f = synth.smooth_field(c5["shape"], c5["seed_f"], c5["sigma"], np.float32)
        w = synth.real_normal(c5["shape"], c5["seed_w"], np.float32)
        fd, wd = torch.from_numpy(f).cuda(), torch.from_numpy(w).cuda()
        p = fft3d.Plan(c5["shape"], torch.float32, r2c=True)
        phi = p.poisson(fd)
        g = p.poisson_backward(wd)
        ms = _time(lambda: (p.poisson(fd, out=phi), p.poisson_backward(wd, out=g)), reps, torch)
        m = int(np.prod(c5["shape"]))
        mh = (c5["shape"][2] // 2 + 1) * c5["shape"][0] * c5["shape"][1]
        pbytes = 2 * (2 * m * 4 + 8 * mh * 8)  # per solve: real in/out + 4 half-spectrum passes
        rep["poisson_256cubed_f32_solve_plus_adjoint"] = {
            "ms": round(ms, 4), "hbm_frac": round(pbytes / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
        checks.append(("poisson_256cubed_solution", phi.cpu().numpy(), lambda: _oracle().poisson(f.astype(np.float64))))
        checks.append(("poisson_256cubed_gradient", g.cpu().numpy(), lambda: _oracle().poisson_grad(w.astype(np.float64))))
        p.close()
    if want("ppb"):
        # (Periodic, Periodic, Bounded) topology, 256^3 float32: Poisson solve
        # and forward + inverse with a DCT (Neumann) or DST (Dirichlet) z axis
        c5 = synth.CFG5
        f = synth.smooth_field(c5["shape"], c5["seed_f"], c5["sigma"], np.float32)
        fd = torch.from_numpy(f).cuda()
        m = int(np.prod(c5["shape"]))
        mh = (c5["shape"][2] // 2 + 1) * c5["shape"][0] * c5["shape"][1]
        for wall, bc in (("neumann", 0), ("dirichlet", 1)):
            _progress(f"extras: 256^3 (P,P,B) {wall}")
            p = fft3d.Plan(c5["shape"], torch.float32, z_bc=wall)
            phi = p.poisson(fd)
            H = p.forward(fd)
            y = torch.empty_like(fd)
            ms_s = _time(lambda: p.poisson(fd, out=phi), reps, torch)
            ms_t = _time(lambda: (p.forward(fd, out=H), p.inverse(H, out=y)), reps, torch)
            sbytes = 2 * m * 4 + 8 * mh * 8  # real in/out + x, y, fused z, y, x half-spectrum passes
            tbytes = 2 * m * 4 + 10 * mh * 8  # real side once each way + 5 half-spectrum transfers each way
            rep[f"ppb_256cubed_f32_{wall}"] = {
                "poisson_ms": round(ms_s, 4), "poisson_hbm_frac": round(sbytes / (ms_s * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                "fwd_inv_ms": round(ms_t, 4), "fwd_inv_hbm_frac": round(tbytes / (ms_t * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
            checks.append((f"ppb_256cubed_{wall}_solution", phi.cpu().numpy(),
                           lambda bc=bc: _oracle().poisson_ppb(f.astype(np.float64), bc)))
            p.close()
    return rep, checks


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle():
    import oracle  # test infrastructure: used by the CPU-baseline leg only

    return oracle


def _extras_names(spec):
    if spec == "all":
        return EXTRAS
    names = tuple(v for v in spec.split(",") if v)
    bad = [v for v in names if v not in EXTRAS]
    if bad:
        raise SystemExit(f"unknown extras {bad}; choose from {EXTRAS}")
    return names


def _run_extras_child(args):
    """The other workloads in a child process (its own HIP context), so that a
    failure there cannot take the headline record with it.  Returns (report,
    rel-L2 errors against the oracle)."""
    import subprocess
    import tempfile

    fd, path = tempfile.mkstemp(prefix="fft3d_extras_", suffix=".json")
    os.close(fd)
    cmd = [sys.executable, os.path.abspath(__file__), "--extras-child", path, "--steps", str(args.steps),
           "--extras", args.extras]
    if args.no_cpu_baseline:
        cmd.append("--no-cpu-baseline")
    try:
        rc = subprocess.run(cmd).returncode
        if rc != 0:
            return {"error": f"extras process exited with status {rc}"}, {}
        with open(path) as fh:
            rec = json.load(fh)
        return rec["extras"], rec["errs"]
    finally:
        try:
            os.remove(path)
        except OSError:
            pass


def _extras_child(args):
    import numpy as np
    import torch

    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    import synth
    from paper_2601_12209_amd import fft3d

    fft3d.load()
    rep, checks = _extras(max(3, min(args.steps, 10)), torch, fft3d, synth, np, _extras_names(args.extras))
    errs = {}
    if not args.no_cpu_baseline:
        oracle = _oracle()
        _progress("extras: oracle comparisons")
        for name, got, ref_fn in checks:
            ref = ref_fn()
            if isinstance(got, list):
                errs[name] = max(oracle.rel_l2(g, r) for g, r in zip(got, ref))
            else:
                errs[name] = oracle.rel_l2(got, ref)
    with open(args.extras_child, "w") as fh:
        json.dump({"extras": rep, "errs": errs}, fh)


def main():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--size", type=int, default=512, help="grid edge (default 512)")
    ap.add_argument("--grid", type=int, nargs=2, default=list(DEFAULT_GRID), help="pencil grid P1 P2")
    ap.add_argument("--streams", type=int, default=DEFAULT_STREAMS)
    ap.add_argument("--staging", choices=sorted(STAGINGS), default=DEFAULT_STAGING,
                    help="in_place: y and z stages in place on the output; swap_yz: the y stage "
                         "writes a y/z-swapped workspace that the z stage reads back")
    ap.add_argument("--no-fp64", action="store_true", help="skip the complex128 run")
    ap.add_argument("--no-cpu-baseline", action="store_true", help="skip the oracle on the host")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the other workloads (R2C 512^3, 256^3 grid, batch, Poisson)")
    ap.add_argument("--extras", default="all",
                    help="comma-separated subset of the other workloads: " + ",".join(EXTRAS) + " (default all)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="after timing, copy the complex64 field once with a plain device copy "
                         "(a known-size reference for HBM byte counters)")
    ap.add_argument("--extras-child", metavar="PATH", help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.extras_child:
        _extras_child(args)
        return

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the pencil FFT here runs on a single MI355X "
              "(no multi-GPU path is built); run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))
    import synth
    from paper_2601_12209_amd import fft3d

    fft3d.load()
    n_edge = args.size
    shape = (n_edge, n_edge, n_edge)
    N = n_edge ** 3
    flop_per_transform = 5.0 * N * math.log2(N)
    grid = tuple(args.grid)
    print(f"# input: {shape} complex N(0,1), seed {synth.HEADLINE['seed']}", file=sys.stderr, flush=True)
    a = synth.complex_normal(shape, synth.HEADLINE["seed"], np.complex64)

    staging = STAGINGS[args.staging]
    r32 = _measure(torch.complex64, shape, grid, args.streams, args.steps, args.warmup, a, torch, fft3d, staging)
    print(f"# c64: {r32['ms']:.3f} ms/step", file=sys.stderr, flush=True)
    if args.copy_calibration:
        dst = torch.empty_like(r32["X"])
        dst.copy_(r32["X"])
        torch.cuda.synchronize()
        print(f"# copy calibration: {dst.numel() * 8} bytes read and written", file=sys.stderr, flush=True)
        del dst
    r64 = None
    if not args.no_fp64:
        a64 = a.astype(np.complex128)
        r64 = _measure(torch.complex128, shape, grid, args.streams, args.steps, args.warmup, a64, torch, fft3d,
                       staging)
        del a64
        print(f"# c128: {r64['ms']:.3f} ms/step", file=sys.stderr, flush=True)

    def stage_report(r, elem):
        names = ["x", "y", "z"]
        out = {}
        inv_order = names if staging == STAGINGS["swap_yz"] else names[::-1]
        for tag, st, order in (("fwd", r["fwd_stages"], names), ("inv", r["inv_stages"], inv_order)):
            for nm, ms in zip(order, st):
                gbs = 2.0 * elem * N / (ms * 1e-3) / 1e9
                out[f"{tag}_{nm}"] = {"ms": round(ms, 4), "GB/s": round(gbs, 1),
                                      "hbm_frac": round(gbs / HBM_PEAK_GBS, 4)}
        return out

    st32 = stage_report(r32, 8)
    gflops32 = 2 * flop_per_transform / (r32["ms"] * 1e-3) / 1e9
    # dominant kernel: the slowest stage (one kernel launch over the whole field at grid 1x1)
    dom_name, dom = max(st32.items(), key=lambda kv: kv[1]["ms"])
    bytes_per_launch = 2.0 * 8 * N
    achieved = bytes_per_launch / (dom["ms"] * 1e-3) / 1e9
    roofline = {"bound": "hbm", "kernel": f"stage {dom_name} (k_c2c<float, {n_edge}>)",
                "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(n_edge),
                "algorithmic_bytes_per_launch": bytes_per_launch}
    whole_frac = 6 * 2.0 * 8 * N / (r32["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS

    result = {
        "metric": "3D FFT GFLOP/s (5N·log2N/t) + % HBM peak, 512^3 C2C, FP32 vs FP64",
        "value": round(gflops32, 1),
        "unit": "GFLOP/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r32["ms"], 4),
        "ms_per_step_median": round(r32["ms_median"], 4),
        "higher_is_better": True,
        "scaling": "strong",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic: complex N(0,1) field, seed 0, resident in HBM",
        "config": {"workload": f"c2c_{n_edge}cubed_forward_plus_inverse", "nx": n_edge, "ny": n_edge,
                   "nz": n_edge, "precision": "complex64", "pencil_grid": list(grid),
                   "streams": args.streams, "staging": args.staging},
        "hbm_frac_whole_step": round(whole_frac, 4),
        "stages_c64": st32,
        "roofline": roofline,
        "wall_s_timed": round(r32["wall"], 4),
    }
    if r64 is not None:
        gflops64 = 2 * flop_per_transform / (r64["ms"] * 1e-3) / 1e9
        result["fp64"] = {"value": round(gflops64, 1), "unit": "GFLOP/s", "ms_per_step": round(r64["ms"], 4),
                          "ms_per_step_median": round(r64["ms_median"], 4),
                          "hbm_frac_whole_step": round(6 * 2.0 * 16 * N / (r64["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
                          "stages_c128": stage_report(r64, 16),
                          "fp32_over_fp64_speedup": round(r64["ms"] / r32["ms"], 3)}

    extras_errs = {}
    if not args.no_extras:
        # keep the headline results on the host for the oracle comparison, free the GPU
        for r in (r32, r64):
            if r is not None and not args.no_cpu_baseline:
                r["X"], r["Y"] = r["X"].cpu().numpy(), r["Y"].cpu().numpy()
            elif r is not None:
                r.pop("X"), r.pop("Y")
        torch.cuda.empty_cache()
        print("# extras (child process)", file=sys.stderr, flush=True)
        result["extras"], extras_errs = _run_extras_child(args)

    if not args.no_cpu_baseline:
        import oracle  # test infrastructure: the CPU baseline leg only

        a128 = a.astype(np.complex128)
        # the same step (forward + inverse) on the host cores, repeated for about
        # 10 s of work (at least 3 runs); the median run is reported
        runs = []
        while len(runs) < 3 or (sum(runs) < 10.0 and len(runs) < 9):
            t0 = time.perf_counter()
            X_ref = oracle.fftn(a128)
            Y_ref = oracle.ifftn(X_ref)
            runs.append(time.perf_counter() - t0)
        t_cpu = sorted(runs)[len(runs) // 2]
        def host(v):
            return v.cpu().numpy() if hasattr(v, "cpu") else v

        errs = {}
        if "X" in r32:
            errs["c64_forward"] = oracle.rel_l2(host(r32["X"]), X_ref)
            errs["c64_inverse_of_forward"] = oracle.rel_l2(host(r32["Y"]), a128)
        if r64 is not None:
            errs["c128_forward"] = oracle.rel_l2(host(r64["X"]), X_ref)
            errs["c128_inverse_of_forward"] = oracle.rel_l2(host(r64["Y"]), a128)
        del X_ref, Y_ref
        errs.update(extras_errs)
        result["cpu_baseline"] = {
            "value": round(2 * flop_per_transform / t_cpu / 1e9, 3), "unit": "GFLOP/s",
            "cores": oracle.num_threads(), "kind": "oracle",
            "host_cpus_available": len(os.sched_getaffinity(0)), "cpu_model": _cpu_model(),
            "sample": (f"FP64 forward + inverse of the same {n_edge}^3 field, median of {len(runs)} runs "
                       f"({t_cpu:.2f} s each, {sum(runs):.1f} s total)"),
            "rel_l2_vs_oracle": {k: float(f"{v:.3e}") for k, v in errs.items()},
        }
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
