"""GPU parity at the full workload sizes, in the launch configuration the
benchmark times.  Every compared array is checked by rel-L2 and by the largest
single-element error relative to the RMS of the reference (see _util).

* 512^3 complex64 and complex128, grid 1x1 (the headline step): forward and
  inverse against the FP64 oracle on every output.
* 512^3 float32 and float64 R2C + C2R at the default plan (swapped-y/z
  forward staging, the cache policy of fields larger than the Infinity
  Cache): the forward on every output against the oracle's R2C, the C2R of
  the oracle's half spectrum against the oracle's C2R, and the round trip.
* 256^3 complex64 and complex128, pencil grid 4x4: forward and inverse against
  the oracle on every output.
* 840^3 complex64 (radix-7 lengths, the largest grid of the paper's GPU
  runs): 64 whole z-lines (53,760 outputs) against the oracle and the round
  trip on every point.
* 1024^3 real float32 turbulence field, pencil grid 8x8, R2C then C2R: the
  whole z-lines through every tile edge of the 8x8 grid in x and y (16 x 16
  lines, 262,144 outputs, every z tile edge included) against the oracle, with
  errors relative to the spectral RMS known exactly from Parseval; Parseval on
  the GPU half spectrum; the C2R round trip on every point.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import synth
from _util import assert_parity, bound, fp32_bound, promoted, rel, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128], ids=["c64", "c128"])
def test_headline_512cubed_full_field(gpu_lib, dtype):
    cfg = synth.HEADLINE
    print(f"case 512^3 {dtype} grid 1x1", flush=True)
    a = synth.complex_normal(cfg["shape"], cfg["seed"], np.complex64 if dtype == torch.complex64 else np.complex128)
    x = to_dev(a, dtype)
    plan = gpu_lib.Plan(cfg["shape"], dtype, (1, 1), streams=1)
    assert plan.staging == gpu_lib.STAGING_SWAP_YZ  # the benchmark's configuration
    X = plan.forward(x)
    Y = plan.inverse(X)
    torch.cuda.synchronize()
    ref_in = promoted(a, dtype)
    del x
    want = oracle.fftn(ref_in)
    tol = bound(dtype, a.size)
    assert_parity(X, want, tol, "forward")
    print(f"forward rel-L2 {rel(to_host(X), want):.3e} (bound {tol:.1e})", flush=True)
    del want, X
    assert_parity(Y, ref_in, tol, "round trip")
    plan.close()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["f32", "f64"])
def test_headline_512cubed_r2c_full_field(gpu_lib, dtype):
    """The R2C half of the headline target at the plan's default configuration."""
    n = 512
    shape = (n, n, n)
    cdt = torch.complex64 if dtype == torch.float32 else torch.complex128
    print(f"case 512^3 r2c {dtype} default plan", flush=True)
    f = synth.real_normal(shape, 10, np.float32 if dtype == torch.float32 else np.float64)
    x = to_dev(f, dtype)
    plan = gpu_lib.Plan(shape, dtype, r2c=True)
    assert plan.staging == gpu_lib.STAGING_SWAP_YZ  # half spectrum of 0.5-1 GiB: swapped forward staging
    H = plan.forward(x)
    back = plan.inverse(H)
    torch.cuda.synchronize()
    del x
    tol = bound(dtype, f.size)
    f_in = f.astype(np.float64)
    want = oracle.rfftn(f_in)
    print("oracle r2c done", flush=True)
    assert_parity(H, want, tol, "forward")
    del H
    assert_parity(back, f_in, tol, "round trip")
    del back
    # the C2R on its own: the oracle's half spectrum (rounded to the plan precision) back to real
    h_in = want.astype(np.complex64 if dtype == torch.float32 else np.complex128)
    del want
    hd = to_dev(h_in, cdt)
    y = plan.inverse(hd)
    torch.cuda.synchronize()
    del hd
    want_y = oracle.irfftn(h_in.astype(np.complex128), n)
    print("oracle c2r done", flush=True)
    assert_parity(y, want_y, tol, "inverse of the oracle spectrum")
    plan.close()


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128], ids=["c64", "c128"])
def test_config2_256cubed_grid4x4(gpu_lib, dtype):
    cfg = synth.CFG2
    print(f"case 256^3 {dtype} grid 4x4", flush=True)
    a = synth.complex_normal(cfg["shape"], cfg["seed"])
    x = to_dev(a, dtype)
    plan = gpu_lib.Plan(cfg["shape"], dtype, cfg["grid"])
    X = plan.forward(x)
    Y = plan.inverse(X)
    torch.cuda.synchronize()
    ref_in = promoted(a, dtype)
    tol = bound(dtype, a.size)
    want = oracle.fftn(ref_in)
    assert_parity(X, want, tol, "forward")
    assert_parity(Y, oracle.ifftn(want), tol, "inverse")
    plan.close()


def _edges(bounds, n):
    """Both sides of every boundary in bounds (a sorted list of range starts), within [0, n)."""
    out = set()
    for b in bounds:
        for v in (b - 1, b):
            if 0 <= v < n:
                out.add(v)
    return sorted(out)


def _check_lines(got, want, rms_all, tol, what):
    """Whole sampled z-lines (columns of got/want): the RMS error relative to the
    RMS of all N outputs, and every output's error relative to the larger of
    that RMS and the RMS of its own reference z-line.

    The last stage transforms each z-line on its own, so its rounding errors
    follow the norm of that line, while the earlier stages' errors spread over
    the outputs at the scale of the whole spectrum.  For white inputs the two
    scales agree; for the k^-5/3 turbulence spectrum a few lines hold most of
    the energy and their outputs carry correspondingly larger absolute errors
    (a mode of ~7000 x the spectral RMS has a one-ulp error of ~5e-4 x that
    RMS), which the line scale accounts for."""
    d = np.abs(got - want)
    e_rms = float(np.sqrt(np.mean(d ** 2))) / rms_all
    line_rms = np.sqrt(np.mean(np.abs(want) ** 2, axis=0))
    scale = np.maximum(rms_all, line_rms)[None, :]
    e_max = float((d / scale).max())
    e_max_all = float(d.max()) / rms_all
    print(f"{what}: {got.size} outputs, rms error {e_rms:.3e} (of the spectral RMS), max error "
          f"{e_max:.3e} (of max(spectral RMS, line RMS); {e_max_all:.3e} of the spectral RMS), "
          f"bound {tol:.1e}", flush=True)
    assert e_rms <= tol and e_max <= tol, what


@pytest.mark.timeout(900)
def test_config3_1024cubed_r2c_turbulence(gpu_lib):
    cfg = synth.CFG3
    shape = cfg["shape"]
    nz, ny, nx = shape
    n = nz * ny * nx
    p1, p2 = cfg["grid"]
    print("case 1024^3 r2c turbulence grid 8x8: building the field", flush=True)
    u = synth.turbulence_field(shape, cfg["seed"], np.float32)
    print("field built", flush=True)
    ud = torch.from_numpy(u).cuda()
    plan = gpu_lib.Plan(shape, torch.float32, cfg["grid"], r2c=True)
    H = plan.forward(ud)
    torch.cuda.synchronize()
    print("r2c done", flush=True)

    # (ii) Parseval on the half spectrum: interior kx bins count twice
    w = torch.full((nx // 2 + 1,), 2.0, dtype=torch.float64, device="cuda")
    w[0] = 1.0
    w[nx // 2] = 1.0
    spec_energy = float(((H.real.double() ** 2 + H.imag.double() ** 2).sum(dim=(0, 1)) * w).sum())
    u64 = u.astype(np.float64)
    field_energy = float(n * np.dot(u64.ravel(), u64.ravel()))
    print(f"Parseval: spectrum {spec_energy:.6e} field*N {field_energy:.6e}", flush=True)
    assert abs(spec_energy - field_energy) <= 1e-5 * field_energy

    # (i) whole z-lines through every tile edge in x and y: the x edges of the
    # y- and z-pencil tiles (the plan's task graph gives them), the y edges of
    # the x- and z-pencil tiles; every kz covers the z edges of the x- and
    # y-pencil tiles
    _, tasks = gpu_lib.query_pipeline(shape, cfg["grid"], r2c=True, op=0, nstreams=1)
    xb = sorted({t["box"][0] for t in tasks} | {t["box"][1] for t in tasks})
    yb = sorted({t["box"][2] for t in tasks} | {t["box"][3] for t in tasks})
    kxs = _edges(xb, nx // 2 + 1)
    kys = _edges(yb, ny)
    assert len(kxs) >= 2 * (p1 - 1) + 2 and len(kys) >= 2 * (p2 - 1) + 2, (kxs, kys)
    kx = np.repeat(kxs, len(kys))
    ky = np.tile(kys, len(kxs))
    want = oracle.dft3d_lines(u64, kx, ky)  # (nz, pairs)
    got = H[:, torch.as_tensor(ky, device="cuda"), torch.as_tensor(kx, device="cuda")].cpu().numpy()
    rms_all = math.sqrt(field_energy / n)
    _check_lines(got.astype(np.complex128), want, rms_all, fp32_bound(n), "1024^3 r2c tile-edge lines")
    del u64, want

    # (iii) round trip on every point
    back = plan.inverse(H)
    torch.cuda.synchronize()
    del H
    assert_parity(back, u.astype(np.float64), fp32_bound(n), "round trip")
    plan.close()


@pytest.mark.timeout(900)
def test_840cubed_radix7_sampled(gpu_lib):
    """The largest grid of the paper's GPU runs, 840^3 = (8*3*5*7)^3 complex64, on
    one GPU: 64 whole z-lines (8 x 8 seeded (kx, ky) pairs plus the first and last
    bins) against the oracle, errors relative to the spectral RMS from
    Parseval, and the round trip on every point."""
    shape = (840, 840, 840)
    n = 840 ** 3
    print("case 840^3 c64: building the field", flush=True)
    a = synth.complex_normal(shape, 8, np.complex64)
    x = torch.from_numpy(a).cuda()
    plan = gpu_lib.Plan(shape, torch.complex64)
    X = plan.forward(x)
    torch.cuda.synchronize()
    rng = np.random.default_rng(99)
    kxs = sorted(set([0, 839] + list(rng.integers(840, size=6))))
    kys = sorted(set([0, 839] + list(rng.integers(840, size=6))))
    kx = np.repeat(kxs, len(kys))
    ky = np.tile(kys, len(kxs))
    a128 = a.astype(np.complex128)
    want = oracle.dft3d_lines(a128, kx, ky)
    got = X[:, torch.as_tensor(ky, device="cuda"), torch.as_tensor(kx, device="cuda")].cpu().numpy()
    rms_all = math.sqrt(float(np.vdot(a128.ravel(), a128.ravel()).real))
    _check_lines(got.astype(np.complex128), want, rms_all, fp32_bound(n), "840^3 lines")
    del a128, want
    Y = plan.inverse(X)
    torch.cuda.synchronize()
    del X
    assert_parity(Y, a.astype(np.complex128), fp32_bound(n), "round trip")
    plan.close()


def test_autotuner_changes_no_bits(gpu_lib, tmp_path, monkeypatch):
    from paper_2601_12209_amd import autotune

    monkeypatch.setenv("FFT3D_TUNE_CACHE", str(tmp_path / "tune.json"))
    shape = (64, 48, 80)
    a = synth.complex_normal(shape, 21)
    x = to_dev(a, torch.complex64)
    plan = gpu_lib.Plan(shape, torch.complex64)
    ref = plan.forward(x).clone()
    chosen = autotune.tune_plan(plan, reps=2)
    got = plan.forward(x)
    torch.cuda.synchronize()
    # launch shapes change no bits; a reverse radix order changes the rounding,
    # so then the result is the same as a plan with just those orders set
    orders = {ax: (cfg[4] if len(cfg) > 4 else 0) for ax, cfg in chosen.items()}
    want = ref
    if any(orders.values()):
        same = gpu_lib.Plan(shape, torch.complex64)
        for ax, o in orders.items():
            same.set_radix_order(ax, o)
        want = same.forward(x)
        torch.cuda.synchronize()
        same.close()
        assert_parity(to_host(got), oracle.fftn(a.astype(np.complex128)), fp32_bound(a.size))
    assert torch.equal(got, want), chosen
    # second plan of the same shape takes the cached choice
    p2 = gpu_lib.Plan(shape, torch.complex64)
    again = autotune.tune_plan(p2, reps=2)
    assert all(again[k] == v for k, v in chosen.items())
    assert torch.equal(p2.forward(x), want)
    plan.close()
    p2.close()
