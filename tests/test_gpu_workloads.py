"""GPU parity at the full workload sizes, in the launch configuration the
benchmark times.

* 512^3 complex64 and complex128, grid 1x1 (the headline step): forward and
  inverse against the FP64 oracle on every output.
* 256^3 complex64 and complex128, pencil grid 4x4: forward and inverse against
  the oracle on every output.
* 840^3 complex64 (radix-7 lengths, the largest grid of the paper's GPU
  runs) by 32 sampled outputs and the round trip.
* 1024^3 real float32 turbulence field, pencil grid 8x8, R2C then C2R: the
  FP64 oracle cannot take the whole transform in test time, so (i) 82 outputs
  (18 low and Nyquist modes plus 64 seeded random ones) against
  per-point O(N) oracle sums, with their error measured against the field's
  spectral RMS known exactly from Parseval; (ii) Parseval on the GPU half
  spectrum; (iii) the C2R round trip on every point.
"""
import math

import numpy as np
import pytest
import torch

import oracle
import synth
from _util import bound, fp32_bound, promoted, rel, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", [torch.complex64, torch.complex128], ids=["c64", "c128"])
def test_headline_512cubed_full_field(gpu_lib, dtype):
    cfg = synth.HEADLINE
    print(f"case 512^3 {dtype} grid 1x1", flush=True)
    a = synth.complex_normal(cfg["shape"], cfg["seed"], np.complex64 if dtype == torch.complex64 else np.complex128)
    x = to_dev(a, dtype)
    plan = gpu_lib.Plan(cfg["shape"], dtype, (1, 1), streams=1)
    X = plan.forward(x)
    Y = plan.inverse(X)
    torch.cuda.synchronize()
    ref_in = promoted(a, dtype)
    del x
    want = oracle.fftn(ref_in)
    tol = bound(dtype, a.size)
    err = rel(to_host(X), want)
    print(f"forward rel-L2 {err:.3e} (bound {tol:.1e})", flush=True)
    assert err <= tol
    del want, X
    err = rel(to_host(Y), ref_in)
    print(f"round trip rel-L2 {err:.3e}", flush=True)
    assert err <= tol
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
    assert rel(to_host(X), oracle.fftn(ref_in)) <= tol
    assert rel(to_host(Y), oracle.ifftn(oracle.fftn(ref_in))) <= tol
    plan.close()


def _sample_points(shape, fixed, rng, n_random):
    """The fixed (kz, ky, kx) points plus n_random distinct seeded ones."""
    nz, ny, nx = shape
    pts = [tuple(p) for p in fixed]
    while len(pts) < len(fixed) + n_random:
        p = (int(rng.integers(nz)), int(rng.integers(ny)), int(rng.integers(nx // 2 + 1)))
        if p not in pts:
            pts.append(p)
    return np.array(pts, dtype=np.int64)


@pytest.mark.timeout(900)
def test_config3_1024cubed_r2c_turbulence(gpu_lib):
    cfg = synth.CFG3
    shape = cfg["shape"]
    nz, ny, nx = shape
    n = nz * ny * nx
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

    # (i) sampled outputs against per-point oracle sums; error relative to the
    # spectral RMS over all N outputs (= sqrt(field_energy / N))
    rng = np.random.default_rng(1234)
    low = [(0, 0, 1), (0, 1, 0), (1, 0, 0), (0, 1, 1), (1, 1, 0), (1, 0, 1), (1, 1, 1), (0, 0, 2),
           (0, 2, 0), (2, 0, 0), (0, ny - 1, 1), (nz - 1, 0, 1), (nz - 1, ny - 1, 1), (0, 0, nx // 2),
           (0, ny // 2, 0), (nz // 2, 0, 0), (nz // 2, ny // 2, nx // 2), (0, 0, 0)]
    pts = _sample_points(shape, low, rng, 64)
    want = oracle.dft3d_points(u64, pts)
    Hh = H[pts[:, 0], pts[:, 1], pts[:, 2]].cpu().numpy().astype(np.complex128)
    rms_all = math.sqrt(field_energy / n)
    err = float(np.sqrt(np.mean(np.abs(Hh - want) ** 2)) / rms_all)
    print(f"sampled error / spectral RMS: {err:.3e} (bound {fp32_bound(n):.1e})", flush=True)
    assert err <= fp32_bound(n)
    del u64

    # (iii) round trip on every point
    back = plan.inverse(H)
    torch.cuda.synchronize()
    del H
    err = rel(to_host(back), u.astype(np.float64))
    print(f"round trip rel-L2 {err:.3e}", flush=True)
    assert err <= fp32_bound(n)
    plan.close()


@pytest.mark.timeout(900)
def test_840cubed_radix7_sampled(gpu_lib):
    """The largest grid of the paper's GPU runs, 840^3 = (8*3*5*7)^3 complex64, on
    one GPU: 32 seeded outputs against per-point oracle sums (error measured
    against the spectral RMS from Parseval) and the round trip on every point."""
    shape = (840, 840, 840)
    n = 840 ** 3
    print("case 840^3 c64: building the field", flush=True)
    a = synth.complex_normal(shape, 8, np.complex64)
    x = torch.from_numpy(a).cuda()
    plan = gpu_lib.Plan(shape, torch.complex64)
    X = plan.forward(x)
    torch.cuda.synchronize()
    rng = np.random.default_rng(99)
    pts = np.stack([rng.integers(840, size=32) for _ in range(3)], axis=1)
    pts[0] = (0, 0, 0)
    pts[1] = (0, 0, 1)
    a128 = a.astype(np.complex128)
    want = oracle.dft3d_points(a128, pts)
    got = X[pts[:, 0], pts[:, 1], pts[:, 2]].cpu().numpy().astype(np.complex128)
    rms_all = math.sqrt(n * float(np.vdot(a128.ravel(), a128.ravel()).real) / n)
    err = float(np.sqrt(np.mean(np.abs(got - want) ** 2)) / rms_all)
    print(f"sampled error / spectral RMS: {err:.3e}", flush=True)
    assert err <= fp32_bound(n)
    del a128
    Y = plan.inverse(X)
    torch.cuda.synchronize()
    del X
    err = rel(to_host(Y), a.astype(np.complex128))
    print(f"round trip rel-L2 {err:.3e}", flush=True)
    assert err <= fp32_bound(n)
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
    assert torch.equal(got, ref), chosen
    # second plan of the same shape takes the cached choice
    p2 = gpu_lib.Plan(shape, torch.complex64)
    again = autotune.tune_plan(p2, reps=2)
    assert all(again[k] == v for k, v in chosen.items())
    assert torch.equal(p2.forward(x), ref)
    plan.close()
    p2.close()
