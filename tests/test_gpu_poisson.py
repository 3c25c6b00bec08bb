"""GPU parity of the spectral Poisson solve and its adjoint (autograd).

phi = irfftn(M * rfftn(f)), M = -1/|k|^2, M(0) = 0, on a 2 pi periodic box.
The forward is compared with the FP64 oracle; the gradient of
L = sum(phi * w) is compared with the FP64 reference gradient (the solve is
self-adjoint, a fact the oracle pins separately) and with finite differences
(L is linear in f, so differences carry no truncation error).
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from _util import assert_parity, bound, promoted, rel, to_dev, to_host

pytestmark = pytest.mark.gpu

REAL = [torch.float32, torch.float64]


@pytest.mark.parametrize("dtype", REAL, ids=["f32", "f64"])
@pytest.mark.parametrize("shape,grid", [((8, 8, 8), (1, 1)), ((16, 12, 20), (2, 3)), ((32, 24, 40), (2, 2)),
                                        ((5, 6, 4), (1, 1)), ((64, 48, 100), (3, 3))])
def test_poisson_forward_and_adjoint(gpu_lib, shape, grid, dtype):
    print(f"case shape={shape} grid={grid} dtype={dtype}", flush=True)
    f = synth.real_normal(shape, 21)
    w = synth.real_normal(shape, 22)
    plan = gpu_lib.Plan(shape, dtype, grid, r2c=True)
    phi = plan.poisson(to_dev(f, dtype))
    gf = plan.poisson_backward(to_dev(w, dtype))
    torch.cuda.synchronize()
    n = f.size
    assert_parity(to_host(phi), oracle.poisson(promoted(f, dtype)), bound(dtype, n))
    assert_parity(to_host(gf), oracle.poisson_grad(promoted(w, dtype)), bound(dtype, n))
    plan.close()


def test_poisson_closed_form(gpu_lib):
    shape = (16, 12, 10)
    z, y, x = np.meshgrid(*(2 * np.pi * np.arange(n) / n for n in shape), indexing="ij")
    f = np.cos(3 * x + 2 * y + 1 * z)
    plan = gpu_lib.Plan(shape, torch.float64, (2, 2), r2c=True)
    phi = to_host(plan.poisson(to_dev(f, torch.float64)))
    np.testing.assert_allclose(phi, -f / 14.0, atol=1e-13)
    plan.close()


def test_poisson_in_place(gpu_lib):
    shape = (12, 10, 16)
    f = synth.real_normal(shape, 5)
    plan = gpu_lib.Plan(shape, torch.float64, (2, 2), r2c=True)
    t = to_dev(f, torch.float64)
    plan.poisson(t, out=t)
    torch.cuda.synchronize()
    assert_parity(to_host(t), oracle.poisson(f), 1e-12)
    plan.close()


def test_autograd_gradcheck_fp64(gpu_lib):
    f = to_dev(synth.real_normal((6, 4, 8), 3), torch.float64).requires_grad_(True)
    assert torch.autograd.gradcheck(lambda t: gpu_lib.poisson(t), (f,), eps=1e-6, atol=1e-9)


@pytest.mark.parametrize("dtype", REAL, ids=["f32", "f64"])
def test_config5_256cubed_gradient(gpu_lib, dtype):
    """256^3: f smooth (Gaussian sigma = 4 cells, zero mean), w ~ N(0,1); L = sum(phi * w)."""
    cfg = synth.CFG5
    shape = cfg["shape"]
    f = synth.smooth_field(shape, cfg["seed_f"], cfg["sigma"], np.float64)
    w = synth.real_normal(shape, cfg["seed_w"])
    fd = to_dev(f, dtype).requires_grad_(True)
    wd = to_dev(w, dtype)
    phi = gpu_lib.poisson(fd)
    loss = (phi.double() * wd.double()).sum()
    loss.backward()
    torch.cuda.synchronize()
    n = f.size
    f_in, w_in = promoted(f, dtype), promoted(w, dtype)
    assert_parity(to_host(phi), oracle.poisson(f_in), bound(dtype, n))
    grad = to_host(fd.grad)
    ref_grad = oracle.poisson_grad(w_in)  # FP64 reference gradient
    assert_parity(grad, ref_grad, bound(dtype, n))
    # directional finite difference, loss summed in FP64
    d = synth.real_normal(shape, 7)
    eps = np.linalg.norm(f) / np.linalg.norm(d)  # L is linear: any step is exact up to rounding
    with torch.no_grad():
        lp = (gpu_lib.poisson(to_dev(f + eps * d, dtype)).double() * wd.double()).sum().item()
        lm = (gpu_lib.poisson(to_dev(f - eps * d, dtype)).double() * wd.double()).sum().item()
    fd_dir = (lp - lm) / (2 * eps)
    an_dir = float(np.dot(grad.astype(np.float64).ravel(), d.ravel()))
    assert abs(fd_dir - an_dir) <= 1e-4 * abs(an_dir)
