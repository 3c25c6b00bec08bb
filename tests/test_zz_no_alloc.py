"""GPU test of fft3d_forward_noalloc: the forward transform with the library's
static device scratch as its workspace, every tile enqueued in order on the
caller's stream, nothing allocated.

Its output must equal fft3d_forward's on the same plan and input, bitwise
(the same kernels run on the same tiles), on two calls in a row, the second
with a smaller input, so the second call runs on scratch the first one left
behind.  The smaller case is also checked against the FP64 oracle.
"""
import ctypes

import numpy as np
import pytest
import torch

import oracle
import synth
from _util import bound, check, promoted, to_dev, to_host

pytestmark = pytest.mark.gpu

ERR_WORKSPACE = -6


def _forward_both(plan, x, out_shape, out_dtype):
    ref = plan.forward(x)
    got = torch.full(out_shape, float("nan"), dtype=out_dtype, device="cuda")
    plan.forward_noalloc(x, got)
    torch.cuda.synchronize()
    return ref, got


@pytest.mark.parametrize("dtype", [torch.float32, torch.float64], ids=["f32", "f64"])
def test_noalloc_r2c_matches_forward_twice(gpu_lib, dtype):
    cplx = torch.complex64 if dtype == torch.float32 else torch.complex128
    # a workspace near the scratch size first (256^3 f32 R2C: 75.5 MB; f64
    # 144 MB), then a smaller, non-cubic one on the same scratch
    for shape, grid in (((256, 256, 256), (4, 4)), ((24, 40, 64), (2, 3))):
        print(f"case noalloc r2c shape={shape} grid={grid} dtype={dtype}", flush=True)
        f = synth.real_normal(shape, 700 + sum(shape))
        plan = gpu_lib.Plan(shape, dtype, grid, r2c=True)
        assert 0 < plan.workspace_bytes() <= 256 << 20
        x = to_dev(f, dtype)
        ref, got = _forward_both(plan, x, plan.half_shape, cplx)
        assert torch.equal(got, ref), f"{shape}: noalloc forward differs from fft3d_forward"
        if f.size <= 1 << 16:
            check(to_host(got), oracle.rfftn(promoted(f, dtype)), dtype, f.size, f"{shape} vs oracle")
        plan.close()


def test_noalloc_c2c_in_place_staging(gpu_lib):
    """C2C plans staged in place or in fused planes need no workspace at all."""
    for shape in ((64, 48, 40), (32, 32, 32)):
        print(f"case noalloc c2c shape={shape}", flush=True)
        a = synth.complex_normal(shape, 800 + sum(shape), np.complex64)
        plan = gpu_lib.Plan(shape, torch.complex64, (2, 2))
        assert plan.workspace_bytes() == 0
        x = to_dev(a, torch.complex64)
        ref, got = _forward_both(plan, x, shape, torch.complex64)
        assert torch.equal(got, ref)
        check(to_host(got), oracle.fftn(promoted(a, torch.complex64)), torch.complex64, a.size, "c2c vs oracle")
        plan.close()


def test_noalloc_rejects_workspace_beyond_scratch(gpu_lib):
    """A plan whose workspace exceeds the 256 MiB scratch gets FFT3D_ERR_WORKSPACE
    and its output is left untouched."""
    shape = (512, 512, 256)  # R2C f32: 129 (padded 144) x 512 x 512 x 8 B = 302 MB
    print(f"case noalloc too large shape={shape}", flush=True)
    plan = gpu_lib.Plan(shape, torch.float32, (1, 1), r2c=True)
    assert plan.workspace_bytes() > 256 << 20
    x = torch.zeros(shape, dtype=torch.float32, device="cuda")
    out = torch.full(plan.half_shape, 7.0, dtype=torch.complex64, device="cuda")
    L = gpu_lib._lib.lib()
    st = L.fft3d_forward_noalloc(plan.handle, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                 ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    torch.cuda.synchronize()
    assert st == ERR_WORKSPACE
    assert bool((out == 7.0).all())
    plan.close()
