"""GPU parity of the real-to-complex / complex-to-real pencil 3D FFT.

R2C keeps kx = 0..nx/2 of the forward DFT (Hermitian symmetry); C2R is its
inverse along z, y and then x, ignoring the imaginary parts of the kx = 0 and
kx = nx/2 bins.  Compared element by element with the FP64 oracle on the same
(precision-rounded) inputs.  The R2C adjoint is checked against its defining
identity Re<G, rfftn(f)> = <f, backward(G)> and against the oracle composition.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from _util import assert_parity, bound, promoted, rel, to_dev, to_host

pytestmark = pytest.mark.gpu

REAL = [torch.float32, torch.float64]
CPLX = {torch.float32: torch.complex64, torch.float64: torch.complex128}

CASES = [
    ((8, 8, 8), (1, 1)),
    ((32, 32, 32), (2, 2)),
    ((16, 12, 20), (2, 3)),
    ((5, 6, 4), (2, 2)),
    ((1, 1, 2), (1, 1)),
    ((3, 4, 2), (1, 1)),
    ((64, 48, 100), (3, 3)),
    ((40, 30, 96), (4, 4)),
    ((8, 16, 512), (1, 1)),
    ((4, 4, 1024), (1, 1)),
    ((2, 3, 2048), (1, 1)),
    # radix-7 lengths: 14 = 2*7, 42, 70, 840 = 8*3*5*7, half length 420
    ((14, 21, 28), (2, 2)),
    ((7, 35, 84), (1, 3)),
    ((4, 3, 840), (1, 1)),
    ((840, 2, 6), (1, 1)),
    # the generic odd-prime radix: half lengths 11, 13, 104
    ((13, 11, 22), (1, 1)),
    ((11, 26, 208), (2, 1)),
]


@pytest.mark.parametrize("dtype", REAL, ids=["f32", "f64"])
@pytest.mark.parametrize("shape,grid", CASES, ids=[f"{s}-{g}" for s, g in CASES])
def test_r2c_c2r(gpu_lib, shape, grid, dtype):
    print(f"case shape={shape} grid={grid} dtype={dtype}", flush=True)
    nz, ny, nx = shape
    f = synth.real_normal(shape, 200 + sum(shape))
    f_in = promoted(f, dtype)
    n = f.size
    plan = gpu_lib.Plan(shape, dtype, grid, r2c=True)
    x = to_dev(f, dtype)
    H = plan.forward(x)
    torch.cuda.synchronize()
    assert_parity(to_host(H), oracle.rfftn(f_in), bound(dtype, n))
    # inverse of a consistent half spectrum, and of an arbitrary one
    h_cons = oracle.rfftn(f_in)
    h_rand = synth.complex_normal((nz, ny, nx // 2 + 1), 300 + sum(shape))
    for h in (h_cons, h_rand):
        h_in = promoted(h, CPLX[dtype])
        hd = to_dev(h, CPLX[dtype])
        y = plan.inverse(hd)
        torch.cuda.synchronize()
        assert_parity(to_host(y), oracle.irfftn(h_in, nx), bound(dtype, n))
        assert torch.equal(hd, to_dev(h, CPLX[dtype]))  # input half spectrum left intact
    plan.close()


SWAP_CASES = [((8, 8, 8), (1, 1)), ((32, 32, 32), (2, 2)), ((16, 12, 20), (2, 3)), ((5, 6, 4), (2, 2)),
              ((64, 48, 100), (3, 3)), ((8, 16, 512), (1, 1)), ((7, 35, 84), (1, 3)), ((40, 30, 96), (4, 4))]


@pytest.mark.parametrize("dtype", REAL, ids=["f32", "f64"])
@pytest.mark.parametrize("shape,grid", SWAP_CASES, ids=[f"{s}-{g}" for s, g in SWAP_CASES])
def test_r2c_swap_yz_staging(gpu_lib, shape, grid, dtype):
    """Forward with the y/z-swapped workspace against the oracle, bitwise equal to
    in-place staging (the same line arithmetic at other addresses)."""
    print(f"case r2c swap_yz shape={shape} grid={grid} dtype={dtype}", flush=True)
    f = synth.real_normal(shape, 400 + sum(shape))
    x = to_dev(f, dtype)
    base = gpu_lib.Plan(shape, dtype, grid, streams=2, r2c=True, staging=gpu_lib.STAGING_IN_PLACE)
    plan = gpu_lib.Plan(shape, dtype, grid, streams=3, r2c=True, staging=gpu_lib.STAGING_SWAP_YZ)
    H0 = base.forward(x)
    H1 = plan.forward(x)
    torch.cuda.synchronize()
    assert_parity(to_host(H1), oracle.rfftn(promoted(f, dtype)), bound(dtype, f.size))
    assert torch.equal(H0, H1)
    # the inverse and the Poisson solve of a swapped plan stage as before
    y = plan.inverse(H1)
    torch.cuda.synchronize()
    assert_parity(to_host(y), promoted(f, dtype), bound(dtype, f.size))
    base.close()
    plan.close()


@pytest.mark.parametrize("dtype", REAL, ids=["f32", "f64"])
@pytest.mark.parametrize("shape,grid", [((8, 6, 10), (2, 2)), ((16, 32, 64), (1, 1)), ((15, 10, 12), (3, 2))])
def test_r2c_backward_is_adjoint(gpu_lib, shape, grid, dtype):
    nz, ny, nx = shape
    f = synth.real_normal(shape, 11)
    G = synth.complex_normal((nz, ny, nx // 2 + 1), 12)
    plan = gpu_lib.Plan(shape, dtype, grid, r2c=True)
    g = plan.backward(to_dev(G, CPLX[dtype]))
    torch.cuda.synchronize()
    g = to_host(g).astype(np.float64)
    G_in = promoted(G, CPLX[dtype])
    lhs = np.vdot(G_in, oracle.rfftn(f)).real  # Re <G, rfftn f>
    rhs = float(np.dot(f.ravel(), g.ravel()))
    tol = 1e-12 if dtype == torch.float64 else 1e-5
    assert abs(lhs - rhs) <= tol * (abs(lhs) + np.linalg.norm(f) * np.linalg.norm(g))
    # the same operator written with oracle pieces: unscaled c2r of G with interior bins halved
    Gh = G_in.copy()
    Gh[:, :, 1:(nx + 1) // 2] *= 0.5
    assert_parity(g, oracle.irfftn(Gh, nx, scale=False), bound(dtype, f.size))
    plan.close()


def test_r2c_errors(gpu_lib):
    from paper_2601_12209_amd._lib import Fft3dError

    with pytest.raises(Fft3dError):
        gpu_lib.Plan((4, 4, 5), torch.float32, r2c=True)  # odd nx
    plan = gpu_lib.Plan((4, 4, 8), torch.float32, r2c=True)
    buf = torch.zeros(4 * 4 * 5 * 2, dtype=torch.complex64, device="cuda")
    real_view = buf.view(torch.float32)[: 4 * 4 * 8].view(4, 4, 8)
    with pytest.raises(Fft3dError):  # out overlaps in
        plan.forward(real_view, out=buf[:80].view(4, 4, 5))
    plan.close()
