"""GPU parity of the (Periodic, Periodic, Bounded) transforms: DFT along x
(half spectrum) and y, DCT-II (Neumann walls) or DST-II (Dirichlet walls)
along the bounded z axis, their inverse and adjoint, and the spectral Poisson
solve of that topology (the paper's second Poisson-solver case, Sec. VI-B).

Every result is compared element by element with the FP64 oracle (the plain
O(n^2) DCT/DST sums along z, pinned on the CPU against closed forms, scipy and
their inverses).  The adjoint has no oracle function of its own: it is checked
against its defining identity <forward(f), G> = <f, backward(G)> (the real
inner product of the stored values, sum Re(conj(G) H) on the half spectrum:
the one a reverse-mode gradient of a real loss needs) and, at a tiny size,
against the explicit transpose of the forward built column by column from the
oracle.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from _util import assert_parity, bound, promoted, to_dev, to_host

pytestmark = pytest.mark.gpu

REAL = [torch.float32, torch.float64]
CPLX = {torch.float32: torch.complex64, torch.float64: torch.complex128}
BCS = [("neumann", oracle.BC_NEUMANN), ("dirichlet", oracle.BC_DIRICHLET)]

CASES = [
    ((8, 8, 8), (1, 1)),
    ((16, 12, 20), (2, 3)),
    ((7, 6, 4), (1, 1)),      # odd nz
    ((15, 10, 16), (2, 2)),   # odd nz, several tiles
    ((1, 4, 8), (1, 1)),      # one cell between the walls
    ((64, 48, 100), (3, 3)),  # radix-3/5 lengths, ragged tiles
    ((96, 40, 30), (4, 2)),
    ((21, 14, 28), (1, 2)),   # radix 7
    ((512, 4, 6), (1, 1)),    # long bounded axis
    ((13, 22, 26), (1, 1)),   # the generic odd-prime radix (11, 13)
]


@pytest.mark.parametrize("dtype", REAL, ids=["f32", "f64"])
@pytest.mark.parametrize("bc,obc", BCS, ids=[b for b, _ in BCS])
@pytest.mark.parametrize("shape,grid", CASES, ids=[f"{s}-{g}" for s, g in CASES])
def test_ppb_forward_inverse(gpu_lib, shape, grid, bc, obc, dtype):
    print(f"case ppb shape={shape} grid={grid} bc={bc} dtype={dtype}", flush=True)
    nz, ny, nx = shape
    n = nz * ny * nx
    f = synth.real_normal(shape, 900 + sum(shape))
    f_in = promoted(f, dtype)
    plan = gpu_lib.Plan(shape, dtype, grid, z_bc=bc)
    H = plan.forward(to_dev(f, dtype))
    torch.cuda.synchronize()
    ref_h = oracle.ppb_forward(f_in, obc)
    assert_parity(to_host(H), ref_h, bound(dtype, n), "forward")
    # the inverse of an arbitrary half spectrum (the imaginary parts of the
    # kx = 0 and nx/2 bins are dropped on both sides) and the round trip
    h = synth.complex_normal((nz, ny, nx // 2 + 1), 950 + sum(shape))
    h_in = promoted(h, CPLX[dtype])
    y = plan.inverse(to_dev(h, CPLX[dtype]))
    back = plan.inverse(H)
    torch.cuda.synchronize()
    assert_parity(to_host(y), oracle.ppb_inverse(h_in, nx, obc), bound(dtype, n), "inverse")
    assert_parity(to_host(back), f_in, bound(dtype, n), "round trip")
    plan.close()


@pytest.mark.parametrize("dtype", REAL, ids=["f32", "f64"])
@pytest.mark.parametrize("bc,obc", BCS, ids=[b for b, _ in BCS])
@pytest.mark.parametrize("shape,grid", [((16, 12, 20), (2, 3)), ((7, 6, 4), (1, 1)), ((40, 24, 32), (2, 2))])
def test_ppb_backward_is_adjoint(gpu_lib, shape, grid, bc, obc, dtype):
    """backward(G) = F^T G for the real-linear forward map F (real field -> half
    spectrum): sum Re(conj(G) F f) = sum f backward(G)."""
    print(f"case ppb adjoint shape={shape} grid={grid} bc={bc} dtype={dtype}", flush=True)
    nz, ny, nx = shape
    f = synth.real_normal(shape, 960)
    G = synth.complex_normal((nz, ny, nx // 2 + 1), 961)
    plan = gpu_lib.Plan(shape, dtype, grid, z_bc=bc)
    Ff = to_host(plan.forward(to_dev(f, dtype))).astype(np.complex128)
    BG = to_host(plan.backward(to_dev(G, CPLX[dtype]))).astype(np.float64)
    torch.cuda.synchronize()
    lhs = float(np.sum(G.real * Ff.real + G.imag * Ff.imag))
    rhs = float(np.sum(f * BG))
    tol = 1e-12 if dtype == torch.float64 else 1e-5 * np.log2(f.size)
    scale = np.linalg.norm(G.ravel()) * np.linalg.norm(Ff.ravel()) + np.linalg.norm(f.ravel()) * np.linalg.norm(BG.ravel())
    assert abs(lhs - rhs) <= tol * scale, (lhs, rhs)
    # against the oracle: the same identity with the oracle's forward in FP64
    ref_Ff = oracle.ppb_forward(promoted(f, dtype), obc)
    lhs_ref = float(np.sum(G.real * ref_Ff.real + G.imag * ref_Ff.imag))
    assert abs(lhs_ref - rhs) <= tol * scale, (lhs_ref, rhs)
    plan.close()


@pytest.mark.parametrize("bc,obc", BCS, ids=[b for b, _ in BCS])
def test_ppb_backward_explicit_transpose(gpu_lib, bc, obc):
    """At 3 x 2 x 4 (x, y, z = 4, 2, 3) the forward is a 24-column real matrix:
    built from the oracle one unit vector at a time, its transpose applied to G
    must equal backward(G) in FP64."""
    shape = (3, 2, 4)
    nz, ny, nx = shape
    nh = nx // 2 + 1
    cols = []
    for i in range(nz * ny * nx):
        e = np.zeros(nz * ny * nx)
        e[i] = 1.0
        h = oracle.ppb_forward(e.reshape(shape), obc).ravel()
        cols.append(np.concatenate([h.real, h.imag]))
    A = np.stack(cols, axis=1)  # (2 * nz*ny*nh, nz*ny*nx)
    G = synth.complex_normal((nz, ny, nh), 962)
    want = (A.T @ np.concatenate([G.real.ravel(), G.imag.ravel()])).reshape(shape)
    plan = gpu_lib.Plan(shape, torch.float64, (1, 1), z_bc=bc)
    got = to_host(plan.backward(to_dev(G, torch.complex128)))
    torch.cuda.synchronize()
    assert_parity(got, want, 1e-12, "explicit transpose")
    plan.close()


@pytest.mark.parametrize("dtype", REAL, ids=["f32", "f64"])
@pytest.mark.parametrize("bc,obc", BCS, ids=[b for b, _ in BCS])
@pytest.mark.parametrize("shape,grid", [((8, 8, 8), (1, 1)), ((16, 12, 20), (2, 3)), ((15, 10, 16), (2, 2)),
                                        ((64, 48, 100), (3, 3)), ((128, 128, 128), (1, 1))])
def test_ppb_poisson_and_gradient(gpu_lib, shape, grid, bc, obc, dtype):
    """The solve against the oracle, and its backward (the gradient of
    sum(phi * w)) against the oracle solve of w: the solve is self-adjoint,
    which the oracle pins on the CPU."""
    print(f"case ppb poisson shape={shape} grid={grid} bc={bc} dtype={dtype}", flush=True)
    n = int(np.prod(shape))
    f = synth.real_normal(shape, 970)
    w = synth.real_normal(shape, 971)
    plan = gpu_lib.Plan(shape, dtype, grid, z_bc=bc)
    phi = plan.poisson(to_dev(f, dtype))
    gf = plan.poisson_backward(to_dev(w, dtype))
    torch.cuda.synchronize()
    assert_parity(to_host(phi), oracle.poisson_ppb(promoted(f, dtype), obc), bound(dtype, n), "solve")
    assert_parity(to_host(gf), oracle.poisson_ppb(promoted(w, dtype), obc), bound(dtype, n), "gradient")
    plan.close()


@pytest.mark.parametrize("bc", ["neumann", "dirichlet"])
def test_ppb_poisson_closed_form(gpu_lib, bc):
    """A single mode is an eigenfunction of the bounded Laplacian: for
    f = cos(a x + b y) cos(c z) (Neumann) or sin(c z) (Dirichlet) on cell centres
    z = pi (j + 1/2) / nz, the solve returns -f / (a^2 + b^2 + c^2)."""
    shape = (16, 12, 10)
    nz, ny, nx = shape
    zc = np.pi * (np.arange(nz) + 0.5) / nz
    z, y, x = np.meshgrid(zc, 2 * np.pi * np.arange(ny) / ny, 2 * np.pi * np.arange(nx) / nx, indexing="ij")
    a, b, c = 3, 2, 5
    f = np.cos(a * x + b * y) * (np.cos(c * z) if bc == "neumann" else np.sin(c * z))
    plan = gpu_lib.Plan(shape, torch.float64, (2, 2), z_bc=bc)
    phi = to_host(plan.poisson(to_dev(f, torch.float64)))
    np.testing.assert_allclose(phi, -f / (a * a + b * b + c * c), atol=1e-13)
    plan.close()


def test_ppb_errors(gpu_lib):
    from paper_2601_12209_amd._lib import Fft3dError

    with pytest.raises((Fft3dError, KeyError)):
        gpu_lib.Plan((8, 8, 8), torch.float32, z_bc="periodic")
    with pytest.raises(Fft3dError):
        gpu_lib.Plan((8, 8, 9), torch.float32, z_bc="neumann")  # odd nx
    plan = gpu_lib.Plan((8, 8, 8), torch.float32, z_bc="dirichlet")
    with pytest.raises(Fft3dError):
        plan.set_staging(gpu_lib.STAGING_SWAP_YZ)
    plan.close()
