"""Pins of the FP64 oracle against facts that do not come from the oracle itself.

Each test fixes the oracle to something the paper or mathematics determines:
hand-derived values (tests/golden), closed forms of special inputs, theorems
(Parseval, shift, convolution/adjointness), brute force on tiny grids, and
an independent library FFT (numpy.fft).  A dropped term, a wrong sign, a
swapped axis or a missing scale in the oracle fails at least one of them.
"""
import json
import os

import numpy as np
import pytest

import oracle
import synth

HERE = os.path.dirname(os.path.abspath(__file__))
SHAPES = [(1, 1, 1), (2, 3, 4), (5, 6, 4), (7, 3, 5), (4, 4, 4), (3, 8, 12), (9, 10, 6), (8, 16, 11)]


def _rand(shape, seed):
    return synth.complex_normal(shape, seed)


def test_golden_hand_derived():
    with open(os.path.join(HERE, "golden", "dft_small.json")) as fh:
        gold = json.load(fh)
    for case in gold["cases"]:
        shape = tuple(case["shape"])
        a = (np.array(case["input_re"]) + 1j * np.array(case["input_im"])).reshape(shape)
        want = (np.array(case["output_re"]) + 1j * np.array(case["output_im"])).reshape(shape)
        np.testing.assert_allclose(oracle.fftn(a), want, rtol=0, atol=1e-13, err_msg=case["note"])
        np.testing.assert_allclose(oracle.brute3d(a), want, rtol=0, atol=1e-13, err_msg=case["note"])


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 7, 8, 11, 12, 13, 16, 30, 48, 97, 100, 120, 128, 160, 512])
def test_dft1d_vs_numpy(n):
    x = _rand((n,), n)
    got = oracle.dft1d(x)
    want = np.fft.fft(x)
    assert oracle.rel_l2(got, want) < 1e-14
    # sign +1 is the conjugate-exponent sum: n * ifft
    assert oracle.rel_l2(oracle.dft1d(x, +1), n * np.fft.ifft(x)) < 1e-14


@pytest.mark.parametrize("shape", SHAPES)
def test_fftn_vs_brute_force(shape):
    a = _rand(shape, 11)
    fast = oracle.fftn(a)
    slow = oracle.brute3d(a)
    assert oracle.rel_l2(fast, slow) < 1e-13
    assert oracle.rel_l2(oracle.bfftn(a), oracle.brute3d(a, +1)) < 1e-13


def test_fftn_vs_brute_force_32cubed():
    """The 32^3 complex128 workload on its seeded input: recursive FFT vs the literal sum."""
    a = synth.complex_normal(synth.CFG1["shape"], synth.CFG1["seed"])
    assert oracle.rel_l2(oracle.fftn(a), oracle.brute3d(a)) < 1e-13


@pytest.mark.parametrize("shape", SHAPES + [(32, 24, 20), (17, 19, 23)])
def test_against_numpy_fft(shape):
    a = _rand(shape, 3)
    assert oracle.rel_l2(oracle.fftn(a), np.fft.fftn(a)) < 1e-14
    assert oracle.rel_l2(oracle.ifftn(a), np.fft.ifftn(a)) < 1e-14
    r = a.real.copy()
    assert oracle.rel_l2(oracle.rfftn(r), np.fft.rfftn(r)) < 1e-14
    h = np.fft.rfftn(r)
    nx = shape[2]
    assert oracle.rel_l2(oracle.irfftn(h, nx), np.fft.irfftn(h, s=shape, axes=(0, 1, 2))) < 1e-14


def test_irfftn_ignores_imag_of_dc_and_nyquist_like_numpy():
    """Non-Hermitian half spectra: both drop Im of the kx = 0 and kx = nx/2 bins after z, y."""
    shape = (6, 5, 8)
    h = synth.complex_normal((6, 5, 5), 9)
    want = np.fft.irfftn(h, s=shape, axes=(0, 1, 2))
    assert oracle.rel_l2(oracle.irfftn(h, 8), want) < 1e-14
    shape = (4, 3, 7)  # odd nx: only the kx = 0 bin is special
    h = synth.complex_normal((4, 3, 4), 10)
    assert oracle.rel_l2(oracle.irfftn(h, 7), np.fft.irfftn(h, s=shape, axes=(0, 1, 2))) < 1e-14


@pytest.mark.parametrize("shape", [(4, 6, 8), (5, 3, 10), (8, 8, 8)])
def test_delta_closed_forms(shape):
    nz, ny, nx = shape
    a = np.zeros(shape, complex)
    a[0, 0, 0] = 1
    np.testing.assert_allclose(oracle.fftn(a), np.ones(shape), atol=1e-15)
    # impulse at (x0, y0, z0) -> phase ramp exp(-2 pi i (kx x0/nx + ky y0/ny + kz z0/nz))
    x0, y0, z0 = nx - 1, 1 % ny, nz // 2
    a = np.zeros(shape, complex)
    a[z0, y0, x0] = 1
    kz, ky, kx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ramp = np.exp(-2j * np.pi * (kx * x0 / nx + ky * y0 / ny + kz * z0 / nz))
    np.testing.assert_allclose(oracle.fftn(a), ramp, atol=1e-14)
    np.testing.assert_allclose(oracle.brute3d(a), ramp, atol=1e-14)


@pytest.mark.parametrize("shape", [(4, 6, 8), (3, 5, 7)])
def test_constant_and_cosine_closed_forms(shape):
    nz, ny, nx = shape
    n = nx * ny * nz
    c = 0.75 - 0.5j
    want = np.zeros(shape, complex)
    want[0, 0, 0] = n * c
    np.testing.assert_allclose(oracle.fftn(np.full(shape, c)), want, atol=1e-12)
    # cos(2 pi p x / nx) -> n/2 at kx = p and kx = nx - p, zero elsewhere
    p = 2
    x = np.arange(nx)
    a = np.broadcast_to(np.cos(2 * np.pi * p * x / nx), shape).astype(complex)
    want = np.zeros(shape, complex)
    want[0, 0, p] = n / 2
    want[0, 0, nx - p] += n / 2
    np.testing.assert_allclose(oracle.fftn(a), want, atol=1e-12)
    # a sine along z -> -i n/2 at kz = 1 and +i n/2 at kz = nz - 1
    z = np.arange(nz)
    a = np.broadcast_to(np.sin(2 * np.pi * z / nz)[:, None, None], shape).astype(complex)
    want = np.zeros(shape, complex)
    want[1, 0, 0] = -0.5j * n
    want[nz - 1, 0, 0] = 0.5j * n
    np.testing.assert_allclose(oracle.fftn(a), want, atol=1e-12)


def test_parseval_linearity_roundtrip():
    shape = (12, 10, 9)
    a, b = _rand(shape, 1), _rand(shape, 2)
    n = a.size
    A, B = oracle.fftn(a), oracle.fftn(b)
    assert abs(np.vdot(A, A).real - n * np.vdot(a, a).real) < 1e-12 * n * np.vdot(a, a).real
    alpha, beta = 0.3 - 1.2j, -2.0 + 0.1j
    assert oracle.rel_l2(oracle.fftn(alpha * a + beta * b), alpha * A + beta * B) < 1e-14
    assert oracle.rel_l2(oracle.ifftn(A), a) < 1e-14
    assert oracle.rel_l2(oracle.bfftn(A), n * a) < 1e-14
    r = a.real.copy()
    assert oracle.rel_l2(oracle.irfftn(oracle.rfftn(r), 9), r) < 1e-14


def test_shift_theorem():
    shape = (6, 10, 8)
    nz, ny, nx = shape
    a = _rand(shape, 4)
    sz, sy, sx = 2, 3, 5
    shifted = np.roll(a, (sz, sy, sx), axis=(0, 1, 2))
    kz, ky, kx = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ramp = np.exp(-2j * np.pi * (kx * sx / nx + ky * sy / ny + kz * sz / nz))
    assert oracle.rel_l2(oracle.fftn(shifted), ramp * oracle.fftn(a)) < 1e-14


def test_adjoint_and_hermitian_symmetry():
    shape = (5, 6, 8)
    a, b = _rand(shape, 5), _rand(shape, 6)
    # <F a, b> = <a, F^H b> with F^H = bfftn
    lhs = np.vdot(b, oracle.fftn(a))
    rhs = np.vdot(oracle.bfftn(b), a)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    r = a.real.copy()
    X = oracle.fftn(r.astype(complex))
    flip = np.roll(X[::-1, ::-1, ::-1], 1, axis=(0, 1, 2))  # X[-k]
    assert oracle.rel_l2(flip, np.conj(X)) < 1e-14
    assert oracle.rel_l2(oracle.rfftn(r), X[:, :, : shape[2] // 2 + 1]) < 1e-15


def test_axis_order_invariance():
    """Separability (Sec. III-A): 1D DFTs along z, then x, then y give the same 3D result."""
    shape = (6, 5, 8)
    a = _rand(shape, 7)
    b = a.copy()
    for axis in (0, 2, 1):
        b = np.apply_along_axis(oracle.dft1d, axis, b)
    assert oracle.rel_l2(b, oracle.fftn(a)) < 1e-14


@pytest.mark.parametrize("real", [False, True])
def test_dft3d_points_vs_fftn(real):
    shape = (10, 12, 16)
    a = _rand(shape, 8)
    if real:
        a = a.real.copy()
    X = oracle.fftn(a.astype(complex))
    rng = np.random.default_rng(0)
    pts = np.stack([rng.integers(0, s, 40) for s in shape], axis=1)
    got = oracle.dft3d_points(a, pts)
    want = X[pts[:, 0], pts[:, 1], pts[:, 2]]
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-11)


def _wavenumbers(n):
    k = np.arange(n)
    return np.where(2 * k <= n, k, k - n)


def test_poisson_closed_form():
    """f = cos(k0 . x) on a 2 pi box solves to phi = -cos(k0 . x)/|k0|^2 exactly."""
    shape = (16, 12, 10)
    nz, ny, nx = shape
    z, y, x = np.meshgrid(*(2 * np.pi * np.arange(n) / n for n in shape), indexing="ij")
    for k0 in [(1, 2, 3), (0, 0, 1), (8, 6, 5), (3, 0, 5)]:  # (kz, ky, kx); includes Nyquist modes
        kz, ky, kx = k0
        f = np.cos(kx * x + ky * y + kz * z)
        phi = oracle.poisson(f)
        np.testing.assert_allclose(phi, -f / (kx * kx + ky * ky + kz * kz), atol=1e-13)
    # a constant has no zero-mean part: the k = 0 mode is dropped
    np.testing.assert_allclose(oracle.poisson(np.full(shape, 3.0)), 0, atol=1e-14)


def test_poisson_laplacian_and_mean():
    """The spectral Laplacian of phi gives back f minus its mean."""
    shape = (8, 10, 12)
    f = synth.real_normal(shape, 3)
    phi = oracle.poisson(f)
    assert abs(phi.mean()) < 1e-14
    # spectral Laplacian with numpy (independent library FFT)
    kz, ky, kx = np.meshgrid(*(_wavenumbers(n) for n in shape), indexing="ij")
    lap = np.fft.ifftn(-(kx ** 2 + ky ** 2 + kz ** 2) * np.fft.fftn(phi)).real
    np.testing.assert_allclose(lap, f - f.mean(), atol=1e-12)


def test_poisson_self_adjoint_and_gradient():
    """<P f, w> = <f, P w>, and L(f) = sum(P(f) w) has gradient P(w) (checked by differences)."""
    shape = (8, 6, 10)
    f, w, d = (synth.real_normal(shape, s) for s in (1, 2, 3))
    lhs = np.sum(oracle.poisson(f) * w)
    rhs = np.sum(f * oracle.poisson(w))
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)
    g = oracle.poisson_grad(w)
    eps = 1e-3
    fd = (np.sum(oracle.poisson(f + eps * d) * w) - np.sum(oracle.poisson(f - eps * d) * w)) / (2 * eps)
    assert abs(fd - np.sum(g * d)) < 1e-10 * abs(fd)


# ------------------------------------------------------------------ input recipes

def test_turbulence_field_recovers_projected_spectrum():
    """The FP64 R2C of the turbulence field is its half spectrum made Hermitian
    (the kx = 0 and kx = nx/2 planes averaged with their mirrored conjugates)
    and scaled by the normalisation: pins the recipe of the 1024^3 workload on
    a small grid."""
    shape = (12, 10, 16)
    nz, ny, nx = shape
    u = synth.turbulence_field(shape, 3, np.float64)
    assert abs(u.mean()) < 1e-12 and abs(u.std() - 1.0) < 1e-12
    S = synth.turbulence_spectrum(shape, 3, np.complex128)
    P = S.copy()
    for kx in (0, nx // 2):
        plane = S[:, :, kx]
        mirror = np.conj(plane[(-np.arange(nz)) % nz][:, (-np.arange(ny)) % ny])
        P[:, :, kx] = 0.5 * (plane + mirror)
    P[0, 0, 0] = 0.0
    H = oracle.rfftn(u)
    # u = (irfftn(S) - mean) / std and irfftn carries 1/N: H = P * N_scale
    scale = H.ravel()[np.argmax(np.abs(P.ravel()))] / P.ravel()[np.argmax(np.abs(P.ravel()))]
    assert abs(scale.imag) < 1e-12 * abs(scale) and scale.real > 0
    assert oracle.rel_l2(H, P * scale.real) < 1e-12
    # spectrum amplitudes follow |k|^(-11/6) off the projected planes
    k = np.sqrt(synth._wavenumbers(nz)[:, None, None] ** 2 + synth._wavenumbers(ny)[None, :, None] ** 2
                + np.arange(nx // 2 + 1)[None, None, :] ** 2)
    inner = np.abs(S[:, :, 1:nx // 2])
    assert np.allclose(inner, k[:, :, 1:nx // 2] ** (-11.0 / 6.0), rtol=1e-12)


# ------------------------------------------------------------------ sampled lines

@pytest.mark.parametrize("shape", [(4, 6, 8), (5, 3, 7), (8, 8, 9)])
def test_dft3d_lines_against_brute_force_and_numpy(shape):
    """Whole z-lines of the DFT at chosen (kx, ky) against the literal triple sum
    (complex input) and numpy.fft (real input)."""
    nz, ny, nx = shape
    a = _rand(shape, 71)
    kx = [0, nx - 1, 1, nx // 2, 0]
    ky = [0, 1, ny - 1, ny // 2, ny - 1]
    want = oracle.brute3d(a)[:, ky, kx]
    np.testing.assert_allclose(oracle.dft3d_lines(a, kx, ky), want, rtol=0, atol=1e-12)
    r = a.real.copy()
    np.testing.assert_allclose(oracle.dft3d_lines(r, kx, ky), np.fft.fftn(r)[:, ky, kx], rtol=0, atol=1e-12)
    np.testing.assert_allclose(oracle.dft3d_lines(a, kx, ky, +1), oracle.brute3d(a, +1)[:, ky, kx], atol=1e-12)


def test_dft3d_lines_cosine_closed_form():
    """cos(2 pi (p x/nx + q y/ny + s z/nz)) has N/2 at (p, q, s) and (-p, -q, -s), 0 elsewhere."""
    shape = (6, 10, 12)
    nz, ny, nx = shape
    n = nx * ny * nz
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    p, q, s = 3, 2, 1
    a = np.cos(2 * np.pi * (p * x / nx + q * y / ny + s * z / nz))
    lines = oracle.dft3d_lines(a, [p, nx - p, 0], [q, ny - q, q])
    want = np.zeros((nz, 3), complex)
    want[s, 0] = n / 2
    want[nz - s, 1] = n / 2
    np.testing.assert_allclose(lines, want, atol=1e-10)


# ------------------------------------------------------------------ real-to-real

@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 8, 12, 16, 30, 64])
def test_r2r1d_against_scipy(n):
    """DCT-II/III and DST-II/III (unnormalised) against scipy.fft (an independent library)."""
    import scipy.fft as sfft

    x = synth.real_normal((n,), 80 + n)
    np.testing.assert_allclose(oracle.r2r1d(x, 0), sfft.dct(x, type=2), rtol=0, atol=1e-12 * n)
    np.testing.assert_allclose(oracle.r2r1d(x, 1), sfft.dct(x, type=3), rtol=0, atol=1e-12 * n)
    np.testing.assert_allclose(oracle.r2r1d(x, 2), sfft.dst(x, type=2), rtol=0, atol=1e-12 * n)
    np.testing.assert_allclose(oracle.r2r1d(x, 3), sfft.dst(x, type=3), rtol=0, atol=1e-12 * n)


@pytest.mark.parametrize("n", [4, 7, 16])
def test_r2r1d_closed_forms_and_inverses(n):
    j = np.arange(n)
    for p in range(n):
        # a sampled Neumann mode maps to one spike (2n for the constant, n otherwise)
        spike = np.zeros(n)
        spike[p] = 2 * n if p == 0 else n
        np.testing.assert_allclose(oracle.r2r1d(np.cos(np.pi * p * (j + 0.5) / n), 0), spike, atol=1e-12)
        # a sampled Dirichlet mode sin((p+1) z) maps to one spike n (2n for the
        # alternating top mode sin(n z), as the constant for the DCT)
        spike = np.zeros(n)
        spike[p] = 2 * n if p == n - 1 else n
        np.testing.assert_allclose(oracle.r2r1d(np.sin(np.pi * (p + 1) * (j + 0.5) / n), 2), spike, atol=1e-12)
    x = synth.real_normal((n,), 5)
    np.testing.assert_allclose(oracle.r2r1d(oracle.r2r1d(x, 0), 1), 2 * n * x, atol=1e-12)
    np.testing.assert_allclose(oracle.r2r1d(oracle.r2r1d(x, 2), 3), 2 * n * x, atol=1e-12)
    # the type-III sums are the transposes of the type-II sums, up to the single
    # weight-1 term (first input of DCT-III, last of DST-III): <A x, y> = <x, B(e y)>
    y = synth.real_normal((n,), 6)
    e = np.ones(n)
    e[0] = 2.0
    assert abs(np.dot(oracle.r2r1d(x, 0), y) - np.dot(x, oracle.r2r1d(y * e, 1))) < 1e-11 * n
    e = np.ones(n)
    e[-1] = 2.0
    assert abs(np.dot(oracle.r2r1d(x, 2), y) - np.dot(x, oracle.r2r1d(y * e, 3))) < 1e-11 * n


@pytest.mark.parametrize("shape", [(4, 6, 8), (6, 5, 10), (3, 4, 6)])
@pytest.mark.parametrize("bc", [0, 1], ids=["neumann", "dirichlet"])
def test_ppb_transforms_against_library_composition(shape, bc):
    """(P, P, B) forward = numpy rfft along x, fft along y, scipy DCT-II / DST-II along z;
    the inverse undoes it."""
    import scipy.fft as sfft

    nz, ny, nx = shape
    f = synth.real_normal(shape, 90 + bc)
    h = np.fft.fft(np.fft.rfft(f, axis=2), axis=1)
    r2r = sfft.dct if bc == 0 else sfft.dst
    want = r2r(h.real, type=2, axis=0) + 1j * r2r(h.imag, type=2, axis=0)
    got = oracle.ppb_forward(f, bc)
    assert oracle.rel_l2(got, want) < 1e-14
    np.testing.assert_allclose(oracle.ppb_inverse(got, nx, bc), f, atol=1e-13)


@pytest.mark.parametrize("bc", [0, 1], ids=["neumann", "dirichlet"])
def test_poisson_ppb_closed_form(bc):
    """cos(a x + b y) cos(c z) (Neumann) or cos(a x + b y) sin(c z) (Dirichlet), with
    x, y on 2 pi-periodic grids and z at the cell centres of (0, pi): phi = -f / (a^2+b^2+c^2)."""
    shape = (12, 10, 16)
    nz, ny, nx = shape
    zc = np.pi * (np.arange(nz) + 0.5) / nz
    z, y, x = np.meshgrid(zc, 2 * np.pi * np.arange(ny) / ny, 2 * np.pi * np.arange(nx) / nx, indexing="ij")
    for a, b, c in ((1, 0, 0), (3, 2, 1), (0, 4, 5), (2, 1, 3)):
        if bc == 1 and c == 0:
            continue
        f = np.cos(a * x + b * y) * (np.cos(c * z) if bc == 0 else np.sin(c * z))
        np.testing.assert_allclose(oracle.poisson_ppb(f, bc), -f / (a * a + b * b + c * c), atol=1e-13)
    if bc == 0:  # the constant (zero wavenumber) is dropped
        np.testing.assert_allclose(oracle.poisson_ppb(np.full(shape, 2.0), 0), 0, atol=1e-14)


@pytest.mark.parametrize("bc", [0, 1], ids=["neumann", "dirichlet"])
def test_poisson_ppb_self_adjoint_and_laplacian(bc):
    """<P f, w> = <f, P w> (so the gradient of sum(P(f) w) is P(w)); and the spectral
    Laplacian of phi, taken with library transforms, gives back f (minus its mean for Neumann)."""
    import scipy.fft as sfft

    shape = (8, 6, 10)
    nz, ny, nx = shape
    f, w = synth.real_normal(shape, 11), synth.real_normal(shape, 12)
    lhs = np.sum(oracle.poisson_ppb(f, bc) * w)
    rhs = np.sum(f * oracle.poisson_ppb(w, bc))
    assert abs(lhs - rhs) < 1e-13 * abs(lhs)
    phi = oracle.poisson_ppb(f, bc)
    r2r = sfft.dct if bc == 0 else sfft.dst
    kz = np.arange(nz) + (0 if bc == 0 else 1)
    k2 = (kz[:, None, None] ** 2 + _wavenumbers(ny)[None, :, None] ** 2
          + _wavenumbers(nx)[None, None, :] ** 2)
    spec = np.fft.fft2(r2r(phi, type=2, axis=0), axes=(1, 2))
    lap_spec = -k2 * spec
    lap = np.fft.ifft2(lap_spec, axes=(1, 2))
    lap = r2r(lap.real, type=3, axis=0) / (2 * nz)
    want = f - f.mean() if bc == 0 else f
    np.testing.assert_allclose(lap, want, atol=1e-12)
