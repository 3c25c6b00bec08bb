"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This module holds no FFT arithmetic of the method: it only draws random
numbers and shapes them.  Two recipes need a smoothing or spectral-shaping
step; they use library routines (``scipy.ndimage`` and ``scipy.fft``), never
the oracle or the GPU library, so neither side of a parity test produces the
other's input.

Arrays use the shape ``(nz, ny, nx)`` with x fastest in memory.  All draws come
from ``numpy.random.default_rng(seed)`` (PCG64) in float64 and are cast to the
requested precision afterwards, so the complex64 and complex128 variants of a
workload share their underlying values.
"""
from __future__ import annotations

import numpy as np

# The five workloads (sizes and seeds), plus the 512^3 headline transform.
HEADLINE = dict(name="c2c_512cubed", shape=(512, 512, 512), grid=(4, 4), seed=0)
CFG1 = dict(name="c2c_32cubed_c128", shape=(32, 32, 32), grid=(2, 2), seed=1)
CFG2 = dict(name="c2c_256cubed", shape=(256, 256, 256), grid=(4, 4), seed=2)
CFG3 = dict(name="r2c_1024cubed_turbulence", shape=(1024, 1024, 1024), grid=(8, 8), seed=3)
CFG4 = dict(name="batched_uneven_64", count=64, seed=4,
            sizes=((48, 48, 48), (64, 64, 64), (96, 96, 96), (128, 120, 100), (80, 160, 160)))
CFG5 = dict(name="poisson_256cubed", shape=(256, 256, 256), seed_f=5, seed_w=6, sigma=4.0)


def complex_normal(shape, seed: int, dtype=np.complex128) -> np.ndarray:
    """Real and imaginary parts i.i.d. N(0, 1)."""
    rng = np.random.default_rng(seed)
    re = rng.standard_normal(shape)
    im = rng.standard_normal(shape)
    out = np.empty(shape, dtype=dtype)
    out.real = re
    out.imag = im
    return out


def real_normal(shape, seed: int, dtype=np.float64) -> np.ndarray:
    """Entries i.i.d. N(0, 1)."""
    return np.random.default_rng(seed).standard_normal(shape).astype(dtype)


def smooth_field(shape, seed: int, sigma: float = 4.0, dtype=np.float32) -> np.ndarray:
    """N(0,1) noise smoothed by a periodic Gaussian of ``sigma`` cells, mean removed.

    The Gaussian is applied in real space with wrap-around boundaries
    (``scipy.ndimage.gaussian_filter``, kernel truncated at 4 sigma), which is
    the periodic Gaussian filter up to the truncated tail.
    """
    from scipy.ndimage import gaussian_filter

    f = np.random.default_rng(seed).standard_normal(shape)
    f = gaussian_filter(f, sigma=sigma, mode="wrap", truncate=4.0)
    f -= f.mean()
    return f.astype(dtype)


def _wavenumbers(n: int) -> np.ndarray:
    k = np.arange(n, dtype=np.float64)
    return np.where(2 * k <= n, k, k - n)


def turbulence_spectrum(shape, seed: int, cdtype=np.complex64) -> np.ndarray:
    """Half spectrum (nz, ny, nx//2+1) of random-phase modes: amplitude
    |k|^(-11/6) for k != 0 (energy ~ k^(-5/3)), 0 at k = 0, phases uniform on
    [0, 2*pi) from the seed, one (ny, nx//2+1) plane of draws per kz."""
    nz, ny, nx = shape
    rdt = np.float32 if cdtype == np.complex64 else np.float64
    rng = np.random.default_rng(seed)
    kx = _wavenumbers(nx)[: nx // 2 + 1].astype(rdt)
    ky = _wavenumbers(ny).astype(rdt)
    kz = _wavenumbers(nz).astype(rdt)
    spec = np.empty((nz, ny, nx // 2 + 1), dtype=cdtype)
    for z in range(nz):  # plane by plane keeps the temporaries small
        k2 = kz[z] ** 2 + ky[:, None] ** 2 + kx[None, :] ** 2
        with np.errstate(divide="ignore"):
            amp = np.where(k2 > 0, k2 ** rdt(-11.0 / 12.0), rdt(0.0))
        ph = rng.uniform(0.0, 2.0 * np.pi, size=(ny, nx // 2 + 1)).astype(rdt)
        spec[z] = amp * (np.cos(ph) + 1j * np.sin(ph))
    return spec


def turbulence_field(shape, seed: int, dtype=np.float32, workers: int | None = None) -> np.ndarray:
    """Real field of the turbulence spectrum, normalised to zero mean and unit
    variance.  A library inverse real FFT (``scipy.fft.irfftn``) turns the half
    spectrum into the field; for float32 output the spectrum is built in
    complex64 to bound host memory at 1024^3, for float64 in complex128."""
    import os

    import scipy.fft

    nz, ny, nx = shape
    spec = turbulence_spectrum(shape, seed, np.complex64 if dtype == np.float32 else np.complex128)
    if workers is None:
        workers = max(1, min(16, len(os.sched_getaffinity(0))))
    u = scipy.fft.irfftn(spec, s=(nz, ny, nx), axes=(0, 1, 2), workers=workers)
    del spec
    u = u.astype(np.float64)
    u -= u.mean()
    u /= u.std()
    return u.astype(dtype)


def batch_sizes(seed: int = CFG4["seed"], count: int = CFG4["count"]):
    """The (nz, ny, nx) shapes of the batched workload: uniform draws with replacement."""
    sizes = CFG4["sizes"]
    idx = np.random.default_rng(seed).choice(len(sizes), size=count)
    return [tuple(sizes[i]) for i in idx]


def batch_inputs(shapes, seed: int, dtype=np.complex64):
    """One N(0,1) complex field per shape, from consecutive draws of one generator."""
    rng = np.random.default_rng(seed + 1000)
    out = []
    for s in shapes:
        a = np.empty(s, dtype=dtype)
        a.real = rng.standard_normal(s)
        a.imag = rng.standard_normal(s)
        out.append(a)
    return out
