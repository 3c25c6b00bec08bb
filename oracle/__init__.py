"""FP64 CPU oracle for the pencil 3D FFT -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product library never calls it, and
this package imports nothing from the product.

Every routine evaluates the 3D DFT of the paper's Sec. III-A definition (sign
-1 forward, unscaled) in double precision, either as the literal sum
(``brute3d``, ``dft3d_points``) or as 1D DFTs along x, y, z (the tensor-product
structure stated in the same section); see ``oracle.c`` for the readings of
inverse scaling, R2C/C2R and the Poisson multiplier.  All arrays use the torch
/ numpy shape ``(nz, ny, nx)`` with x fastest.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile ``oracle.c`` with gcc (OpenMP, -O2) into ``liboracle.so``."""
    stale = (not os.path.exists(_LIB_PATH)
             or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC))
    if force or stale:
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-Wall", "-fPIC", "-shared",
                               "-fopenmp", _SRC, "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB_PATH)
        L, I, P = ctypes.c_long, ctypes.c_int, ctypes.c_void_p
        lib.oracle_dft1d.argtypes = [L, P, P, I]
        lib.oracle_c2c3d.argtypes = [L, L, L, P, P, I, I]
        lib.oracle_brute3d.argtypes = [L, L, L, P, P, I]
        lib.oracle_dft3d_points.argtypes = [L, L, L, P, I, L, P, P, I]
        lib.oracle_r2c3d.argtypes = [L, L, L, P, P]
        lib.oracle_c2r3d.argtypes = [L, L, L, P, P, I]
        lib.oracle_poisson3d.argtypes = [L, L, L, P, P]
        lib.oracle_num_threads.argtypes = []
        lib.oracle_r2r1d.argtypes = [L, P, P, I]
        lib.oracle_ppb_forward3d.argtypes = [L, L, L, P, P, I]
        lib.oracle_ppb_inverse3d.argtypes = [L, L, L, P, P, I]
        lib.oracle_poisson_ppb3d.argtypes = [L, L, L, P, P, I]
        for f in ("oracle_dft1d", "oracle_c2c3d", "oracle_brute3d", "oracle_dft3d_points",
                  "oracle_r2c3d", "oracle_c2r3d", "oracle_poisson3d", "oracle_num_threads",
                  "oracle_r2r1d", "oracle_ppb_forward3d", "oracle_ppb_inverse3d", "oracle_poisson_ppb3d"):
            getattr(lib, f).restype = ctypes.c_int
        _lib = lib
    return _lib


def _check(rc: int, name: str) -> None:
    if rc != 0:
        raise RuntimeError(f"oracle {name} failed with code {rc}")


def _c128(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.complex128)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def num_threads() -> int:
    """OpenMP threads the oracle uses (set OMP_NUM_THREADS to change)."""
    return int(_load().oracle_num_threads())


def dft1d(x, sign: int = -1) -> np.ndarray:
    """1D DFT of a complex vector by recursive mixed-radix decimation in time."""
    x = _c128(x).ravel()
    out = np.empty_like(x)
    _check(_load().oracle_dft1d(x.size, _ptr(x), _ptr(out), int(sign)), "dft1d")
    return out


def fftn(a) -> np.ndarray:
    """Forward 3D DFT (sign -1, unscaled) of a complex (nz, ny, nx) array."""
    a = _c128(a)
    nz, ny, nx = a.shape
    out = np.empty_like(a)
    _check(_load().oracle_c2c3d(nx, ny, nz, _ptr(a), _ptr(out), -1, 0), "c2c3d")
    return out


def ifftn(a) -> np.ndarray:
    """Inverse 3D DFT (sign +1, scaled by 1/N), stages z, y, x."""
    a = _c128(a)
    nz, ny, nx = a.shape
    out = np.empty_like(a)
    _check(_load().oracle_c2c3d(nx, ny, nz, _ptr(a), _ptr(out), +1, 1), "c2c3d")
    return out


def bfftn(a) -> np.ndarray:
    """Unscaled sign +1 3D DFT: the adjoint of ``fftn``."""
    a = _c128(a)
    nz, ny, nx = a.shape
    out = np.empty_like(a)
    _check(_load().oracle_c2c3d(nx, ny, nz, _ptr(a), _ptr(out), +1, 0), "c2c3d")
    return out


def brute3d(a, sign: int = -1) -> np.ndarray:
    """The literal O(N^2) triple sum of the 3D DFT definition (tiny grids only)."""
    a = _c128(a)
    nz, ny, nx = a.shape
    out = np.empty_like(a)
    _check(_load().oracle_brute3d(nx, ny, nz, _ptr(a), _ptr(out), int(sign)), "brute3d")
    return out


def dft3d_points(a, points, sign: int = -1) -> np.ndarray:
    """Selected outputs X[kz, ky, kx] of the 3D DFT, each by its own O(N) sum.

    ``a`` is real (float64) or complex, shape (nz, ny, nx); ``points`` is an
    (n, 3) integer array of (kz, ky, kx) indices.
    """
    real = not np.iscomplexobj(a)
    a = _f64(a) if real else _c128(a)
    nz, ny, nx = a.shape
    pts = np.asarray(points, dtype=np.int64).reshape(-1, 3)
    kxyz = np.ascontiguousarray(pts[:, ::-1], dtype=np.int64)  # (kx, ky, kz) per row
    out = np.empty(pts.shape[0], dtype=np.complex128)
    _check(_load().oracle_dft3d_points(nx, ny, nz, _ptr(a), int(real), pts.shape[0],
                                       _ptr(kxyz), _ptr(out), int(sign)), "dft3d_points")
    return out


def rfftn(a) -> np.ndarray:
    """kx = 0..nx//2 of the forward 3D DFT of a real (nz, ny, nx) array."""
    a = _f64(a)
    nz, ny, nx = a.shape
    out = np.empty((nz, ny, nx // 2 + 1), dtype=np.complex128)
    _check(_load().oracle_r2c3d(nx, ny, nz, _ptr(a), _ptr(out)), "r2c3d")
    return out


def irfftn(h, nx: int, scale: bool = True) -> np.ndarray:
    """Real (nz, ny, nx) field from its half spectrum (nz, ny, nx//2+1).

    ``scale`` True gives the inverse of ``rfftn`` (1/N); False is unscaled.
    """
    h = _c128(h)
    nz, ny, nh = h.shape
    if nh != nx // 2 + 1:
        raise ValueError("half-spectrum width must be nx//2+1")
    out = np.empty((nz, ny, nx), dtype=np.float64)
    _check(_load().oracle_c2r3d(nx, ny, nz, _ptr(h), _ptr(out), int(bool(scale))), "c2r3d")
    return out


def poisson(f) -> np.ndarray:
    """Spectral periodic Poisson solve phi = irfftn(M * rfftn(f)), M = -1/|k|^2, M(0) = 0."""
    f = _f64(f)
    nz, ny, nx = f.shape
    out = np.empty_like(f)
    _check(_load().oracle_poisson3d(nx, ny, nz, _ptr(f), _ptr(out)), "poisson3d")
    return out


def poisson_grad(w) -> np.ndarray:
    """Gradient of L(f) = sum(poisson(f) * w) with respect to f.

    The solve is a real circular convolution with an even kernel (M is real and
    M(k) = M(-k)), so its adjoint is itself and the gradient is poisson(w).  The
    CPU tests pin this identity numerically (adjointness and finite differences).
    """
    return poisson(w)


def dft3d_lines(a, kx, ky, sign: int = -1) -> np.ndarray:
    """Whole z-lines of the 3D DFT: out[:, i] = X[0..nz-1, ky[i], kx[i]].

    The definition's triple sum factored per axis, X[kz, ky, kx] =
    sum_z w_z^(kz z) sum_y w_y^(ky y) sum_x w_x^(kx x) a[z, y, x]: first the
    x sums for the distinct kx (a matrix product with those root columns), then
    the y sums, then the z sums for every kz (the length-nz DFT matrix).  Each
    root is exp(sign 2 pi i m / n) with the exponent m = k j reduced mod n
    before it is evaluated.  ``a`` is real or complex (nz, ny, nx); kx, ky are
    equal-length integer sequences.  Costs O(N * #distinct kx), so whole lines
    of a 1024^3 field take seconds.
    """
    a = np.asarray(a)
    nz, ny, nx = a.shape
    kx = np.asarray(kx, dtype=np.int64).ravel()
    ky = np.asarray(ky, dtype=np.int64).ravel()
    if kx.shape != ky.shape or np.any(kx < 0) or np.any(kx >= nx) or np.any(ky < 0) or np.any(ky >= ny):
        raise ValueError("kx, ky must be equal-length index sequences within the grid")

    def roots(k, n):  # (n, len(k)) matrix exp(sign 2 pi i (k j mod n) / n)
        m = (np.arange(n, dtype=np.int64)[:, None] * k[None, :]) % n
        return np.exp(sign * 2j * np.pi * m / n)

    ux, inv_x = np.unique(kx, return_inverse=True)
    flat = a.reshape(nz * ny, nx)
    wx = roots(ux, nx)
    if np.iscomplexobj(flat):
        sx = flat.astype(np.complex128, copy=False) @ wx
    else:  # real field: two real products keep the temporaries real
        f64 = flat.astype(np.float64, copy=False)
        sx = f64 @ np.ascontiguousarray(wx.real) + 1j * (f64 @ np.ascontiguousarray(wx.imag))
    sx = sx.reshape(nz, ny, len(ux))
    wy = roots(ky, ny)                                  # (ny, npairs)
    sxy = np.empty((nz, kx.size), dtype=np.complex128)
    for i in range(len(ux)):                            # the y sums of the pairs with this kx
        sel = np.nonzero(inv_x == i)[0]
        sxy[:, sel] = sx[:, :, i] @ wy[:, sel]
    wz = roots(np.arange(nz, dtype=np.int64), nz)       # (nz, nz), symmetric
    return wz @ sxy


def r2r1d(x, kind: int) -> np.ndarray:
    """Real-to-real transform of one real line, unnormalised (FFTW's REDFT/RODFT kinds):
    0 DCT-II, 1 DCT-III, 2 DST-II, 3 DST-III; kinds 1 and 3 undo 0 and 2 up to 2n."""
    x = _f64(x).ravel()
    out = np.empty_like(x)
    _check(_load().oracle_r2r1d(x.size, _ptr(x), _ptr(out), int(kind)), "r2r1d")
    return out


BC_NEUMANN, BC_DIRICHLET = 0, 1


def ppb_forward(f, bc: int = BC_NEUMANN) -> np.ndarray:
    """(Periodic, Periodic, Bounded) forward transform of a real (nz, ny, nx) field:
    DFT along x (kx = 0..nx//2) and y, then DCT-II (Neumann) or DST-II (Dirichlet)
    along z, unscaled; shape (nz, ny, nx//2 + 1)."""
    f = _f64(f)
    nz, ny, nx = f.shape
    out = np.empty((nz, ny, nx // 2 + 1), dtype=np.complex128)
    _check(_load().oracle_ppb_forward3d(nx, ny, nz, _ptr(f), _ptr(out), int(bc)), "ppb_forward3d")
    return out


def ppb_inverse(h, nx: int, bc: int = BC_NEUMANN) -> np.ndarray:
    """Inverse of :func:`ppb_forward` (DCT-III / DST-III over 2 nz, inverse DFT along y, C2R along x)."""
    h = _c128(h)
    nz, ny, nh = h.shape
    if nh != nx // 2 + 1:
        raise ValueError("half-spectrum width must be nx//2+1")
    out = np.empty((nz, ny, nx), dtype=np.float64)
    _check(_load().oracle_ppb_inverse3d(nx, ny, nz, _ptr(h), _ptr(out), int(bc)), "ppb_inverse3d")
    return out


def poisson_ppb(f, bc: int = BC_NEUMANN) -> np.ndarray:
    """Spectral Poisson solve with x, y periodic (side 2 pi) and z bounded (0, pi), cell-centred:
    phi = ppb_inverse(M * ppb_forward(f)), M = -1/|k|^2 (0 for the zero wavenumber); z
    wavenumbers k (Neumann, cos modes) or k + 1 (Dirichlet, sin modes)."""
    f = _f64(f)
    nz, ny, nx = f.shape
    out = np.empty_like(f)
    _check(_load().oracle_poisson_ppb3d(nx, ny, nz, _ptr(f), _ptr(out), int(bc)), "poisson_ppb3d")
    return out


def rel_l2(y, ref) -> float:
    """||y - ref||_2 / ||ref||_2 over all entries, accumulated in float64."""
    y = np.asarray(y)
    ref = np.asarray(ref)
    yd = y.astype(np.complex128) if np.iscomplexobj(y) else y.astype(np.float64)
    rd = ref.astype(np.complex128) if np.iscomplexobj(ref) else ref.astype(np.float64)
    num = np.linalg.norm((yd - rd).ravel())
    den = np.linalg.norm(rd.ravel())
    return float(num / den) if den > 0 else float(num)
