"""Helpers shared by the GPU tests: tolerances, parity checks and tensor <-> numpy moves.

Parity is checked two ways on every compared array:

* rel-L2 = ||y - ref||_2 / ||ref||_2 over all entries (the whole-field bound),
* max_k |y_k - ref_k| / rms(ref) (the per-element bound): one wrong output of
  typical magnitude moves rel-L2 by only 1/sqrt(N), but moves this by ~1.

Both must stay within the same tolerance: 1e-12 for FP64 and 1e-5 * log2(N)
for FP32 (N = total points of the 3D transform).  For rounding errors the
per-element figure is a few times rel-L2 (the largest of N roughly Gaussian
errors is ~sqrt(2 ln N) times their RMS), so the bound holds with a wide margin.
"""
import math
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

import numpy as np
import torch

import oracle


def fp32_bound(n_total: int) -> float:
    """Tolerance for complex64/float32 results: 1e-5 * log2(N), N = total points."""
    return 1e-5 * max(1.0, math.log2(max(2, n_total)))


FP64_BOUND = 1e-12


def bound(dtype, n_total: int) -> float:
    return FP64_BOUND if dtype in (torch.complex128, torch.float64) else fp32_bound(n_total)


def to_dev(a: np.ndarray, dtype) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype)


def to_host(t: torch.Tensor) -> np.ndarray:
    return t.detach().cpu().numpy()


def promoted(a: np.ndarray, dtype) -> np.ndarray:
    """The input as the GPU sees it (rounded to the plan precision), in float64/complex128."""
    if dtype in (torch.complex64, torch.complex128):
        return a.astype(np.complex64 if dtype == torch.complex64 else np.complex128).astype(np.complex128)
    return a.astype(np.float32 if dtype == torch.float32 else np.float64).astype(np.float64)


def rel(y, ref) -> float:
    return oracle.rel_l2(y, ref)


def max_err_over_rms(y, ref) -> float:
    """max_k |y_k - ref_k| / sqrt(mean_k |ref_k|^2), in float64 (absolute if ref is all zero)."""
    y = np.asarray(y)
    ref = np.asarray(ref)
    cplx = np.iscomplexobj(y) or np.iscomplexobj(ref)
    wide = np.complex128 if cplx else np.float64
    yd = y.astype(wide, copy=False).ravel()
    rd = ref.astype(wide, copy=False).ravel()
    if yd.shape != rd.shape:
        raise ValueError(f"shape mismatch {y.shape} vs {ref.shape}")
    err = 0.0
    ss = 0.0
    step = 1 << 24  # chunks keep the temporaries small for 512^3 fields
    for i in range(0, yd.size, step):
        d = np.abs(yd[i:i + step] - rd[i:i + step])
        if d.size:
            m = float(d.max())
            if not math.isfinite(m):
                return float("inf")
            err = max(err, m)
        r = rd[i:i + step]
        ss += float(np.vdot(r, r).real) if cplx else float(np.dot(r, r))
    rms = math.sqrt(ss / max(1, yd.size))
    return err / rms if rms > 0 else err


def assert_parity(y, ref, tol: float, what: str = "") -> None:
    """rel-L2 and the per-element error (relative to rms(ref)) both within tol."""
    if isinstance(y, torch.Tensor):
        y = to_host(y)
    e2 = rel(y, ref)
    emax = max_err_over_rms(y, ref)
    assert e2 <= tol and emax <= tol, (f"{what}: rel-L2 {e2:.3e}, max|err|/rms(ref) {emax:.3e}, "
                                       f"bound {tol:.1e}")


def check(y, ref, dtype, n_total: int, what: str = "") -> None:
    """assert_parity with the precision's bound for an N-point transform."""
    assert_parity(y, ref, bound(dtype, n_total), what)
