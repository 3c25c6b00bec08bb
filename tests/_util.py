"""Helpers shared by the GPU tests: tolerances and tensor <-> numpy moves."""
import math
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))

import numpy as np
import torch

import oracle


def fp32_bound(n_total: int) -> float:
    """rel-L2 bound for complex64 results: 1e-5 * log2(N), N = total points."""
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
