"""Python binding of the fft3d C ABI over torch tensors.

PyTorch supplies device memory and the current HIP stream; every step of the
transform runs in the library's own kernels.  Shapes are torch order
``(nz, ny, nx)`` with x fastest in memory (the C ABI's x + Nx*(y + Ny*z)).

Plans are cached per (shape, dtype, pencil grid, r2c, device), as the paper's
plan cache is keyed by data type, size and transform type (Sec. V-B).
"""
from __future__ import annotations

import ctypes
import threading

import numpy as np
import torch

from . import _lib
from ._lib import check

C64, C128 = 0, 1
_COMPLEX = {C64: torch.complex64, C128: torch.complex128}
_REAL = {C64: torch.float32, C128: torch.float64}


def load():
    """Load the HIP library (raises if it is not built)."""
    return _lib.lib()


def _dtype_code(dtype) -> int:
    if dtype in (torch.complex64, torch.float32, "c64", "complex64", "f32", C64):
        return C64
    if dtype in (torch.complex128, torch.float64, "c128", "complex128", "f64", C128):
        return C128
    raise ValueError(f"unsupported dtype {dtype!r}")


def _stream_handle(stream=None) -> int:
    s = torch.cuda.current_stream() if stream is None else stream
    return int(s.cuda_stream)


STAGING_IN_PLACE = 0
STAGING_SWAP_YZ = 1
STAGING_FUSED_XY = 2
ISSUE_TILES = 0
ISSUE_STAGES = 1


Z_NEUMANN = 1
Z_DIRICHLET = 2
_ZBC = {"neumann": Z_NEUMANN, "dirichlet": Z_DIRICHLET, Z_NEUMANN: Z_NEUMANN, Z_DIRICHLET: Z_DIRICHLET}


class Plan:
    """A 3D FFT plan: sizes, precision, pencil grid P1 x P2 and transform kind.

    ``z_bc`` ("neumann" or "dirichlet") makes a real-to-complex plan whose z
    axis is bounded (the (Periodic, Periodic, Bounded) topology): DCT-II or
    DST-II along z instead of the DFT."""

    def __init__(self, shape, dtype=torch.complex64, grid=(1, 1), r2c=False, streams=None, staging=None,
                 z_bc=None, issue=None):
        nz, ny, nx = (int(v) for v in shape)
        self.shape = (nz, ny, nx)
        self.code = _dtype_code(dtype)
        self.grid = (int(grid[0]), int(grid[1]))
        self.z_bc = None if z_bc is None else _ZBC[z_bc]
        self.r2c = bool(r2c) or self.z_bc is not None
        h = ctypes.c_void_p()
        if self.z_bc is None:
            check(_lib.lib().fft3d_plan(ctypes.byref(h), nx, ny, nz, self.code, self.grid[0],
                                        self.grid[1], int(self.r2c)), "fft3d_plan")
        else:
            check(_lib.lib().fft3d_plan_ppb(ctypes.byref(h), nx, ny, nz, self.code, self.grid[0],
                                            self.grid[1], self.z_bc), "fft3d_plan_ppb")
        self._h = h
        self.device = torch.cuda.current_device()
        self._ws = None
        if streams is not None:
            self.set_streams(streams)
        if staging is not None:
            self.set_staging(staging)
        if issue is not None:
            self.set_issue(issue)

    # ------------------------------------------------------------ helpers
    @property
    def handle(self):
        return self._h

    @property
    def complex_dtype(self):
        return _COMPLEX[self.code]

    @property
    def real_dtype(self):
        return _REAL[self.code]

    @property
    def half_shape(self):
        """Shape of the half-spectrum tensors this plan exchanges: (nz, ny, nx//2 + 1)."""
        nz, ny, nx = self.shape
        return (nz, ny, nx // 2 + 1)

    @property
    def staging(self) -> int:
        """The plan's current staging (STAGING_IN_PLACE, STAGING_SWAP_YZ or STAGING_FUSED_XY)."""
        return int(_lib.lib().fft3d_get_staging(self._h))

    def _check_tensor(self, t, dtype, shape, name):
        if not isinstance(t, torch.Tensor) or not t.is_cuda:
            raise ValueError(f"{name} must be a CUDA tensor")
        if t.dtype != dtype:
            raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
        if tuple(t.shape) != tuple(shape):
            raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
        if not t.is_contiguous():
            raise ValueError(f"{name} must be contiguous")

    def _call(self, fn, x, out, in_dtype, in_shape, out_dtype, out_shape, stream):
        self._check_tensor(x, in_dtype, in_shape, "input")
        if out is None:
            out = torch.empty(out_shape, dtype=out_dtype, device=x.device)
        self._check_tensor(out, out_dtype, out_shape, "out")
        check(fn(self._h, ctypes.c_void_p(x.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                 ctypes.c_void_p(_stream_handle(stream))), fn.__name__)
        return out

    # ------------------------------------------------------------ transforms
    def forward(self, x, out=None, stream=None):
        """Forward 3D FFT (sign -1, unscaled)."""
        L = _lib.lib()
        if self.r2c:
            return self._call(L.fft3d_forward, x, out, self.real_dtype, self.shape, self.complex_dtype,
                              self.half_shape, stream)
        return self._call(L.fft3d_forward, x, out, self.complex_dtype, self.shape, self.complex_dtype,
                          self.shape, stream)

    def forward_noalloc(self, x, out, stream=None):
        """:meth:`forward` with the library's static device scratch as the workspace,
        every tile enqueued in order on the stream and nothing allocated (``out``
        is required); for code under graph capture or loops that cannot allocate."""
        L = _lib.lib()
        if self.r2c:
            return self._call(L.fft3d_forward_noalloc, x, out, self.real_dtype, self.shape,
                              self.complex_dtype, self.half_shape, stream)
        return self._call(L.fft3d_forward_noalloc, x, out, self.complex_dtype, self.shape,
                          self.complex_dtype, self.shape, stream)

    def inverse(self, x, out=None, stream=None):
        """Inverse 3D FFT (sign +1, scaled by 1/N)."""
        L = _lib.lib()
        if self.r2c:
            return self._call(L.fft3d_inverse, x, out, self.complex_dtype, self.half_shape,
                              self.real_dtype, self.shape, stream)
        return self._call(L.fft3d_inverse, x, out, self.complex_dtype, self.shape, self.complex_dtype,
                          self.shape, stream)

    def backward(self, x, out=None, stream=None):
        """Adjoint of forward (C2C: unscaled sign +1 transform)."""
        L = _lib.lib()
        if self.r2c:
            return self._call(L.fft3d_backward, x, out, self.complex_dtype, self.half_shape,
                              self.real_dtype, self.shape, stream)
        return self._call(L.fft3d_backward, x, out, self.complex_dtype, self.shape,
                          self.complex_dtype, self.shape, stream)

    def poisson(self, f, out=None, stream=None):
        """phi = irfftn(M * rfftn(f)), M = -1/|k|^2, M(0) = 0 (R2C plans)."""
        return self._call(_lib.lib().fft3d_poisson, f, out, self.real_dtype, self.shape,
                          self.real_dtype, self.shape, stream)

    def poisson_backward(self, g, out=None, stream=None):
        """Backward (adjoint) of :meth:`poisson` applied to g."""
        return self._call(_lib.lib().fft3d_poisson_backward, g, out, self.real_dtype, self.shape,
                          self.real_dtype, self.shape, stream)

    # ------------------------------------------------------------ tuning
    def set_streams(self, n: int):
        check(_lib.lib().fft3d_set_streams(self._h, int(n)), "fft3d_set_streams")

    def set_issue(self, mode: int):
        """ISSUE_TILES (one launch per tile on the plan's streams, event edges per
        producer tile) or ISSUE_STAGES (one grouped launch per stage)."""
        check(_lib.lib().fft3d_set_issue(self._h, int(mode)), "fft3d_set_issue")

    @property
    def issue(self) -> int:
        return int(_lib.lib().fft3d_get_issue(self._h))

    def set_staging(self, staging: int):
        """STAGING_IN_PLACE (C2C: no workspace), STAGING_SWAP_YZ (y stage writes a
        y/z-swapped workspace that the z stage reads back; R2C: forward only) or
        STAGING_FUSED_XY (C2C small planes: x and y FFTs of whole planes in LDS,
        then z)."""
        check(_lib.lib().fft3d_set_staging(self._h, int(staging)), "fft3d_set_staging")
        if not self.r2c:  # a C2C switch replaces the workspace; R2C plans keep theirs
            self._ws = None

    def set_stage_config(self, axis: int, lw: int, tdiv: int = 1, split: int = 0, pad: int = 0):
        """Launch shape of the stage kernels along one axis (lw = 0: default)."""
        check(_lib.lib().fft3d_set_stage_config(self._h, int(axis), int(lw), int(tdiv), int(split),
                                                int(pad)), "fft3d_set_stage_config")

    def set_radix_order(self, axis: int, order: int):
        """Radix order of the complex line kernels along one axis: 0 the default, 1 the reverse
        pass order (changes rounding, not the result beyond it)."""
        check(_lib.lib().fft3d_set_radix_order(self._h, int(axis), int(order)), "fft3d_set_radix_order")

    def radix_order(self, axis: int) -> int:
        return int(_lib.lib().fft3d_get_radix_order(self._h, int(axis)))

    def set_timing(self, enable: bool = True):
        """Record a HIP event after every stage of each call (stages then run one after another)."""
        check(_lib.lib().fft3d_set_timing(self._h, int(bool(enable))), "fft3d_set_timing")

    def stage_times(self):
        """Milliseconds of each stage of the most recent timed call (waits for it)."""
        buf = (ctypes.c_float * 8)()
        k = _lib.lib().fft3d_stage_times(self._h, buf, 8)
        if k < 0:
            raise RuntimeError("fft3d_stage_times: " + _lib.lib().fft3d_last_error().decode())
        return list(buf[:k])

    def workspace_bytes(self) -> int:
        return int(_lib.lib().fft3d_workspace_bytes(self._h))

    def set_workspace(self, buf):
        """Use a caller tensor as the workspace (None: back to a plan-owned one)."""
        ptr = None if buf is None else ctypes.c_void_p(buf.data_ptr())
        nbytes = 0 if buf is None else buf.numel() * buf.element_size()
        check(_lib.lib().fft3d_set_workspace(self._h, ptr, nbytes), "fft3d_set_workspace")
        self._ws = buf

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.lib().fft3d_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchPlan:
    """Many 3D FFTs of different shapes: each stage of every shape's transforms
    goes out as one grouped launch (tile tables cached per pointer set)."""

    def __init__(self, shapes, dtype=torch.complex64):
        self.shapes = [tuple(int(v) for v in s) for s in shapes]
        self.code = _dtype_code(dtype)
        dims = (ctypes.c_int64 * (3 * len(self.shapes)))()
        for i, (nz, ny, nx) in enumerate(self.shapes):
            dims[3 * i], dims[3 * i + 1], dims[3 * i + 2] = nx, ny, nz
        h = ctypes.c_void_p()
        check(_lib.lib().fft3d_plan_batch(ctypes.byref(h), len(self.shapes), dims, self.code),
              "fft3d_plan_batch")
        self._h = h

    def set_stage_config(self, shape, axis: int, lw: int, tdiv: int = 1, split: int = 0, pad: int = 0):
        nz, ny, nx = shape
        check(_lib.lib().fft3d_batch_set_stage_config(self._h, nx, ny, nz, int(axis), int(lw), int(tdiv),
                                                      int(split), int(pad)), "fft3d_batch_set_stage_config")

    def set_staging(self, shape, staging: int):
        """STAGING_IN_PLACE or STAGING_FUSED_XY for the transforms of one (nz, ny, nx) shape."""
        nz, ny, nx = shape
        check(_lib.lib().fft3d_batch_set_staging(self._h, nx, ny, nz, int(staging)), "fft3d_batch_set_staging")

    def set_radix_order(self, shape, axis: int, order: int):
        nz, ny, nx = shape
        check(_lib.lib().fft3d_batch_set_radix_order(self._h, nx, ny, nz, int(axis), int(order)),
              "fft3d_batch_set_radix_order")

    def set_streams(self, n: int):
        """Streams the batch's shapes run on concurrently (1: all on the caller's stream)."""
        check(_lib.lib().fft3d_batch_set_streams(self._h, int(n)), "fft3d_batch_set_streams")

    def staging(self, shape) -> int:
        """The staging of the transforms of one (nz, ny, nx) shape."""
        nz, ny, nx = shape
        v = int(_lib.lib().fft3d_batch_get_staging(self._h, nx, ny, nz))
        if v < 0:
            raise _lib.Fft3dError(-1, "fft3d_batch_get_staging")
        return v

    def _run(self, fn, xs, outs, stream):
        dt = _COMPLEX[self.code]
        if len(xs) != len(self.shapes):
            raise ValueError("one input per transform")
        for x, s in zip(xs, self.shapes):
            if not (x.is_cuda and x.dtype == dt and tuple(x.shape) == s and x.is_contiguous()):
                raise ValueError(f"inputs must be contiguous {dt} CUDA tensors of shapes {self.shapes}")
        if outs is None:
            outs = [torch.empty_like(x) for x in xs]
        for o, s in zip(outs, self.shapes):
            if not (o.is_cuda and o.dtype == dt and tuple(o.shape) == s and o.is_contiguous()):
                raise ValueError("outputs must match the inputs")
        n = len(xs)
        ins = (ctypes.c_void_p * n)(*[x.data_ptr() for x in xs])
        ous = (ctypes.c_void_p * n)(*[o.data_ptr() for o in outs])
        check(fn(self._h, ins, ous, ctypes.c_void_p(_stream_handle(stream))), fn.__name__)
        return outs

    def forward(self, xs, outs=None, stream=None):
        return self._run(_lib.lib().fft3d_forward_batch, xs, outs, stream)

    def inverse(self, xs, outs=None, stream=None):
        return self._run(_lib.lib().fft3d_inverse_batch, xs, outs, stream)

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            _lib.lib().fft3d_batch_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def query_batch_placement(shapes, nstreams=4):
    """Transform indices per stream, in issue order (host-only)."""
    n = len(shapes)
    dims = (ctypes.c_int64 * (3 * n))()
    for i, (nz, ny, nx) in enumerate(shapes):
        dims[3 * i], dims[3 * i + 1], dims[3 * i + 2] = nx, ny, nz
    L = _lib.lib()
    need = L.fft3d_query_batch_placement(n, dims, nstreams, None, 0)
    if need < 0:
        raise ValueError("invalid batch")
    buf = (ctypes.c_int64 * need)()
    L.fft3d_query_batch_placement(n, dims, nstreams, buf, need)
    v = list(buf)
    out, pos = [], 1
    for _ in range(v[0]):
        k = v[pos]
        out.append(v[pos + 1:pos + 1 + k])
        pos += 1 + k
    return out


_cache: dict = {}
_cache_lock = threading.Lock()


def get_plan(shape, dtype, grid=(1, 1), r2c=False) -> Plan:
    """Plan cache keyed by (shape, precision, grid, r2c, device).  A cached plan
    may be shared by several threads and streams: the library serialises its
    calls on the host and orders a call on a new stream after the previous
    call on the device."""
    key = (tuple(int(v) for v in shape), _dtype_code(dtype), tuple(grid), bool(r2c),
           torch.cuda.current_device())
    with _cache_lock:
        p = _cache.get(key)
        if p is None:
            p = Plan(shape, dtype, grid, r2c)
            _cache[key] = p
        return p


def clear_plan_cache():
    with _cache_lock:
        for p in _cache.values():
            p.close()
        _cache.clear()


def fftn(x, grid=(1, 1), out=None):
    return get_plan(x.shape, x.dtype, grid).forward(x, out)


def ifftn(x, grid=(1, 1), out=None):
    return get_plan(x.shape, x.dtype, grid).inverse(x, out)


def bfftn(x, grid=(1, 1), out=None):
    return get_plan(x.shape, x.dtype, grid).backward(x, out)


def rfftn(x, grid=(1, 1), out=None):
    return get_plan(x.shape, x.dtype, grid, r2c=True).forward(x, out)


def irfftn(h, nx: int, grid=(1, 1), out=None):
    nz, ny, _ = h.shape
    return get_plan((nz, ny, nx), h.dtype, grid, r2c=True).inverse(h, out)


class SpectralPoisson(torch.autograd.Function):
    """phi = irfftn(rfftn(f) / (-|k|^2)), k = 0 mode zeroed, differentiable in f.

    The backward pass runs the library's fft3d_poisson_backward (each stage of
    the solve replaced by its adjoint, in reverse order).
    """

    @staticmethod
    def forward(ctx, f, grid=(1, 1)):
        plan = get_plan(f.shape, f.dtype, grid, r2c=True)
        ctx.plan = plan
        return plan.poisson(f.contiguous())

    @staticmethod
    def backward(ctx, gphi):
        return ctx.plan.poisson_backward(gphi.contiguous()), None


def poisson(f, grid=(1, 1)):
    return SpectralPoisson.apply(f, grid)


# ---------------------------------------------------------------- host queries
def length_supported(n: int) -> bool:
    return bool(_lib.lib().fft3d_length_supported(int(n)))


def query_radix_plan(n: int):
    buf = (ctypes.c_int * 16)()
    k = _lib.lib().fft3d_query_radix_plan(int(n), buf, 16)
    if k < 0:
        raise ValueError(f"length {n} is not supported")
    np_ = buf[0]
    return list(buf[1:1 + np_]), buf[np_ + 1]


def query_twiddles(n: int, dtype) -> np.ndarray:
    code = _dtype_code(dtype)
    out = np.empty(n, dtype=np.complex64 if code == C64 else np.complex128)
    check(_lib.lib().fft3d_query_twiddles(int(n), code, out.ctypes.data), "fft3d_query_twiddles")
    return out


LAUNCH_FIELDS = ("lw", "tdiv", "split", "pad", "strided", "align", "xcd", "nt")


def query_launches(shape, dtype, grid=(1, 1), r2c=False, op=0, staging=0):
    """Default launch configuration of every task (task order of a one-stream
    plan): dicts with the keys of LAUNCH_FIELDS.  dtype: the plan precision."""
    nz, ny, nx = shape
    L = _lib.lib()
    args = (nx, ny, nz, _dtype_code(dtype), grid[0], grid[1], int(r2c), int(staging), int(op))
    need = L.fft3d_query_launches(*args, None, 0)
    if need < 0:
        raise ValueError("invalid launch query arguments")
    buf = (ctypes.c_int64 * need)()
    L.fft3d_query_launches(*args, buf, need)
    v = list(buf)
    k = len(LAUNCH_FIELDS)
    return [dict(zip(LAUNCH_FIELDS, v[1 + i * k:1 + (i + 1) * k])) for i in range(v[0])]


def query_pipeline(shape, grid, r2c=False, op=0, nstreams=4, staging=0):
    """Decoded task graph: (stages, tasks) with boxes over the complex (x, y, z) index space."""
    nz, ny, nx = shape
    L = _lib.lib()
    need = L.fft3d_query_pipeline(nx, ny, nz, grid[0], grid[1], int(r2c), int(staging), op, nstreams, None, 0)
    if need < 0:
        raise ValueError("invalid pipeline arguments")
    buf = (ctypes.c_int64 * need)()
    L.fft3d_query_pipeline(nx, ny, nz, grid[0], grid[1], int(r2c), int(staging), op, nstreams, buf, need)
    v = list(buf)
    ntasks, nstages = v[0], v[1]
    pos = 2
    stages = []
    for _ in range(nstages):
        kind, axis, n, conj, weight, src, dst, sbits, lay_src, lay_dst = v[pos:pos + 10]
        scale = float(np.array([sbits], dtype=np.int64).view(np.float64)[0])
        stages.append(dict(kind=kind, axis=axis, n=n, conj=conj, weight=weight, src=src, dst=dst,
                           scale=scale, lay_src=lay_src, lay_dst=lay_dst))
        pos += 10
    tasks = []
    for _ in range(ntasks):
        stage = v[pos]
        box = tuple(v[pos + 1:pos + 7])  # x0, x1, y0, y1, z0, z1
        stream = v[pos + 7]
        nd = v[pos + 8]
        deps = v[pos + 9:pos + 9 + nd]
        pos += 9 + nd
        nw = v[pos]
        waits = v[pos + 1:pos + 1 + nw]
        pos += 1 + nw
        tasks.append(dict(stage=stage, box=box, stream=stream, deps=list(deps), waits=list(waits)))
    return stages, tasks
