"""Host-side checks of the library (no GPU): exported C ABI, radix plans,
twiddle tables, pencil tiles, the tile dependency graph, stream placement and
its event waits, and a CPU simulation of the task graph.

The simulator executes the library's own task graph (as returned by
fft3d_query_pipeline) tile by tile, in random orders that respect only the
stream order and the event waits the library would issue, applying the
oracle's 1D DFT to every line of each tile.  A missing dependency edge, a
wrong stage kind, sign, scale or bin weighting makes its result differ from
the oracle's 3D transform.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle
import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fft3d.h")


@pytest.fixture(scope="module")
def fft3d():
    from paper_2601_12209_amd import _lib, build

    if not os.path.exists(_lib.LIB_PATH):
        build.build(verbose=False)
    from paper_2601_12209_amd import fft3d as mod

    mod.load()
    return mod


def test_header_symbols_exported(fft3d):
    names = re.findall(r"^\s*[a-z_0-9 \*]+?\b(fft3d_[a-z_0-9]+)\s*\(", open(HEADER).read(), re.M)
    assert len(set(names)) >= 18
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2601_12209_amd", "libfft3d.so"))
    for n in set(names):
        assert hasattr(lib, n), f"{n} declared in fft3d.h but not exported"


SUPPORTED = [1, 2, 3, 4, 5, 6, 7, 8, 10, 12, 14, 15, 16, 20, 21, 24, 25, 28, 30, 32, 35, 40, 42, 48, 50,
             56, 60, 64, 70, 75, 80, 84, 96, 100, 105, 112, 120, 125, 128, 140, 150, 160, 168, 192, 200, 210,
             240, 250, 256, 280, 300, 320, 384, 400, 420, 480, 500, 512, 600, 640, 720, 750, 768, 800, 840,
             960, 1000, 1024, 2048, 4096, 11, 13, 22, 26, 44, 52, 88, 104, 176, 208]


def test_supported_lengths_and_radix_plans(fft3d):
    for n in range(1, 4100):
        assert fft3d.length_supported(n) == (n in SUPPORTED), n
    for n in SUPPORTED:
        radices, tpl = fft3d.query_radix_plan(n)
        assert int(np.prod(radices)) == n
        assert set(radices) <= {2, 3, 4, 5, 7, 8, 11, 13, 15, 16}
        if n % 15 == 0:  # a factor 3 and a factor 5 form one radix-15 pass unless a radix 16 sets the threads
            assert (15 in radices) != (16 in radices), (n, radices)
        assert tpl == (n // max(radices) if radices else 1)
    assert fft3d.query_radix_plan(840) == ([8, 15, 7], 56)


@pytest.mark.parametrize("n", [2, 3, 5, 7, 8, 12, 100, 120, 512, 840, 1000, 1024, 4096])
def test_twiddles(fft3d, n):
    w64 = fft3d.query_twiddles(n, "c128")
    m = np.arange(n, dtype=np.longdouble)
    pi = np.longdouble("3.14159265358979323846264338327950288")  # pi to long double precision
    ang = np.longdouble(-2) * pi * m / np.longdouble(n)
    ref = (np.cos(ang), np.sin(ang))
    ulp_re = np.spacing(np.abs(w64.real).astype(np.float64)) + np.finfo(np.float64).tiny
    ulp_im = np.spacing(np.abs(w64.imag).astype(np.float64)) + np.finfo(np.float64).tiny
    # within one ulp of the extended-precision value (x86 long double, ~1e-19 relative)
    assert np.all(np.abs(w64.real - ref[0]) <= ulp_re + 1e-18)
    assert np.all(np.abs(w64.imag - ref[1]) <= ulp_im + 1e-18)
    # exact special values
    assert w64[0] == 1
    if n % 2 == 0:
        assert w64[n // 2] == -1
    if n % 4 == 0:
        assert w64[n // 4] == -1j and w64[3 * n // 4] == 1j
    # the complex64 table is the round-to-nearest-even of the complex128 table
    w32 = fft3d.query_twiddles(n, "c64")
    assert np.array_equal(w32.real, w64.real.astype(np.float32))
    assert np.array_equal(w32.imag, w64.imag.astype(np.float32))


# ------------------------------------------------------------------ task graph

def _cover(shape_c, tasks, stage):
    nz, ny, nxc = shape_c
    count = np.zeros((nz, ny, nxc), dtype=np.int64)
    for t in tasks:
        if t["stage"] != stage:
            continue
        x0, x1, y0, y1, z0, z1 = t["box"]
        count[z0:z1, y0:y1, x0:x1] += 1
    return count


def _overlap(a, b):
    return all(a[2 * d] < b[2 * d + 1] and b[2 * d] < a[2 * d + 1] for d in range(3))


GRAPH_CASES = [((8, 8, 8), (1, 1), 0, 1), ((8, 8, 8), (2, 2), 0, 2), ((12, 10, 20), (3, 4), 0, 4),
               ((12, 10, 20), (3, 4), 1, 3), ((16, 8, 6), (4, 2), 2, 8), ((6, 10, 16), (2, 3), 3, 4),
               ((6, 10, 16), (5, 3), 4, 2), ((32, 32, 32), (8, 8), 0, 16), ((5, 6, 4), (3, 5), 1, 1)]


@pytest.mark.parametrize("shape,grid,op,ns", GRAPH_CASES)
def test_tiles_partition_and_dependencies(fft3d, shape, grid, op, ns):
    r2c = op >= 3
    stages, tasks = fft3d.query_pipeline(shape, grid, r2c=r2c, op=op, nstreams=ns)
    nz, ny, nx = shape
    nxc = nx // 2 + 1 if r2c else nx
    assert len(tasks) == len(stages) * grid[0] * grid[1]
    for s in range(len(stages)):
        assert np.all(_cover((nz, ny, nxc), tasks, s) == 1), "tiles of a stage partition the array"
    pos = {}
    for i, t in enumerate(tasks):
        # topological issue order; deps are exactly the overlapping tiles of the previous stage
        want = sorted(j for j, u in enumerate(tasks)
                      if u["stage"] == t["stage"] - 1 and _overlap(u["box"], t["box"]))
        assert sorted(t["deps"]) == want
        assert all(d < i for d in t["deps"])
        assert 0 <= t["stream"] < ns
        pos[i] = i
    # happens-before: stream order + event waits cover every dependency
    last_on = {}
    hb = []
    for i, t in enumerate(tasks):
        before = set()
        if t["stream"] in last_on:
            j = last_on[t["stream"]]
            before |= {j} | hb[j]
        for w in t["waits"]:
            assert tasks[w]["stream"] != t["stream"]
            before |= {w} | hb[w]
        hb.append(before)
        last_on[t["stream"]] = i
        assert set(t["deps"]) <= before, f"task {i} can start before a producer"


def test_immediate_dispatch_order(fft3d):
    """With a grid of z-slabs, each y tile is issued right after the x tiles of its slab."""
    _, tasks = fft3d.query_pipeline((16, 16, 16), (1, 4), op=0, nstreams=1)
    assert [t["stage"] for t in tasks] == [0, 1] * 4 + [2] * 4
    for k in range(4):
        assert tasks[2 * k + 1]["deps"] == [2 * k]


def test_placement_balances_streams(fft3d):
    _, tasks = fft3d.query_pipeline((32, 32, 32), (4, 4), op=0, nstreams=4)
    for s in range(3):
        per = [sum(1 for t in tasks if t["stage"] == s and t["stream"] == q) for q in range(4)]
        assert max(per) - min(per) <= 1


# ------------------------------------------------------------------ simulator

def _wavenumber(j, n):
    return np.where(2 * j <= n, j, j - n)


def _apply_stage(st, box, bufs, shape):
    nz, ny, nx = shape
    x0, x1, y0, y1, z0, z1 = box
    kind, axis, n, conj, weight, scale = (st[k] for k in ("kind", "axis", "n", "conj", "weight", "scale"))
    src, dst = bufs[st["src"]], bufs[st["dst"]]
    sign = 1 if conj else -1
    if kind == 0:  # C2C along axis
        sub = src[z0:z1, y0:y1, x0:x1]
        ax = {0: 2, 1: 1, 2: 0}[axis]
        res = np.apply_along_axis(lambda v: oracle.dft1d(v, sign), ax, sub) * scale
        dst[z0:z1, y0:y1, x0:x1] = res
    elif kind == 1:  # R2C along x: rows (y, z) of the real source
        h = nx // 2
        rows = src[z0:z1, y0:y1, :]
        res = np.apply_along_axis(lambda v: oracle.dft1d(v.astype(complex))[: h + 1], 2, rows)
        if weight:
            res[..., 1:h] *= 2
        dst[z0:z1, y0:y1, :] = res * scale
    elif kind == 2:  # C2R along x
        h = nx // 2
        rows = src[z0:z1, y0:y1, :].copy()
        rows[..., 0] = rows[..., 0].real
        rows[..., h] = rows[..., h].real
        if weight:
            rows[..., 1:h] *= 0.5

        def c2r(v):
            full = np.concatenate([v, np.conj(v[1:h][::-1])])
            return oracle.dft1d(full, +1).real

        dst[z0:z1, y0:y1, :] = np.apply_along_axis(c2r, 2, rows) * scale
    elif kind == 4:  # whole x-y planes: x FFTs, then y FFTs
        sub = src[z0:z1, y0:y1, x0:x1]
        res = np.apply_along_axis(lambda v: oracle.dft1d(v, sign), 2, sub)
        res = np.apply_along_axis(lambda v: oracle.dft1d(v, sign), 1, res) * scale
        dst[z0:z1, y0:y1, x0:x1] = res
    elif kind == 3:  # Poisson z stage
        sub = src[z0:z1, y0:y1, x0:x1]
        kz = _wavenumber(np.arange(nz), nz)[:, None, None]
        ky = _wavenumber(np.arange(y0, y1), ny)[None, :, None]
        kx = np.arange(x0, x1)[None, None, :]
        k2 = (kx * kx + ky * ky + kz * kz).astype(float)
        m = np.where(k2 == 0, 0.0, -1.0 / np.where(k2 == 0, 1, k2)) * scale
        f = np.apply_along_axis(lambda v: oracle.dft1d(v, -1), 0, sub)
        dst[z0:z1, y0:y1, x0:x1] = np.apply_along_axis(lambda v: oracle.dft1d(v, +1), 0, f * m)
    else:
        raise AssertionError(kind)


def _simulate(fft3d, shape, grid, op, ns, inp, rng, staging=0):
    r2c = op >= 3 or np.isrealobj(inp) or inp.shape[2] != shape[2]
    stages, tasks = fft3d.query_pipeline(shape, grid, r2c=r2c, op=op, nstreams=ns, staging=staging)
    nz, ny, nx = shape
    nxc = nx // 2 + 1
    if not r2c:
        out = np.full(shape, np.nan + 0j)
        ws = np.full(shape, np.nan + 0j) if staging else None
    else:
        out_real = op in (1, 2, 3, 4)
        out = np.full(shape, np.nan) if out_real else np.full((nz, ny, nxc), np.nan + 0j)
        ws = np.full((nz, ny, nxc), np.nan + 0j)
    bufs = [inp.copy(), out, ws]
    # a task may run once the previous task of its stream and every waited task have run
    done = [False] * len(tasks)
    per_stream = {}
    for i, t in enumerate(tasks):
        per_stream.setdefault(t["stream"], []).append(i)
    head = {s: 0 for s in per_stream}
    for _ in range(len(tasks)):
        runnable = []
        for s, lst in per_stream.items():
            if head[s] < len(lst):
                i = lst[head[s]]
                if all(done[w] for w in tasks[i]["waits"]):
                    runnable.append((s, i))
        assert runnable, "deadlock"
        s, i = runnable[rng.integers(len(runnable))]
        _apply_stage(stages[tasks[i]["stage"]], tasks[i]["box"], bufs, shape)
        done[i] = True
        head[s] += 1
    return bufs[1]


SIM_CASES = [((6, 4, 8), (2, 2), 2), ((5, 6, 10), (3, 2), 4), ((8, 6, 4), (1, 3), 1), ((4, 4, 6), (2, 1), 3)]


def _simulate_graph(fft3d, shape, grid, op, inp, rng, staging=0, r2c=False):
    """Run the tasks in a random order that respects only each task's producer
    list (the dependencies of the graph-replay nodes; no stream order)."""
    stages, tasks = fft3d.query_pipeline(shape, grid, r2c=r2c, op=op, nstreams=1, staging=staging)
    nz, ny, nx = shape
    nxc = nx // 2 + 1
    if not r2c:
        out = np.full(shape, np.nan + 0j)
        ws = np.full(shape, np.nan + 0j) if staging == 1 else None
    else:
        out = np.full(shape, np.nan) if op in (1, 2, 3, 4) else np.full((nz, ny, nxc), np.nan + 0j)
        ws = np.full((nz, ny, nxc), np.nan + 0j)
    bufs = [inp.copy(), out, ws]
    done = [False] * len(tasks)
    for _ in range(len(tasks)):
        ready = [i for i, t in enumerate(tasks) if not done[i] and all(done[d] for d in t["deps"])]
        assert ready, "deadlock"
        i = ready[rng.integers(len(ready))]
        _apply_stage(stages[tasks[i]["stage"]], tasks[i]["box"], bufs, shape)
        done[i] = True
    return bufs[1]


@pytest.mark.parametrize("shape,grid", [((6, 4, 8), (2, 2)), ((5, 6, 10), (3, 2)), ((8, 6, 4), (1, 3)),
                                        ((12, 8, 8), (1, 2))])
def test_producer_edges_alone_order_every_pipeline(fft3d, shape, grid):
    """The graph-replay nodes depend only on their producer tiles: every random
    order those edges allow gives the exact transform, for each staging and
    operation."""
    rng = np.random.default_rng(7)
    a = synth.complex_normal(shape, 3)
    stagings = [0, 1] + ([2] if grid[0] == 1 and shape[1] == shape[2] == 8 else [])
    for staging in stagings:
        for _ in range(3):
            for op, want in ((0, oracle.fftn(a)), (1, oracle.ifftn(a)), (2, oracle.bfftn(a))):
                got = _simulate_graph(fft3d, shape, grid, op, a, rng, staging)
                assert oracle.rel_l2(got, want) < 1e-14, (staging, op)
    f = synth.real_normal(shape, 4)
    for staging in (0, 1):
        got = _simulate_graph(fft3d, shape, grid, 0, f, rng, staging, r2c=True)
        assert oracle.rel_l2(got, oracle.rfftn(f)) < 1e-14
    phi = _simulate_graph(fft3d, shape, grid, 3, f, rng, 0, r2c=True)
    assert oracle.rel_l2(phi, oracle.poisson(f)) < 1e-13


@pytest.mark.parametrize("staging", [0, 1], ids=["in_place", "swap_yz"])
@pytest.mark.parametrize("shape,grid,ns", SIM_CASES)
def test_simulated_c2c(fft3d, shape, grid, ns, staging):
    rng = np.random.default_rng(0)
    a = synth.complex_normal(shape, 1)
    for trial in range(3):
        for op, want in ((0, oracle.fftn(a)), (1, oracle.ifftn(a)), (2, oracle.bfftn(a))):
            got = _simulate(fft3d, shape, grid, op, ns, a, rng, staging)
            assert oracle.rel_l2(got, want) < 1e-14, op


FUSED_CASES = [((6, 8, 8), (1, 2), 2), ((5, 16, 16), (1, 1), 1), ((12, 24, 24), (1, 3), 4)]


@pytest.mark.parametrize("shape,grid,ns", FUSED_CASES)
def test_simulated_fused_xy(fft3d, shape, grid, ns):
    rng = np.random.default_rng(5)
    a = synth.complex_normal(shape, 2)
    for op, want in ((0, oracle.fftn(a)), (1, oracle.ifftn(a)), (2, oracle.bfftn(a))):
        stages, _ = fft3d.query_pipeline(shape, grid, op=op, nstreams=ns, staging=2)
        assert [st["kind"] for st in stages] == ([4, 0] if op == 0 else [0, 4])
        got = _simulate(fft3d, shape, grid, op, ns, a, rng, 2)
        assert oracle.rel_l2(got, want) < 1e-14, op
    with pytest.raises(ValueError):  # planes need p1 == 1
        fft3d.query_pipeline(shape, (2, 1), staging=2)
    with pytest.raises(ValueError):  # no kernel for a 6 x 8 plane
        fft3d.query_pipeline((4, 8, 6), (1, 1), staging=2)


def test_swap_yz_staging_layouts(fft3d):
    """y writes the workspace with y/z swapped, z reads it back; x, y, z in every direction."""
    for op in (0, 1, 2):
        stages, _ = fft3d.query_pipeline((8, 6, 4), (2, 2), op=op, nstreams=2, staging=1)
        assert [st["axis"] for st in stages] == [0, 1, 2]
        assert [(st["src"], st["dst"]) for st in stages] == [(0, 1), (1, 2), (2, 1)]
        assert [(st["lay_src"], st["lay_dst"]) for st in stages] == [(0, 0), (0, 1), (1, 0)]
        assert [st["conj"] for st in stages] == [int(op != 0)] * 3
        assert stages[2]["scale"] == (1.0 / (8 * 6 * 4) if op == 1 else 1.0)
    # R2C: only the forward changes (x writes the output, y the swapped workspace)
    stages, _ = fft3d.query_pipeline((8, 6, 4), (2, 2), r2c=True, op=0, nstreams=2, staging=1)
    assert [st["kind"] for st in stages] == [1, 0, 0]
    assert [(st["src"], st["dst"]) for st in stages] == [(0, 1), (1, 2), (2, 1)]
    assert [(st["lay_src"], st["lay_dst"]) for st in stages] == [(0, 0), (0, 1), (1, 0)]
    for op in (1, 2, 3, 4):
        assert (fft3d.query_pipeline((8, 6, 4), (2, 2), r2c=True, op=op, nstreams=2, staging=1)[0]
                == fft3d.query_pipeline((8, 6, 4), (2, 2), r2c=True, op=op, nstreams=2, staging=0)[0])
    with pytest.raises(ValueError):  # fused planes are C2C only
        fft3d.query_pipeline((8, 8, 8), (1, 1), r2c=True, staging=2)


@pytest.mark.parametrize("shape,grid,ns", SIM_CASES)
def test_simulated_r2c_swap_yz(fft3d, shape, grid, ns):
    rng = np.random.default_rng(2)
    f = synth.real_normal(shape, 5)
    for _ in range(3):
        got = _simulate(fft3d, shape, grid, 0, ns, f, rng, staging=1)
        assert oracle.rel_l2(got, oracle.rfftn(f)) < 1e-14


@pytest.mark.parametrize("shape,grid,ns", SIM_CASES)
def test_simulated_r2c_family(fft3d, shape, grid, ns):
    rng = np.random.default_rng(1)
    nz, ny, nx = shape
    f = synth.real_normal(shape, 2)
    w = synth.real_normal(shape, 3)
    H = synth.complex_normal((nz, ny, nx // 2 + 1), 4)
    got = _simulate(fft3d, shape, grid, 0, ns, f, rng)
    assert oracle.rel_l2(got, oracle.rfftn(f)) < 1e-14
    got = _simulate(fft3d, shape, grid, 1, ns, H, rng)
    assert oracle.rel_l2(got, oracle.irfftn(H, nx)) < 1e-14
    # backward = adjoint of rfftn: Re<H, rfftn f> = <f, backward H>
    g = _simulate(fft3d, shape, grid, 2, ns, H, rng)
    lhs = np.vdot(H, oracle.rfftn(f)).real
    assert abs(lhs - np.dot(f.ravel(), g.ravel())) < 1e-12 * abs(lhs)
    phi = _simulate(fft3d, shape, grid, 3, ns, f, rng)
    assert oracle.rel_l2(phi, oracle.poisson(f)) < 1e-13
    gf = _simulate(fft3d, shape, grid, 4, ns, w, rng)
    assert oracle.rel_l2(gf, oracle.poisson_grad(w)) < 1e-13


def test_graph_simulator_catches_a_missing_edge(fft3d, monkeypatch):
    """Drop one producer edge: some order the remaining edges allow goes wrong, so
    the producer-edge simulation above can tell a sufficient edge set."""
    real_query = fft3d.query_pipeline

    def broken(*args, **kw):
        stages, tasks = real_query(*args, **kw)
        for t in tasks:
            if t["stage"] == 2 and t["deps"]:
                t["deps"] = t["deps"][1:]
                break
        return stages, tasks

    monkeypatch.setattr(fft3d, "query_pipeline", broken)
    shape, grid = (6, 4, 8), (2, 2)
    a = synth.complex_normal(shape, 1)
    rng = np.random.default_rng(3)
    errs = [oracle.rel_l2(_simulate_graph(fft3d, shape, grid, 0, a, rng), oracle.fftn(a)) for _ in range(12)]
    assert max(e if np.isfinite(e) else np.inf for e in errs) > 1e-3


def test_simulator_catches_a_missing_edge(fft3d, monkeypatch):
    """Drop one dependency from the library's graph: some random order then goes wrong."""
    real_query = fft3d.query_pipeline

    def broken(*args, **kw):
        stages, tasks = real_query(*args, **kw)
        for t in tasks:  # forget the waits of the first stage-1 task placed on stream 0
            if t["stage"] == 1 and t["stream"] == 0 and t["waits"]:
                t["waits"] = []
                break
        return stages, tasks

    monkeypatch.setattr(fft3d, "query_pipeline", broken)
    shape, grid = (6, 4, 8), (2, 2)
    a = synth.complex_normal(shape, 1)
    rng = np.random.default_rng(3)
    errs = [oracle.rel_l2(_simulate(fft3d, shape, grid, 0, 2, a, rng), oracle.fftn(a)) for _ in range(12)]
    assert max(e if np.isfinite(e) else np.inf for e in errs) > 1e-3


# ------------------------------------------------------------------ batch placement

def test_batch_placement_least_loaded(fft3d):
    shapes = synth.batch_sizes()
    per = fft3d.query_batch_placement(shapes, 4)
    assert len(per) == 4
    assert sorted(i for p in per for i in p) == list(range(len(shapes)))
    cost = [np.prod(s) * np.log2(np.prod(s)) for s in shapes]
    loads = [sum(cost[i] for i in p) for p in per]
    # greedy LPT: the spread is at most the largest single cost
    assert max(loads) - min(loads) <= max(cost) + 1e-6
    for p in per:  # within a stream, larger transforms first
        assert [cost[i] for i in p] == sorted((cost[i] for i in p), reverse=True)


# ------------------------------------------------------------------ launch configuration

def _by_stage(fft3d, shape, dtype, r2c=False, op=0, staging=0, grid=(1, 1)):
    stages, tasks = fft3d.query_pipeline(shape, grid, r2c=r2c, op=op, nstreams=1, staging=staging)
    launches = fft3d.query_launches(shape, dtype, grid, r2c=r2c, op=op, staging=staging)
    assert len(launches) == len(tasks)
    return [(stages[t["stage"]], L) for t, L in zip(tasks, launches)]


@pytest.mark.parametrize("shape,dtype,r2c,grid", [((256, 256, 256), "c64", False, (4, 4)),
                                                   ((256, 256, 256), "c128", False, (4, 4)),
                                                   ((1024, 1024, 1024), "f32", True, (8, 8)),
                                                   ((512, 512, 512), "f32", True, (4, 4)),
                                                   ((512, 512, 512), "c64", False, (3, 3)),
                                                   ((840, 840, 840), "c64", False, (2, 2))])
def test_tiles_of_a_stage_share_a_launch_shape(fft3d, shape, dtype, r2c, grid):
    """Every tile of a stage gets the same launch configuration (the stage then
    goes out as one grouped launch): the defaults are chosen per plan, not per
    tile, for the tiled workloads."""
    for op in (0, 1):
        by = {}
        for st, L in _by_stage(fft3d, shape, dtype, r2c=r2c, op=op, grid=grid):
            key = (st["axis"], st["kind"])
            by.setdefault(key, set()).add(tuple(sorted(L.items())))
        for key, confs in by.items():
            assert len(confs) == 1, (shape, dtype, op, key, confs)


def test_cache_policy_large_c2c(fft3d):
    """512^3 swapped staging: complex128 stages stream with non-temporal loads and
    stores (whole cache lines of another buffer) and XCD-grouped strided tiles;
    complex64 x stages the same, complex64 y/z stages plain accesses, plain order."""
    for dtype in ("c64", "c128"):
        for op in (0, 1):
            got = _by_stage(fft3d, (512, 512, 512), dtype, op=op, staging=1)
            assert [st["axis"] for st, _ in got] == [0, 1, 2]
            for st, L in got:
                assert L["strided"] == int(st["axis"] != 0)
                assert L["xcd"] == int(dtype == "c128" and st["axis"] != 0)
                assert L["align"] <= 1
                want = 0 if (dtype == "c64" and st["axis"] != 0) else 2
                assert L["nt"] == want, (dtype, op, st, L)
    # the complex64 strided stages take 32 lines, half the threads per line, full LDS tile
    _, L = _by_stage(fft3d, (512, 512, 512), "c64", staging=1)[1]
    assert (L["lw"], L["tdiv"], L["split"]) == (32, 2, 0)


def test_cache_policy_in_place_and_cache_resident(fft3d):
    # in place at 512^3 (complex128): non-temporal stores only (the line just read is rewritten)
    for st, L in _by_stage(fft3d, (512, 512, 512), "c128", staging=0)[1:]:
        assert st["src"] == st["dst"] and L["nt"] == 1
    # fields that fit the Infinity Cache keep plain accesses
    for dtype in ("c64", "c128"):
        for staging in (0, 1):
            assert all(L["nt"] == 0 for _, L in _by_stage(fft3d, (256, 256, 256), dtype, staging=staging))


def test_xcd_grouped_order_policy(fft3d):
    """XCD-grouped strided tiles: complex128 always; complex64 C2C only for tiles
    narrower than a cache line (8-line tiles of 720 and 840); R2C y stages from
    a 512 MiB half spectrum, and every R2C strided stage from 2 GiB."""
    def xcd(shape, dtype, r2c=False, op=0):
        return [(st["axis"], L["lw"], L["xcd"]) for st, L in _by_stage(fft3d, shape, dtype, r2c=r2c, op=op)
                if L["strided"]]
    for op in (0, 1):
        assert all(x == 1 for _, _, x in xcd((512, 512, 512), "c128", op=op))
        assert all(x == 0 for _, _, x in xcd((512, 512, 512), "c64", op=op))
        for n in (720, 840):
            got = xcd((n, n, n), "c64", op=op)
            assert got and all(lw == 8 and x == 1 for _, lw, x in got), (n, got)
        assert all(x == (axis == 1) for axis, _, x in xcd((512, 512, 512), "f32", r2c=True, op=op))
        assert all(x == 1 for _, _, x in xcd((1024, 1024, 1024), "f32", r2c=True, op=op))
        assert all(x == 0 for _, _, x in xcd((256, 256, 256), "f32", r2c=True, op=op))


def test_r2c_launches(fft3d):
    """512^3 R2C: padded LDS lines in the real x kernels; output rows of 257 values
    get shifted (cache-line aligned) tiles; non-temporal loads only where whole
    lines of another buffer are read."""
    for dtype in ("f32", "f64"):
        fwd = _by_stage(fft3d, (512, 512, 512), dtype, r2c=True, op=0, staging=1)
        (x, Lx), (y, Ly), (z, Lz) = fwd
        assert x["kind"] == 1 and Lx["pad"] == 1 and Lx["nt"] == 0 and Lx["strided"] == 0
        per_line = 16 if dtype == "f32" else 8
        assert Lz["align"] == per_line and Ly["align"] <= 1  # z writes the 257-value rows of the output
        # rows of 257 values are read misaligned: non-temporal stores only
        assert Ly["nt"] == 1 and Lz["nt"] == 1
        if dtype == "f32":  # 257 columns: 16-line tiles, full complex LDS tile
            assert (Ly["lw"], Ly["tdiv"], Ly["split"]) == (16, 1, 0)
        if dtype == "f64":
            assert Ly["xcd"] == 1 and Lz["xcd"] == 1
        inv = _by_stage(fft3d, (512, 512, 512), dtype, r2c=True, op=1)
        (z, Lz), (y, Ly), (x, Lx) = inv
        # the FP64 C2R x kernel streams its real rows with non-temporal stores
        assert x["kind"] == 2 and Lx["pad"] == 1 and Lx["nt"] == (dtype == "f64")
        assert y["src"] == y["dst"] == 2 and Ly["nt"] == 1  # in place in the workspace
        assert Lz["nt"] == 1
    # small R2C plans: plain accesses, padded real kernels
    for st, L in _by_stage(fft3d, (32, 32, 32), "f32", r2c=True, op=3):
        assert L["nt"] == 0
        if st["kind"] in (1, 2):
            assert L["pad"] == 1


def test_launch_query_rejects_bad_arguments(fft3d):
    with pytest.raises(ValueError):
        fft3d.query_launches((8, 8, 8), "c64", r2c=True, staging=2)
    with pytest.raises(ValueError):
        fft3d.query_launches((8, 8, 17), "c64")


def test_x_ranges_of_tiles_start_on_cache_lines(fft3d):
    """y and z tiles split x on whole cache lines (16 complex64 / 8 complex128
    values) when every tile keeps two lines, else balanced; a partition either way."""
    for nx, p1, dtype_granule in ((1024, 8, 16), (512, 4, 16), (200, 3, 16)):
        for op in (0, 1):
            stages, tasks = fft3d.query_pipeline((16, 16, nx), (p1, 1), r2c=True, op=op, nstreams=1)
            nxc = nx // 2 + 1
            for t in tasks:
                if stages[t["stage"]]["axis"] == 0:
                    continue
                x0, x1 = t["box"][0], t["box"][1]
                if nxc // p1 >= 2 * dtype_granule:
                    assert x0 % dtype_granule == 0, (nx, p1, t["box"])
                assert x1 > x0
    # 513 values over 8 tiles: edges 0, 64, ..., 448, 513
    stages, tasks = fft3d.query_pipeline((8, 8, 1024), (8, 1), r2c=True, op=0, nstreams=1)
    xs = sorted({(t["box"][0], t["box"][1]) for t in tasks if stages[t["stage"]]["axis"] == 1})
    assert xs == [(64 * k, 64 * (k + 1)) for k in range(7)] + [(448, 513)]
    # too narrow for two lines per tile: balanced (20 values over 3 tiles)
    stages, tasks = fft3d.query_pipeline((8, 8, 20), (3, 1), op=0, nstreams=1)
    xs = sorted({(t["box"][0], t["box"][1]) for t in tasks if stages[t["stage"]]["axis"] == 1})
    assert xs == [(0, 7), (7, 14), (14, 20)]
