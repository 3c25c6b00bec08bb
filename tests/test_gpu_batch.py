"""GPU parity of batched uneven-size transforms in one persistent launch.

The 64-transform workload (sizes drawn from a seed among 48^3, 64^3, 96^3,
100x120x128, 160x160x80, complex64): every output against its own FP64
oracle transform; bitwise equality with the same transform run alone through
a single-transform plan (same per-line arithmetic); graph replay, direct
persistent launch and one-launch-per-stage agree bit for bit.
"""
import numpy as np
import pytest
import torch

import oracle
import synth
from _util import fp32_bound, rel, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def workload():
    shapes = synth.batch_sizes()
    host = synth.batch_inputs(shapes, synth.CFG4["seed"])
    xs = [torch.from_numpy(a).cuda() for a in host]
    return shapes, host, xs


def test_config4_each_against_oracle_and_single_plan(gpu_lib, workload):
    shapes, host, xs = workload
    print(f"case batch of {len(shapes)}", flush=True)
    bp = gpu_lib.BatchPlan(shapes)
    outs = bp.forward(xs)
    torch.cuda.synchronize()
    bp.check()
    for i, (s, a) in enumerate(zip(shapes, host)):
        got = to_host(outs[i])
        assert rel(got, oracle.fftn(a.astype(np.complex128))) <= fp32_bound(a.size), (i, s)
    # bitwise equal to the single-transform plan (same per-line arithmetic)
    for i, s in enumerate(shapes[:12]):
        single = gpu_lib.Plan(s, torch.complex64).forward(xs[i])
        torch.cuda.synchronize()
        assert torch.equal(single, outs[i]), (i, s)
    # inverse brings every field back
    back = bp.inverse(outs)
    torch.cuda.synchronize()
    bp.check()
    for i, a in enumerate(host):
        assert rel(to_host(back[i]), a.astype(np.complex128)) <= fp32_bound(a.size), i
    bp.close()


def test_modes_and_graph_replays_agree(gpu_lib, workload):
    shapes, host, xs = workload
    ref = None
    for mode in (2, 1, 0):
        bp = gpu_lib.BatchPlan(shapes, mode=mode)
        outs = [torch.empty_like(x) for x in xs]
        for rep in range(3):  # graph replays, with eager torch work in between
            bp.forward(xs, outs)
            junk = torch.randn(1 << 20, device="cuda").sum()
            torch.cuda.synchronize()
            bp.check()
            if ref is None:
                ref = [o.clone() for o in outs]
            for i in range(len(xs)):
                assert torch.equal(outs[i], ref[i]), (mode, rep, i)
            del junk
        bp.close()


def test_pointer_changes_and_in_place(gpu_lib, workload):
    shapes, host, xs = workload
    sub = [0, 1, 2, 3, 4, 5]
    s6 = [shapes[i] for i in sub]
    bp = gpu_lib.BatchPlan(s6)
    ref = bp.forward([xs[i] for i in sub])
    torch.cuda.synchronize()
    copies = [xs[i].clone() for i in sub]
    bp.forward(copies, copies)  # new pointers, in place
    torch.cuda.synchronize()
    bp.check()
    for r, c in zip(ref, copies):
        assert torch.equal(r, c)
    bp.close()


def test_lines_per_item_do_not_change_bits(gpu_lib, workload):
    shapes, host, xs = workload
    uniq = sorted(set(shapes))
    xs1 = [xs[shapes.index(s)] for s in uniq]
    bp = gpu_lib.BatchPlan(uniq)
    ref = [o.clone() for o in bp.forward(xs1)]
    for n in (48, 64, 96, 100, 120, 128, 160, 80):
        for strided in (0, 1):
            for lw in (1, 3, 8):
                bp.set_lines(n, strided, lw)
                outs = bp.forward(xs1)
                torch.cuda.synchronize()
                bp.check()
                for r, o in zip(ref, outs):
                    assert torch.equal(r, o), (n, strided, lw)
            bp.set_lines(n, strided, 0)
    bp.close()


def test_batch_errors(gpu_lib):
    from paper_2601_12209_amd._lib import Fft3dError

    with pytest.raises(Fft3dError):
        gpu_lib.BatchPlan([(8, 8, 1024)])  # above 512
    bp = gpu_lib.BatchPlan([(8, 8, 8), (8, 8, 8)])
    buf = torch.zeros(1024, dtype=torch.complex64, device="cuda")
    a, b = buf[:512].view(8, 8, 8), buf[256:768].view(8, 8, 8)
    with pytest.raises(Fft3dError):  # two transforms writing overlapping memory
        bp.forward([a.clone(), a.clone()], [a, b])
    bp.close()
