"""athmhd_newdt_noalloc, the allocation-free variant of athmhd_newdt, against
athmhd_newdt through the C ABI: the same dt bit for bit and the same count of
non-physical cells, on two calls in a row whose second input is smaller (its
partial results must not be mixed with the stale ones of the first call, which
stay in the shared device array), on uniform and batched handles, and replayed
from a captured graph."""
import ctypes as C
import gc
import re

import numpy as np
import pytest

from paper_2005_06651_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch, torch.device("cuda:0")


@pytest.fixture(scope="module")
def athmhd():
    from paper_2005_06651_amd import athmhd as A
    A.lib()
    return A


def to_dev(torch, dev, x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev)


def newdt_ref(athmhd, s, cons, bface, nb):
    """athmhd_newdt through the C ABI: (dt, non-physical count); dt is written
    even when it reports ATHMHD_ENONPHYS"""
    out = C.c_double()
    rc = athmhd.lib().athmhd_newdt(s._h, C.c_void_p(cons.data_ptr()), C.c_void_p(bface.data_ptr()), nb,
                                   C.byref(out), C.c_void_p(0))
    if rc == athmhd.OK:
        return out.value, 0
    assert rc == athmhd.ENONPHYS, rc
    msg = athmhd.lib().athmhd_last_error(s._h).decode()
    return out.value, int(re.match(r"(\d+) non-physical", msg).group(1))


def noalloc(athmhd, torch, dev, s, cons, bface, nb):
    dt = torch.full((1,), -1.0, dtype=torch.float64, device=dev)
    nbad = torch.full((1,), -1, dtype=torch.int32, device=dev)
    rc = athmhd.lib().athmhd_newdt_noalloc(s._h, C.c_void_p(cons.data_ptr()), C.c_void_p(bface.data_ptr()), nb,
                                           C.c_void_p(dt.data_ptr()), C.c_void_p(nbad.data_ptr()), C.c_void_p(0))
    assert rc == athmhd.OK, athmhd.lib().athmhd_last_error(s._h).decode()
    torch.cuda.synchronize()
    return float(dt.item()), int(nbad.item())


def _blocks(orc, n, seeds, vmax):
    bl = [inputs.smooth_random(n=n, seed=sd, vmax=v) for sd, v in zip(seeds, vmax)]
    cfg = orc.cfg_for(bl[0])
    cons = np.stack([orc.prim2cons(cfg, b.prim, b.bface) for b in bl])
    return bl, cons, np.stack([b.bface for b in bl])


def test_noalloc_matches_newdt_uniform_two_calls(torch_dev, athmhd, orc):
    """nb = 3 then nb = 1: the second call's minimum is larger than the first's,
    so reading a stale partial of the first call would show."""
    torch, dev = torch_dev
    n = (37, 21, 13)
    bl, cons, bf = _blocks(orc, n, (91, 92, 93), (0.3, 0.6, 0.95))
    s = athmhd.Solver(bl[0].n, bl[0].ng, bl[0].dx, bl[0].gamma, nblocks=3)
    tc, tb = to_dev(torch, dev, cons), to_dev(torch, dev, bf)
    ref3 = newdt_ref(athmhd, s, tc, tb, 3)
    got3 = noalloc(athmhd, torch, dev, s, tc, tb, 3)
    assert got3 == ref3 and ref3[1] == 0
    ref1 = newdt_ref(athmhd, s, tc[:1].contiguous(), tb[:1].contiguous(), 1)
    got1 = noalloc(athmhd, torch, dev, s, tc[:1].contiguous(), tb[:1].contiguous(), 1)
    assert got1 == ref1
    assert ref1[0] > ref3[0]
    s.close()


def test_noalloc_matches_newdt_batched_then_smaller(torch_dev, athmhd, orc):
    """A batch of 12 uneven blocks, then a batch of its first 3 blocks with
    halved velocities on another handle of the same device (the scratch array
    is shared per device): every cell of the second is slower, so its dt is
    larger than the first's, whose partials stay in the array."""
    torch, dev = torch_dev
    blocks = inputs.amr_batch(12, seed=5)
    results = []
    for nblk, vscale in ((12, 1.0), (3, 0.5)):
        sub = blocks[:nblk]
        s = athmhd.BatchSolver([b.n for b in sub], [b.dx for b in sub], sub[0].ng, sub[0].gamma)
        parts_c, parts_b = [], []
        for b in sub:
            prim = b.prim.copy()
            prim[1:4] *= vscale
            parts_c.append(orc.prim2cons(orc.cfg_for(b), prim, b.bface).ravel())
            parts_b.append(b.bface.ravel())
        tc = to_dev(torch, dev, np.concatenate(parts_c))
        tb = to_dev(torch, dev, np.concatenate(parts_b))
        ref = newdt_ref(athmhd, s, tc, tb, nblk)
        got = noalloc(athmhd, torch, dev, s, tc, tb, nblk)
        assert got == ref and ref[1] == 0, (nblk, got, ref)
        results.append(ref[0])
        s.close()
    assert results[1] > results[0]


def test_noalloc_counts_non_physical_cells(torch_dev, athmhd, orc):
    """Cells with negative pressure, and a step that meets them first: the count
    (the step's plus the reduction's) and dt equal athmhd_newdt's, on twin
    handles, and both clear the handle's counter."""
    torch, dev = torch_dev
    b = inputs.smooth_random(n=(16, 12, 10), seed=95)
    cfg = orc.cfg_for(b)
    cons = orc.prim2cons(cfg, b.prim, b.bface)
    g = b.ng
    cons[4, g + 3, g + 4, g + 5] = 0.0  # E = 0: P < 0 there
    cons[4, g + 7, g + 1, g + 9] = -1.0
    res = []
    for which in ("ref", "noalloc"):
        s = athmhd.Solver(b.n, b.ng, b.dx, b.gamma)
        tc, tb = to_dev(torch, dev, cons), to_dev(torch, dev, b.bface)
        s.step(tc, tb, 1e-4)
        if which == "ref":
            res.append(newdt_ref(athmhd, s, tc, tb, 1))
            res.append(newdt_ref(athmhd, s, tc, tb, 1))
        else:
            res.append(noalloc(athmhd, torch, dev, s, tc, tb, 1))
            res.append(noalloc(athmhd, torch, dev, s, tc, tb, 1))
        s.close()
    assert res[0][1] > 0 and res[1][1] > 0 and res[1][1] < res[0][1]
    assert res[0] == res[2] and res[1] == res[3], res


def test_noalloc_replays_from_a_graph(torch_dev, athmhd, orc):
    """Captured once into a graph, replayed three times with eager updates of
    the input and eager work between the replays: each replay equals
    athmhd_newdt of the current state."""
    torch, dev = torch_dev
    b = inputs.smooth_random(n=(24, 16, 12), seed=96)
    cfg = orc.cfg_for(b)
    cons = orc.prim2cons(cfg, b.prim, b.bface)
    s = athmhd.Solver(b.n, b.ng, b.dx, b.gamma)
    tc, tb = to_dev(torch, dev, cons), to_dev(torch, dev, b.bface)
    dt = torch.zeros(1, dtype=torch.float64, device=dev)
    nbad = torch.zeros(1, dtype=torch.int32, device=dev)
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        s.newdt_noalloc(tc, tb, dt, nbad)
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    # thread-local capture after a collection (see test_gpu_amr's graph test)
    gc.collect()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, capture_error_mode="thread_local"):
        s.newdt_noalloc(tc, tb, dt, nbad)
    for it in range(3):
        s.step(tc, tb, 2e-3 * (it + 1))
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        torch.ones(1000, device=dev).sum()
        ref = s.newdt(tc, tb)
        assert float(dt.item()) == ref and int(nbad.item()) == 0, it
    s.close()
