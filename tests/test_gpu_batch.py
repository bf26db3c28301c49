"""Batched blocks of uneven sizes (one persistent launch per stage), the tile
autotuner and hipGraph replay, checked against the CPU oracle run block by
block (every block is its own periodic neighbour, one global dt)."""
import numpy as np
import pytest

from paper_2005_06651_amd import inputs

pytestmark = pytest.mark.gpu

TOL = 1e-12


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


def rel_l1(b, gc, gb, rc, rb):
    g = b.ng
    n1, n2, n3 = b.n
    a = b.active
    worst = 0.0
    for v in range(5):
        worst = max(worst, np.abs(gc[v][a] - rc[v][a]).sum() / max(np.abs(rc[v][a]).sum(), 1e-300))
    for c in range(3):
        sl = (c, slice(g, g + n3), slice(g, g + n2), slice(g, g + n1))
        worst = max(worst, np.abs(gb[sl] - rb[sl]).sum() / max(np.abs(rb[sl]).sum(), 1e-300))
    return worst


def small_batch(seed=7, ng=2):
    """Blocks of several shapes, including non-cubic ones and ones smaller
    than a tile."""
    shapes = [(16, 16, 16), (24, 24, 24), (32, 32, 32), (16, 24, 8), (9, 13, 21), (24, 16, 32), (5, 7, 6)]
    blocks = []
    for b, n in enumerate(shapes):
        dx = (0.5 / n[0], 0.5 / n[1], 0.5 / n[2])
        blocks.append(inputs.smooth_random(n=n, seed=seed * 31 + b, ng=ng, dx=dx))
    return blocks


def setup(torch, dev, athmhd, orc, blocks, **kw):
    s = athmhd.BatchSolver([b.n for b in blocks], [b.dx for b in blocks], blocks[0].ng, blocks[0].gamma, **kw)
    cfgs = [orc.cfg_for(b, **kw) for b in blocks]
    cons = [orc.prim2cons(c, b.prim, b.bface) for c, b in zip(cfgs, blocks)]
    tc = torch.from_numpy(inputs.pack(cons)).to(dev)
    tb = torch.from_numpy(inputs.pack([b.bface for b in blocks])).to(dev)
    return s, cfgs, cons, tc, tb


@pytest.mark.parametrize("shape,split", [(0, 0), (1, 1), (2, 0), (3, 1)])
@pytest.mark.parametrize("integ,recon,rs", [("vl2", "plm", "hlld"), ("rk3", "ppm", "hlle")])
def test_batch_matches_oracle_per_block(torch_dev, athmhd, orc, shape, split, integ, recon, rs):
    torch, dev = torch_dev
    ng = 3 if recon == "ppm" else 2
    blocks = small_batch(ng=ng)
    kw = dict(integrator=integ, recon=recon, riemann=rs)
    s, cfgs, cons, tc, tb = setup(torch, dev, athmhd, orc, blocks, **kw)
    s.set_tile(shape, split)
    rc = [c.copy() for c in cons]
    rb = [b.bface.copy() for b in blocks]
    for _ in range(2):
        dts = [orc.newdt(c, x, y)[0] for c, x, y in zip(cfgs, rc, rb)]
        dt = min(dts)
        gdt = s.newdt(tc, tb)
        assert abs(gdt - dt) <= 1e-14 * dt
        for c, x, y in zip(cfgs, rc, rb):
            assert orc.step(c, x, y, dt) == 0
        s.step(tc, tb, dt)
    s.fill_ghosts(tc, tb)  # the step leaves ghosts and periodic image faces as they were
    gc = s.views(tc.cpu().numpy(), "cons")
    gb = s.views(tb.cpu().numpy(), "bface")
    for b, blk in enumerate(blocks):
        assert rel_l1(blk, gc[b], gb[b], rc[b], rb[b]) <= TOL, (b, blk.n)
        assert inputs.divb_metric(gb[b], blk.n, blk.ng, blk.dx) <= 1e-13
    s.close()


def test_batch_prim2cons_and_ghosts(torch_dev, athmhd, orc):
    torch, dev = torch_dev
    blocks = small_batch(seed=8)
    s = athmhd.BatchSolver([b.n for b in blocks], [b.dx for b in blocks], 2, blocks[0].gamma)
    tb = torch.from_numpy(inputs.pack([b.bface for b in blocks])).to(dev)
    tc = s.prim2cons(torch.from_numpy(inputs.pack([b.prim for b in blocks])).to(dev), tb)
    gc = s.views(tc.cpu().numpy(), "cons")
    for b, blk in enumerate(blocks):
        ref = orc.prim2cons(orc.cfg_for(blk), blk.prim, blk.bface)
        assert np.max(np.abs(gc[b] - ref) / np.maximum(np.abs(ref), 1.0)) < 1e-15
    # ghost fill reproduces the periodic images bitwise after scrambling
    junk = tc.clone()
    for b, blk in enumerate(blocks):
        v = s.views(junk, "cons")[b]
        g = blk.ng
        v[:, :g] = -7.0
        v[:, :, -g:] = 3.0
    s.fill_ghosts(junk, tb)
    assert torch.equal(junk, tc)
    s.close()


def test_autotune_keeps_results(torch_dev, athmhd, orc):
    torch, dev = torch_dev
    blocks = small_batch(seed=9)
    s, cfgs, cons, tc, tb = setup(torch, dev, athmhd, orc, blocks)
    before_c, before_b = tc.clone(), tb.clone()
    shape, split, ms = s.tune(tc, tb)
    assert 0 <= shape < len(athmhd.BATCH_TILES) and split in (0, 1) and ms > 0
    assert torch.equal(tc, before_c) and torch.equal(tb, before_b)  # the tuner does not touch the state
    dt = s.newdt(tc, tb)
    s.step(tc, tb, dt)
    rc = [c.copy() for c in cons]
    rb = [b.bface.copy() for b in blocks]
    for c, x, y in zip(cfgs, rc, rb):
        orc.step(c, x, y, dt)
    gc = s.views(tc.cpu().numpy(), "cons")
    gb = s.views(tb.cpu().numpy(), "bface")
    for b, blk in enumerate(blocks):
        assert rel_l1(blk, gc[b], gb[b], rc[b], rb[b]) <= TOL
    s.close()


def test_graph_replay_matches_eager(torch_dev, athmhd, orc):
    """Uniform and batched handles: a step replayed from a hipGraph (dt updated
    per replay) equals the eagerly launched step bitwise, replay after replay,
    with eager work and synchronisations in between."""
    torch, dev = torch_dev
    stream = torch.cuda.Stream()
    b = inputs.turbulence(n=40, seed=6)
    for kind in ("uniform", "batch"):
        if kind == "uniform":
            mk = lambda: athmhd.Solver(b.n, b.ng, b.dx, b.gamma)
            cons0 = orc.prim2cons(orc.cfg_for(b), b.prim, b.bface)
            c0 = torch.from_numpy(cons0).to(dev)
            b0 = torch.from_numpy(b.bface).to(dev)
        else:
            blocks = small_batch(seed=10)
            mk = lambda: athmhd.BatchSolver([x.n for x in blocks], [x.dx for x in blocks], 2, blocks[0].gamma)
            c0 = torch.from_numpy(inputs.pack([orc.prim2cons(orc.cfg_for(x), x.prim, x.bface) for x in blocks])).to(dev)
            b0 = torch.from_numpy(inputs.pack([x.bface for x in blocks])).to(dev)
        eager, graph = mk(), mk()
        graph.set_graph(True)
        ce, be = c0.clone(), b0.clone()
        cg, bg = c0.clone(), b0.clone()
        with torch.cuda.stream(stream):
            for it in range(4):
                dt = eager.newdt(ce, be, stream=stream) * (0.7 + 0.1 * it)
                eager.step(ce, be, dt, stream=stream)
                graph.step(cg, bg, dt, stream=stream)
                stream.synchronize()
                junk = torch.ones(1000, device=dev).sum()  # unrelated eager work between replays
                assert torch.equal(ce, cg) and torch.equal(be, bg), (kind, it)
        eager.close()
        graph.close()


@pytest.mark.parametrize("integ,recon,rs,ns,floors", [
    ("vl2", "plm", "hlld", 2, None),
    ("rk3", "ppm", "hlle", 1, None),
    ("rk2", "dc", "hlld", 3, (0.8, 0.9)),
])
def test_batch_with_scalars_matches_oracle_per_block(torch_dev, athmhd, orc, integ, recon, rs, ns, floors):
    """Passive scalars (Sec. 3.2.6) on batched blocks of several shapes, some
    smaller than a scalar tile: two steps, every block's MHD arrays and
    scalars against the oracle's within the 1e-12 bar."""
    torch, dev = torch_dev
    ng = 3 if recon == "ppm" else 2
    blocks = [inputs.with_scalars(b, ns, seed=90 + i) for i, b in enumerate(small_batch(seed=9, ng=ng))]
    kw = dict(integrator=integ, recon=recon, riemann=rs)
    s = athmhd.BatchSolver([b.n for b in blocks], [b.dx for b in blocks], ng, blocks[0].gamma, nscalars=ns, **kw)
    fl = floors or (0.0, 0.0)
    if floors:
        s.set_floors(*floors)
    cfgs = [orc.cfg_for(b, nscalars=ns, dfloor=fl[0], pfloor=fl[1], **kw) for b in blocks]
    cons = [orc.prim2cons(orc.cfg_for(b, nscalars=ns, **kw), b.prim, b.bface) for b in blocks]
    tb = torch.from_numpy(inputs.pack([b.bface for b in blocks])).to(dev)
    tc = s.prim2cons(torch.from_numpy(inputs.pack([b.prim for b in blocks])).to(dev), tb)
    gc0 = s.views(tc.cpu().numpy(), "cons")
    for b in range(len(blocks)):
        assert np.array_equal(gc0[b][5:], cons[b][5:])
    rc = [c.copy() for c in cons]
    rb = [b.bface.copy() for b in blocks]
    for _ in range(2):
        dt = min(orc.newdt(c, x, y)[0] for c, x, y in zip(cfgs, rc, rb))
        assert abs(s.newdt(tc, tb) - dt) <= 1e-13 * dt
        for c, x, y in zip(cfgs, rc, rb):
            assert orc.step(c, x, y, dt) == 0
        s.step(tc, tb, dt)
    gc = s.views(tc.cpu().numpy(), "cons")
    gb = s.views(tb.cpu().numpy(), "bface")
    for b, blk in enumerate(blocks):
        g = blk.ng
        a = (slice(None), slice(g, g + blk.n[2]), slice(g, g + blk.n[1]), slice(g, g + blk.n[0]))
        for x, y in ((gc[b][a], rc[b][a]), (gb[b][a], rb[b][a])):
            for v in range(x.shape[0]):
                err = np.abs(x[v] - y[v]).sum() / max(np.abs(y[v]).sum(), 1e-300)
                assert err <= TOL, (b, blk.n, v, err)
    s.close()


def test_batch_graph_replay_with_scalars(torch_dev, athmhd, orc):
    """hipGraph replays of a batched step with scalars equal eager steps."""
    torch, dev = torch_dev
    stream = torch.cuda.Stream()
    blocks = [inputs.with_scalars(b, 2, seed=95 + i) for i, b in enumerate(small_batch(seed=10))]
    mk = lambda: athmhd.BatchSolver([x.n for x in blocks], [x.dx for x in blocks], 2, blocks[0].gamma, nscalars=2)
    eager, graph = mk(), mk()
    graph.set_graph(True)
    b0 = torch.from_numpy(inputs.pack([x.bface for x in blocks])).to(dev)
    c0 = eager.prim2cons(torch.from_numpy(inputs.pack([x.prim for x in blocks])).to(dev), b0)
    ce, be, cg, bg = c0.clone(), b0.clone(), c0.clone(), b0.clone()
    with torch.cuda.stream(stream):
        for it in range(4):
            dt = eager.newdt(ce, be, stream=stream) * (0.7 + 0.1 * it)
            eager.step(ce, be, dt, stream=stream)
            graph.step(cg, bg, dt, stream=stream)
            stream.synchronize()
            torch.ones(1000, device=dev).sum()
            assert torch.equal(ce, cg) and torch.equal(be, bg), it
    eager.close()
    graph.close()
