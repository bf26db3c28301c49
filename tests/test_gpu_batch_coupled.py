"""Coupled batch: cube blocks of uneven sizes tiling one periodic domain at one
cell width (Sec. 2.1: a Mesh of MeshBlocks; Sec. 2.1.1: neighbours exchange
ghost cells and faces), their shell entries exchanged by table on the device
before every stage and after the last.  Across a slab boundary the blocks'
faces do not line up, so a ghost layer can come from several neighbours.

Split into blocks, the domain must step as the single block that covers it:
the dt exactly, the state to 1e-14 (the same kernels on the same values; x3
segments fall on other planes, and the compiler's copies of a segment's first
and last plane may round a face-field update differently by an ulp), and as
the oracle's single block within the 1e-12 bar, with div B at round-off.
"""
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


def to_dev(torch, dev, x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(dev)


def active(ng, n):
    return (slice(None), slice(ng, ng + n[2]), slice(ng, ng + n[1]), slice(ng, ng + n[0]))


def rel_l1(a, b):
    """worst relative L1 over the arrays of a (nv, ...) pair"""
    return max(float(np.abs(a[v] - b[v]).sum() / max(np.abs(b[v]).sum(), 1e-300)) for v in range(a.shape[0]))


def coupled_batch(athmhd, torch, dev, cons, bface, ng, dims, origins, domain, dx, gamma, **kw):
    bs = athmhd.BatchSolver(dims, [dx] * len(dims), ng, gamma, **kw)
    bs.couple(origins, domain)
    cs, fs = inputs.split_boxes(cons, bface, ng, dims, origins)
    return bs, to_dev(torch, dev, inputs.pack(cs)), to_dev(torch, dev, inputs.pack(fs))


def joined(bs, tc, tf, dims, origins, domain):
    c, f = tc.cpu().numpy(), tf.cpu().numpy()
    return inputs.join_boxes(bs.views(c, "cons"), bs.views(f, "bface"), bs.ng, dims, origins, domain)


def test_exchange_is_the_periodic_domain(torch_dev, athmhd):
    """After the exchange every stored entry of every block (ghost cells, the
    faces of its shell, padding) equals the entry at the same position of the
    periodic domain, bitwise, with blocks of 2, 4 and 6 cells (3 ghost layers,
    deeper than the smallest blocks)."""
    torch, dev = torch_dev
    ng = 3
    dims, origins, domain = inputs.brick_layout([2, 4, 6, 2], 12)
    rng = np.random.default_rng(5)
    N = [domain[d] + 2 * ng for d in range(3)]
    cells = rng.standard_normal((5, N[2], N[1], N[0]))
    faces = rng.standard_normal((3, N[2] + 1, N[1] + 1, N[0] + 1))
    want_c, want_f = inputs.split_boxes(cells, faces, ng, dims, origins)
    junk_c, junk_f = [], []
    for wc, wf, n in zip(want_c, want_f, dims):
        jc, jf = np.full_like(wc, -7.0), np.full_like(wf, -7.0)
        a = active(ng, n)
        jc[a] = wc[a]
        jf[a] = wf[a]
        junk_c.append(jc)
        junk_f.append(jf)
    bs = athmhd.BatchSolver(dims, [(0.1, 0.1, 0.1)] * len(dims), ng, 5.0 / 3.0)
    bs.couple(origins, domain)
    tc, tf = to_dev(torch, dev, inputs.pack(junk_c)), to_dev(torch, dev, inputs.pack(junk_f))
    bs.fill_ghosts(tc, tf)
    assert np.array_equal(tc.cpu().numpy(), inputs.pack(want_c))
    assert np.array_equal(tf.cpu().numpy(), inputs.pack(want_f))
    bs.close()


@pytest.mark.parametrize("slabs,kw", [
    ([8, 6, 4], dict(integrator="vl2", recon="plm", riemann="hlld")),
    ([6, 8, 6], dict(integrator="rk3", recon="ppm", riemann="hlle")),
    ([4, 8], dict(integrator="rk1", recon="dc", riemann="hlld")),
    ([8, 4, 6], dict(integrator="rk2", recon="dc", riemann="hlld", ct_eps=1e-3)),
])
def test_coupled_batch_equals_single_block_and_oracle(torch_dev, athmhd, orc, slabs, kw):
    """A 24 x 24 x H domain as slabs of cubes: three steps with the CFL dt of
    the batch, which must equal the single block's exactly and the oracle's;
    then the blocks' cells and faces agree with the single GPU block's to
    1e-14 and the oracle's within the bar, and div B stays at round-off."""
    torch, dev = torch_dev
    ng = 3 if kw["recon"] == "ppm" else 2
    dims, origins, domain = inputs.brick_layout(slabs, 24)
    b = inputs.smooth_random(n=domain, seed=43, ng=ng)
    cfg = orc.cfg_for(b, **kw)
    cons = orc.prim2cons(cfg, b.prim, b.bface)
    single = athmhd.Solver(b.n, ng, b.dx, b.gamma, **kw)
    bs, tc, tf = coupled_batch(athmhd, torch, dev, cons, b.bface, ng, dims, origins, domain, b.dx, b.gamma, **kw)
    tsc, tsf = to_dev(torch, dev, cons), to_dev(torch, dev, b.bface)
    rc, rb = cons.copy(), b.bface.copy()
    for _ in range(3):
        dt, bad = orc.newdt(cfg, rc, rb)
        assert bad == 0
        bdt = bs.newdt(tc, tf)
        assert bdt == single.newdt(tsc, tsf)
        assert abs(bdt - dt) <= 1e-14 * dt
        assert orc.step(cfg, rc, rb, dt) == 0
        single.step(tsc, tsf, dt)
        bs.step(tc, tf, dt)
    jc, jf = joined(bs, tc, tf, dims, origins, domain)
    a = active(ng, b.n)
    sc, sf = tsc.cpu().numpy(), tsf.cpu().numpy()
    err_single = max(rel_l1(jc[a], sc[a]), rel_l1(jf[a], sf[a]))
    err_oracle = max(rel_l1(jc[a], rc[a]), rel_l1(jf[a], rb[a]))
    print(f"coupled batch {kw['integrator']}+{kw['recon']}: vs single block {err_single:.2e}, "
          f"vs oracle {err_oracle:.2e}")
    assert err_single <= 1e-14
    assert err_oracle <= TOL
    orc.fill_ghosts(cfg, jc, jf)
    assert inputs.divb_metric(jf, b.n, ng, b.dx) <= 1e-13
    bs.close()
    single.close()


# boxes of unequal shape whose faces do not line up along x1 and x2 either:
# (origin, dims) tiling a 24 x 24 x 10 domain
GENERAL_BOXES = [
    ((0, 0, 0), (8, 24, 6)), ((8, 0, 0), (16, 10, 6)), ((8, 10, 0), (16, 14, 6)),
    ((0, 0, 6), (12, 9, 4)), ((12, 0, 6), (12, 9, 4)), ((0, 9, 6), (5, 15, 4)), ((5, 9, 6), (19, 15, 4)),
]


@pytest.mark.parametrize("layout,kw", [
    ("general", dict(integrator="vl2", recon="plm", riemann="hlld")),
    ("general", dict(integrator="rk3", recon="ppm", riemann="hlld")),
    ("thin", dict(integrator="rk3", recon="ppm", riemann="hlle")),
])
def test_coupled_batch_general_layouts(torch_dev, athmhd, orc, layout, kw):
    """Blocks that are not cubes and whose neighbours differ along every
    direction (seven boxes tiling 24 x 24 x 10), and slabs of 2-cell cubes
    thinner than PPM's three ghost layers: three steps against the single
    block (dt exactly, state to 1e-14) and the oracle (within the bar)."""
    torch, dev = torch_dev
    ng = 3 if kw["recon"] == "ppm" else 2
    if layout == "general":
        origins = [o for o, _ in GENERAL_BOXES]
        dims = [n for _, n in GENERAL_BOXES]
        domain = (24, 24, 10)
    else:
        dims, origins, domain = inputs.brick_layout([2, 4, 2, 6], 12)
    b = inputs.smooth_random(n=domain, seed=46, ng=ng)
    cfg = orc.cfg_for(b, **kw)
    cons = orc.prim2cons(cfg, b.prim, b.bface)
    single = athmhd.Solver(b.n, ng, b.dx, b.gamma, **kw)
    bs, tc, tf = coupled_batch(athmhd, torch, dev, cons, b.bface, ng, dims, origins, domain, b.dx, b.gamma, **kw)
    tsc, tsf = to_dev(torch, dev, cons), to_dev(torch, dev, b.bface)
    rc, rb = cons.copy(), b.bface.copy()
    for _ in range(3):
        dt, bad = orc.newdt(cfg, rc, rb)
        assert bad == 0
        bdt = bs.newdt(tc, tf)
        assert bdt == single.newdt(tsc, tsf)
        assert orc.step(cfg, rc, rb, dt) == 0
        single.step(tsc, tsf, dt)
        bs.step(tc, tf, dt)
    jc, jf = joined(bs, tc, tf, dims, origins, domain)
    a = active(ng, b.n)
    sc, sf = tsc.cpu().numpy(), tsf.cpu().numpy()
    err_single = max(rel_l1(jc[a], sc[a]), rel_l1(jf[a], sf[a]))
    err_oracle = max(rel_l1(jc[a], rc[a]), rel_l1(jf[a], rb[a]))
    print(f"coupled batch, {layout} layout, {kw['integrator']}+{kw['recon']}: vs single block {err_single:.2e}, "
          f"vs oracle {err_oracle:.2e}")
    assert err_single <= 1e-14
    assert err_oracle <= TOL
    orc.fill_ghosts(cfg, jc, jf)
    assert inputs.divb_metric(jf, b.n, ng, b.dx) <= 1e-13
    bs.close()
    single.close()


@pytest.mark.parametrize("shape", [0, 1, 2, 3])
@pytest.mark.parametrize("split", [0, 1])
def test_coupled_batch_every_tile(torch_dev, athmhd, orc, shape, split):
    """Every tile candidate of the batched stage kernel, with and without the
    x3 split, on the seven general boxes: two VL2+PLM+HLLD steps equal the
    single block's to 1e-14."""
    torch, dev = torch_dev
    origins = [o for o, _ in GENERAL_BOXES]
    dims = [n for _, n in GENERAL_BOXES]
    domain = (24, 24, 10)
    b = inputs.smooth_random(n=domain, seed=47, ng=2)
    cons = orc.prim2cons(orc.cfg_for(b), b.prim, b.bface)
    single = athmhd.Solver(b.n, 2, b.dx, b.gamma)
    bs, tc, tf = coupled_batch(athmhd, torch, dev, cons, b.bface, 2, dims, origins, domain, b.dx, b.gamma)
    bs.set_tile(shape, split)
    tsc, tsf = to_dev(torch, dev, cons), to_dev(torch, dev, b.bface)
    for _ in range(2):
        dt = single.newdt(tsc, tsf)
        assert bs.newdt(tc, tf) == dt
        single.step(tsc, tsf, dt)
        bs.step(tc, tf, dt)
    jc, jf = joined(bs, tc, tf, dims, origins, domain)
    a = active(2, b.n)
    sc, sf = tsc.cpu().numpy(), tsf.cpu().numpy()
    assert max(rel_l1(jc[a], sc[a]), rel_l1(jf[a], sf[a])) <= 1e-14
    bs.close()
    single.close()


def test_coupled_batch_chain_graph_and_tuner(torch_dev, athmhd, orc):
    """Chained steps (which take their input's shell entries as current)
    equal newdt + step (which exchanges before every stage) bit for bit, also
    after active entries next to block boundaries were changed and
    athmhd_fill_ghosts was called; after the tuner has timed its candidates,
    three steps replayed from a hipGraph equal three eager steps bit for
    bit."""
    from test_gpu_chain import chain_vs_newdt_step
    torch, dev = torch_dev
    dims, origins, domain = inputs.brick_layout([8, 4, 8], 16)
    b = inputs.smooth_random(n=domain, seed=44, ng=2)
    cons = orc.prim2cons(orc.cfg_for(b), b.prim, b.bface)
    bs, tc, tf = coupled_batch(athmhd, torch, dev, cons, b.bface, 2, dims, origins, domain, b.dx, b.gamma)
    chain_vs_newdt_step(torch, dev, bs, tc, tf)
    # raise the density of the first and last active cells of every block
    pc, pf = tc.clone(), tf.clone()
    for v, n in zip(bs.views(pc, "cons"), dims):
        v[0, 2, 2, 2] *= 1.01
        v[0, 1 + n[2], 1 + n[1], 1 + n[0]] *= 0.99
    bs.fill_ghosts(pc, pf)
    chain_vs_newdt_step(torch, dev, bs, pc, pf)
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        bs.tune(tc, tf, stream=stream)
        dts, states = [], []
        ec, ef = tc.clone(), tf.clone()
        for it in range(3):
            dt = bs.newdt(ec, ef, stream=stream) * (0.7 + 0.1 * it)
            bs.step(ec, ef, dt, stream=stream)
            dts.append(dt)
            states.append((ec.clone(), ef.clone()))
        bs.set_graph(True)
        gc, gf = tc.clone(), tf.clone()
        for it, dt in enumerate(dts):
            bs.step(gc, gf, dt, stream=stream)
            stream.synchronize()
            torch.ones(1000, device=dev).sum()  # unrelated eager work between replays
            assert torch.equal(gc, states[it][0]) and torch.equal(gf, states[it][1]), it
    bs.close()


def test_couple_rejects_bad_layouts(torch_dev, athmhd):
    """Overlap, gap, a block outside the domain, unequal cell widths, floors,
    passive scalars and a second call are refused with the documented codes;
    floors cannot be switched on once coupled."""
    A = athmhd
    dims, origins, domain = inputs.brick_layout([4, 4], 8)
    dx = [(0.1, 0.1, 0.1)] * len(dims)

    def code(fn):
        with pytest.raises(A.AthmhdError) as e:
            fn()
        return e.value.code

    def attempt(o, dom, dxs=dx, floors=False, ns=0):
        bs = A.BatchSolver(dims, dxs, 2, 5.0 / 3.0, nscalars=ns)
        try:
            if floors:
                bs.set_floors(1e-6, 1e-6)
            bs.couple(o, dom)
        finally:
            bs.close()

    over = list(origins)
    over[1] = over[0]
    assert code(lambda: attempt(over, domain)) == A.EINVAL
    assert code(lambda: attempt(origins, (8, 8, 12))) == A.EINVAL       # a slab of cells in no block
    assert code(lambda: attempt(origins, (8, 8, 6))) == A.EINVAL        # blocks past the domain
    odd = list(dx)
    odd[3] = (0.1, 0.1, 0.2)
    assert code(lambda: attempt(origins, domain, dxs=odd)) == A.EINVAL
    assert code(lambda: attempt(origins, domain, floors=True)) == A.EUNSUP
    assert code(lambda: attempt(origins, domain, ns=1)) == A.EUNSUP
    bs = A.BatchSolver(dims, dx, 2, 5.0 / 3.0)
    bs.couple(origins, domain)
    assert code(lambda: bs.couple(origins, domain)) == A.EINVAL
    assert code(lambda: bs.set_floors(1e-6, 1e-6)) == A.EUNSUP
    bs.close()


def test_coupled_batch_1032_blocks_equals_single_block(torch_dev, athmhd):
    """The benchmarked layout: 1032 cubes (432 of 16^3, 384 of 24^3, 216 of
    32^3) in x3 slabs of a 192 x 192 x 384 periodic domain.  Two steps agree
    with the single 192 x 192 x 384 block's to 1e-14, with equal dt."""
    torch, dev = torch_dev
    dims, origins, domain = inputs.brick_layout(inputs.brick_slabs(), 192)
    assert len(dims) == 1032
    b = inputs.smooth_random(n=domain, seed=45, ng=2)
    single = athmhd.Solver(b.n, 2, b.dx, b.gamma)
    tsf = to_dev(torch, dev, b.bface)
    tsc = single.prim2cons(to_dev(torch, dev, b.prim), tsf)
    bs, tc, tf = coupled_batch(athmhd, torch, dev, tsc.cpu().numpy(), b.bface, 2, dims, origins, domain, b.dx,
                               b.gamma)
    for _ in range(2):
        dt = single.newdt(tsc, tsf)
        assert bs.newdt(tc, tf) == dt
        single.step(tsc, tsf, dt)
        bs.step(tc, tf, dt)
    jc, jf = joined(bs, tc, tf, dims, origins, domain)
    a = active(2, b.n)
    sc, sf = tsc.cpu().numpy(), tsf.cpu().numpy()
    err = max(rel_l1(jc[a], sc[a]), rel_l1(jf[a], sf[a]))
    print(f"1032 coupled blocks vs the single block: {err:.2e}")
    assert err <= 1e-14
    bs.close()
    single.close()
