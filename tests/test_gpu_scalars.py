"""Passive scalars on the GPU (Sec. 3.2.6, Eq. (passive_scalars)): the fused
stage kernel stores the face mass fluxes and the scalar kernels carry C_i with
them.  Checked against the oracle element by element at the 1e-12 bar, on
ragged blocks spanning several tiles and x3 segments, for every
reconstruction, both Riemann solvers, floors and several blocks; plus the
properties the transport equation fixes (C = 1 follows rho, the MHD state
does not see the scalars), graph replay, and sampled windows of the 256^3
turbulence with two scalars.
"""
import numpy as np
import pytest

import windows as W
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


def act(b):
    g = b.ng
    n1, n2, n3 = b.n
    return (slice(None), slice(g, g + n3), slice(g, g + n2), slice(g, g + n1))


def rel_l1_each(a, b):
    """relative L1 of every array of a (nv, ...) pair"""
    return [float(np.abs(a[v] - b[v]).sum() / max(np.abs(b[v]).sum(), 1e-300)) for v in range(a.shape[0])]


CASES = [
    # (integrator, recon, riemann, nscalars, extra oracle/GPU settings)
    ("vl2", "plm", "hlld", 1, {}),
    ("rk3", "ppm", "hlle", 2, {}),
    ("rk2", "dc", "hlld", 3, {"ct_eps": 1e-3}),
    ("rk1", "plm", "hlle", 1, {}),
    ("vl2", "plm", "hlld", 2, {"floors": (0.8, 0.9)}),
    ("rk3", "dc", "hlld", 1, {"floors": (0.8, 0.9)}),
]


@pytest.mark.parametrize("integ,recon,rs,ns,extra", CASES)
def test_scalar_steps_match_oracle(torch_dev, athmhd, orc, integ, recon, rs, ns, extra):
    """Three steps of a 40 x 30 x 20 block (two tiles along x1 and three along
    x2, both ragged, several x3 segments) against the oracle: dt, the MHD
    state and every scalar."""
    torch, dev = torch_dev
    ng = 3 if recon == "ppm" else 2
    b = inputs.with_scalars(inputs.smooth_random(n=(40, 30, 20), seed=61, ng=ng), ns, seed=62)
    kw = dict(integrator=integ, recon=recon, riemann=rs, ct_eps=extra.get("ct_eps", 0.0))
    fl = extra.get("floors", (0.0, 0.0))
    s = athmhd.Solver(b.n, b.ng, b.dx, b.gamma, nscalars=ns, **kw)
    if fl[0] > 0:
        s.set_floors(*fl)
    cfg = orc.cfg_for(b, nscalars=ns, dfloor=fl[0], pfloor=fl[1], **kw)
    cons = orc.prim2cons(orc.cfg_for(b, nscalars=ns, **kw), b.prim, b.bface)
    tc, tb = to_dev(torch, dev, cons), to_dev(torch, dev, b.bface)
    got = s.prim2cons(to_dev(torch, dev, b.prim), tb).cpu().numpy()
    assert np.array_equal(got[5:], cons[5:])  # rho C_i = rho * C_i, one rounding on both sides
    assert np.max(np.abs(got[:5] - cons[:5]) / np.maximum(np.abs(cons[:5]), 1.0)) < 1e-15
    rc, rb = cons.copy(), b.bface.copy()
    orc.take_floor_count()
    for _ in range(3):
        dt, bad = orc.newdt(cfg, rc, rb)
        assert bad == 0
        assert abs(s.newdt(tc, tb) - dt) <= 1e-13 * dt
        assert orc.step(cfg, rc, rb, dt) == 0
        s.step(tc, tb, dt)
    if fl[0] > 0:
        assert orc.take_floor_count() > 0 and s.floor_count() > 0
    a = act(b)
    errs = rel_l1_each(tc.cpu().numpy()[a], rc[a]) + rel_l1_each(tb.cpu().numpy()[a], rb[a])
    print("rel L1 per array", " ".join(f"{e:.1e}" for e in errs), flush=True)
    assert max(errs) <= TOL
    s.close()


def test_unit_concentration_follows_density(torch_dev, athmhd, orc):
    """C = 1 turns the scalar equation into the continuity equation: rho C
    follows rho (to rounding: the two are summed in different orders)."""
    torch, dev = torch_dev
    b = inputs.with_scalars(inputs.smooth_random(n=(36, 20, 12), seed=63), 1, seed=64)
    prim = b.prim.copy()
    prim[5] = 1.0
    s = athmhd.Solver(b.n, b.ng, b.dx, b.gamma, nscalars=1)
    tb = to_dev(torch, dev, b.bface)
    tc = s.prim2cons(to_dev(torch, dev, prim), tb)
    for _ in range(4):
        s.step(tc, tb, s.newdt(tc, tb))
    c = tc.cpu().numpy()[act(b)]
    err = np.abs(c[5] - c[0]).max() / np.abs(c[0]).max()
    print("max |rho C - rho| / max rho", err, flush=True)
    assert err <= 1e-14
    s.close()


@pytest.mark.parametrize("recon,integ", [("plm", "vl2"), ("ppm", "rk3")])
def test_mhd_state_does_not_see_the_scalars(torch_dev, athmhd, orc, recon, integ):
    torch, dev = torch_dev
    ng = 3 if recon == "ppm" else 2
    b = inputs.with_scalars(inputs.smooth_random(n=(40, 30, 20), seed=65, ng=ng), 2, seed=66)
    kw = dict(integrator=integ, recon=recon, riemann="hlld")
    s2 = athmhd.Solver(b.n, b.ng, b.dx, b.gamma, nscalars=2, **kw)
    s0 = athmhd.Solver(b.n, b.ng, b.dx, b.gamma, **kw)
    tb2 = to_dev(torch, dev, b.bface)
    tc2 = s2.prim2cons(to_dev(torch, dev, b.prim), tb2)
    tb0 = tb2.clone()
    tc0 = tc2[:5].clone()
    for _ in range(3):
        dt = s0.newdt(tc0, tb0)
        assert s2.newdt(tc2, tb2) == dt
        s0.step(tc0, tb0, dt)
        s2.step(tc2, tb2, dt)
    same = torch.equal(tc2[:5], tc0) and torch.equal(tb2, tb0)
    a = act(b)
    errs = rel_l1_each(tc2[:5].cpu().numpy()[a], tc0.cpu().numpy()[a]) + rel_l1_each(tb2.cpu().numpy()[a],
                                                                                    tb0.cpu().numpy()[a])
    print("bitwise equal:", same, "worst rel L1", max(errs), flush=True)
    assert max(errs) <= 1e-14
    s0.close()
    s2.close()


def test_scalar_blocks_are_independent(torch_dev, athmhd, orc):
    """Two blocks with scalars in one handle: each against its own oracle step."""
    torch, dev = torch_dev
    bl = [inputs.with_scalars(inputs.smooth_random(n=(24, 16, 10), seed=67 + i), 2, seed=70 + i) for i in range(2)]
    s = athmhd.Solver(bl[0].n, 2, bl[0].dx, bl[0].gamma, nscalars=2, nblocks=2)
    cfg = orc.cfg_for(bl[0], nscalars=2)
    cons = np.stack([orc.prim2cons(cfg, x.prim, x.bface) for x in bl])
    bf = np.stack([x.bface for x in bl])
    tc, tb = to_dev(torch, dev, cons), to_dev(torch, dev, bf)
    dt = 0.004
    s.step(tc, tb, dt)
    gc, gb = tc.cpu().numpy(), tb.cpu().numpy()
    a = act(bl[0])
    for i in range(2):
        rc, rb = cons[i].copy(), bf[i].copy()
        assert orc.step(cfg, rc, rb, dt) == 0
        assert max(rel_l1_each(gc[i][a], rc[a]) + rel_l1_each(gb[i][a], rb[a])) <= TOL
    s.close()


def test_graph_replay_with_scalars(torch_dev, athmhd, orc):
    """hipGraph replays of a step with scalars equal eager steps bitwise, with
    eager work and synchronisations between replays."""
    torch, dev = torch_dev
    stream = torch.cuda.Stream()
    b = inputs.with_scalars(inputs.turbulence(n=40, seed=6), 2, seed=68)
    cfg = orc.cfg_for(b, nscalars=2)
    c0 = to_dev(torch, dev, orc.prim2cons(cfg, b.prim, b.bface))
    b0 = to_dev(torch, dev, b.bface)
    eager = athmhd.Solver(b.n, b.ng, b.dx, b.gamma, nscalars=2)
    graph = athmhd.Solver(b.n, b.ng, b.dx, b.gamma, nscalars=2)
    graph.set_graph(True)
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


def test_scalars_reject_reverse_mode(torch_dev, athmhd):
    torch, dev = torch_dev
    b = inputs.with_scalars(inputs.smooth_random(n=(8, 8, 8), seed=69), 1, seed=70)
    s = athmhd.Solver(b.n, b.ng, b.dx, b.gamma, nscalars=1)
    tb = to_dev(torch, dev, b.bface)
    tc = s.prim2cons(to_dev(torch, dev, b.prim), tb)
    with pytest.raises(athmhd.AthmhdError) as e:
        s.step_vjp(tc, tb, 1e-3, tc.clone(), tb.clone())
    assert e.value.code == athmhd.EUNSUP
    s.close()


def test_turbulence_256_with_scalars_sampled_windows(torch_dev, athmhd, orc):
    """The benchmark's 256^3 turbulence with two scalars (a dye and a smooth
    field), VL2 + PLM + HLLD: one step on 6 windows of 16^3 inner cells against
    the oracle, every array at the 1e-12 bar; scalar mass conserved."""
    torch, dev = torch_dev
    n = 256
    b = inputs.with_scalars(inputs.turbulence(n=n, seed=1), 2, seed=71)
    kw = dict(integrator="vl2", recon="plm", riemann="hlld", cfl=0.3)
    s = athmhd.Solver(b.n, b.ng, b.dx, b.gamma, nscalars=2, **kw)
    tb = to_dev(torch, dev, b.bface)
    tc = s.prim2cons(to_dev(torch, dev, b.prim), tb)
    c0, b0 = tc.cpu().numpy(), tb.cpu().numpy()
    dt = s.newdt(tc, tb)
    s.step(tc, tb, dt)
    c1, b1 = tc.cpu().numpy(), tb.cpu().numpy()
    a = act(b)
    for v in (5, 6):
        m0, m1 = c0[v][a[1:]].sum(), c1[v][a[1:]].sum()
        assert abs(m1 - m0) <= 1e-12 * abs(m0)
    margin = 6
    m = 16 + 2 * margin
    rng = np.random.default_rng(72)
    origins = [tuple(int(x) for x in rng.integers(0, n, 3)) for _ in range(5)] + [(n - 9, n - 4, n - 11)]
    worst = 0.0
    for origin in origins:
        wc, wb = W.extract(c0, b0, b.ng, b.n, origin, m)
        wcfg = orc.make_cfg((m, m, m), b.ng, b.dx, b.gamma, nscalars=2, **kw)
        assert orc.step(wcfg, wc, wb, dt) == 0
        ref = W.inner_of_window(wc, wb, b.ng, m, margin)
        got = W.inner(c1, b1, b.ng, b.n, origin, m, margin)
        errs = W.rel_l1_arrays(got[0], got[1], ref[0], ref[1])
        print("window", origin, " ".join(f"{e:.1e}" for e in errs), flush=True)
        worst = max(worst, max(errs))
    assert worst <= TOL
    s.close()


@pytest.mark.parametrize("recon,integ", [("plm", "vl2"), ("ppm", "rk3")])
def test_the_maximum_number_of_scalars(torch_dev, athmhd, orc, recon, integ):
    """64 scalars, the largest count the library accepts, on a ragged block:
    two steps against the oracle, every array at the 1e-12 bar."""
    torch, dev = torch_dev
    ng = 3 if recon == "ppm" else 2
    ns = 64
    b = inputs.with_scalars(inputs.smooth_random(n=(20, 12, 10), seed=67, ng=ng), ns, seed=68)
    kw = dict(integrator=integ, recon=recon, riemann="hlld")
    s = athmhd.Solver(b.n, b.ng, b.dx, b.gamma, nscalars=ns, **kw)
    cfg = orc.cfg_for(b, nscalars=ns, **kw)
    cons = orc.prim2cons(cfg, b.prim, b.bface)
    tc, tb = to_dev(torch, dev, cons), to_dev(torch, dev, b.bface)
    rc, rb = cons.copy(), b.bface.copy()
    for _ in range(2):
        dt, bad = orc.newdt(cfg, rc, rb)
        assert bad == 0
        assert orc.step(cfg, rc, rb, dt) == 0
        s.step(tc, tb, dt)
    a = act(b)
    errs = rel_l1_each(tc.cpu().numpy()[a], rc[a]) + rel_l1_each(tb.cpu().numpy()[a], rb[a])
    print("worst rel L1 over", len(errs), "arrays", max(errs), flush=True)
    assert max(errs) <= TOL
    s.close()
