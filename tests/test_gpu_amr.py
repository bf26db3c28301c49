"""Level operators of block refinement on the GPU (Sec. 2.1.5):
athmhd_restrict and athmhd_prolong against the oracle, element by element.

Restriction and the cell and outer-face prolongation add the same values in
the same order on both sides, so they must agree bitwise; the faces inside
each coarse cell come from a closed form on the GPU and from a least-squares
solve of Toth & Roe's conditions in the oracle, so those agree to a tolerance
of 1e-14 of the field's scale (a few roundings of sums of 25 terms with
weights up to 1/2).  Every octant, several block shapes (ragged: unequal and
non-multiple-of-tile sizes, 2 and 3 ghosts, scalar rows), the entries that
must stay untouched, round trip and divergence properties on the device, a
128^3 block, prolongation in primitive variables (1e-13), the pressure floor
on refined cells (E within 1e-14 of the oracle, activations counted), and the
error paths.
"""
import gc
import itertools

import numpy as np
import pytest

from paper_2005_06651_amd import inputs

pytestmark = pytest.mark.gpu

OCTANTS = list(itertools.product((0, 1), repeat=3))
FACE_TOL = 1e-14


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


def shapes(n, ng):
    N = (n[2] + 2 * ng, n[1] + 2 * ng, n[0] + 2 * ng)
    return N, tuple(x + 1 for x in N)


def random_pair(N, F, nv, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((nv,) + N), rng.standard_normal((3,) + F)


def solver(athmhd, n, ng, ns=0, dx=0.1):
    return athmhd.Solver(n, ng, (dx, dx, dx), 5.0 / 3.0, nscalars=ns)


def dev(torch, d, x):
    return torch.from_numpy(np.ascontiguousarray(x)).to(d)


def active_faces(n, ng, d):
    e = [0, 0, 0]
    e[d] = 1
    return (slice(ng, ng + n[2] + e[2]), slice(ng, ng + n[1] + e[1]), slice(ng, ng + n[0] + e[0]))


def octant_mask_cells(N, n, ng, o):
    m = np.zeros(N, bool)
    h = [x // 2 for x in n]
    m[tuple(slice(ng + o[d] * h[d], ng + (o[d] + 1) * h[d]) for d in (2, 1, 0))] = True
    return m


def octant_mask_faces(F, n, ng, o, d):
    m = np.zeros(F, bool)
    h = [x // 2 for x in n]
    e = [0, 0, 0]
    e[d] = 1
    m[tuple(slice(ng + o[k] * h[k], ng + (o[k] + 1) * h[k] + e[k]) for k in (2, 1, 0))] = True
    return m


CASES = [((8, 6, 4), 2, 0), ((10, 14, 6), 3, 1), ((32, 24, 16), 2, 2)]


@pytest.mark.parametrize("n,ng,ns", CASES)
@pytest.mark.parametrize("o", OCTANTS)
def test_restrict_matches_the_oracle_bitwise(torch_dev, athmhd, orc, n, ng, ns, o):
    torch, d = torch_dev
    nv = 5 + ns
    N, F = shapes(n, ng)
    fc, fb = random_pair(N, F, nv, seed=21)
    cc, cb = random_pair(N, F, nv, seed=22)
    cfg = orc.make_cfg(n, ng, (0.1,) * 3, 5.0 / 3.0, nscalars=ns)
    want_c, want_b = cc.copy(), cb.copy()
    orc.restrict(cfg, fc, fb, want_c, want_b, tuple(o[k] * n[k] // 2 for k in range(3)))
    s = solver(athmhd, n, ng, ns)
    gc, gb = dev(torch, d, cc), dev(torch, d, cb)
    s.restrict(dev(torch, d, fc), dev(torch, d, fb), gc, gb, o)
    torch.cuda.synchronize()
    got_c, got_b = gc.cpu().numpy(), gb.cpu().numpy()
    assert np.array_equal(got_c, want_c)
    assert np.array_equal(got_b, want_b)
    # and only the octant changed
    m = octant_mask_cells(N, n, ng, o)
    assert np.array_equal(got_c[:, ~m], cc[:, ~m])
    for k in range(3):
        mf = octant_mask_faces(F, n, ng, o, k)
        assert np.array_equal(got_b[k][~mf], cb[k][~mf])


def check_prolong(got_c, got_b, want_c, want_b, fc0, fb0, n, ng):
    """Cells bitwise everywhere (ghosts untouched); faces: the outer ones
    (even offsets along their own direction) bitwise, interior ones within
    FACE_TOL of the field scale, ghost entries untouched."""
    assert np.array_equal(got_c, want_c)
    scale = np.abs(want_b).max()
    for k in range(3):
        a = active_faces(n, ng, k)
        g, w = got_b[k][a], want_b[k][a]
        idx = [slice(None)] * 3
        idx[2 - k] = slice(0, None, 2)          # outer faces: even fine index along k
        assert np.array_equal(g[tuple(idx)], w[tuple(idx)]), k
        assert np.abs(g - w).max() <= FACE_TOL * scale, (k, np.abs(g - w).max())
        mask = np.ones(got_b.shape[1:], bool)
        mask[a] = False
        assert np.array_equal(got_b[k][mask], fb0[k][mask])


@pytest.mark.parametrize("n,ng,ns", CASES)
@pytest.mark.parametrize("o", OCTANTS)
def test_prolong_matches_the_oracle(torch_dev, athmhd, orc, n, ng, ns, o):
    torch, d = torch_dev
    nv = 5 + ns
    N, F = shapes(n, ng)
    cc, cb = random_pair(N, F, nv, seed=31)
    fc0, fb0 = random_pair(N, F, nv, seed=32)
    cfg = orc.make_cfg(n, ng, (0.1,) * 3, 5.0 / 3.0, nscalars=ns)
    want_c, want_b = fc0.copy(), fb0.copy()
    orc.prolong(cfg, cc, cb, want_c, want_b, tuple(o[k] * n[k] // 2 for k in range(3)))
    s = solver(athmhd, n, ng, ns)
    gc, gb = dev(torch, d, fc0), dev(torch, d, fb0)
    s.prolong(dev(torch, d, cc), dev(torch, d, cb), gc, gb, o)
    torch.cuda.synchronize()
    check_prolong(gc.cpu().numpy(), gb.cpu().numpy(), want_c, want_b, fc0, fb0, n, ng)


def test_prolong_of_a_smooth_state_matches_the_oracle(torch_dev, athmhd, orc):
    """A physical state (divergence-free faces from a vector potential,
    conserved variables): the limiter takes both branches and zero slopes."""
    torch, d = torch_dev
    b = inputs.smooth_random(n=(16, 16, 16), seed=4, ng=2)
    cfg = orc.cfg_for(b)
    cc = orc.prim2cons(cfg, b.prim, b.bface)
    s = athmhd.Solver(b.n, b.ng, b.dx, b.gamma)
    for o in OCTANTS:
        want_c, want_b = np.zeros_like(cc), np.zeros_like(b.bface)
        orc.prolong(cfg, cc, b.bface, want_c, want_b, tuple(o[k] * 8 for k in range(3)))
        gc, gb = torch.zeros_like(dev(torch, d, cc)), torch.zeros_like(dev(torch, d, b.bface))
        s.prolong(dev(torch, d, cc), dev(torch, d, b.bface), gc, gb, o)
        torch.cuda.synchronize()
        check_prolong(gc.cpu().numpy(), gb.cpu().numpy(), want_c, want_b, want_c, want_b, b.n, b.ng)
        div = inputs.divb_metric(gb.cpu().numpy(), b.n, b.ng, tuple(x / 2 for x in b.dx))
        assert div <= 1e-12, div


def test_round_trip_on_the_device(torch_dev, athmhd):
    """restrict(prolong(U)) gives back the octant of U, to rounding."""
    torch, d = torch_dev
    n, ng = (24, 16, 12), 2
    N, F = shapes(n, ng)
    cc, cb = random_pair(N, F, 6, seed=41)
    s = solver(athmhd, n, ng, 1)
    gcc, gcb = dev(torch, d, cc), dev(torch, d, cb)
    for o in OCTANTS:
        fc, fb = torch.zeros_like(gcc), torch.zeros_like(gcb)
        back_c, back_b = torch.full_like(gcc, np.nan), torch.full_like(gcb, np.nan)
        s.prolong(gcc, gcb, fc, fb, o)
        s.restrict(fc, fb, back_c, back_b, o)
        torch.cuda.synchronize()
        m = octant_mask_cells(N, n, ng, o)
        bc = back_c.cpu().numpy()
        assert np.abs(bc[:, m] - cc[:, m]).max() <= 4e-15
        bb = back_b.cpu().numpy()
        for k in range(3):
            mf = octant_mask_faces(F, n, ng, o, k)
            assert np.abs(bb[k][mf] - cb[k][mf]).max() <= 4e-15


def test_large_block_prolong_and_restrict(torch_dev, athmhd, orc):
    """A 128^3 block (the size of one octant of the 256^3 domain): full
    comparison against the oracle for one octant of each operator."""
    torch, d = torch_dev
    n, ng = (128, 128, 128), 2
    N, F = shapes(n, ng)
    cc, cb = random_pair(N, F, 5, seed=51)
    cfg = orc.make_cfg(n, ng, (0.1,) * 3, 5.0 / 3.0)
    o = (1, 0, 1)
    org = tuple(o[k] * 64 for k in range(3))
    want_c, want_b = np.zeros_like(cc), np.zeros_like(cb)
    orc.prolong(cfg, cc, cb, want_c, want_b, org)
    s = solver(athmhd, n, ng)
    gc, gb = torch.zeros(cc.shape, dtype=torch.float64, device=d), torch.zeros(cb.shape, dtype=torch.float64, device=d)
    s.prolong(dev(torch, d, cc), dev(torch, d, cb), gc, gb, o)
    torch.cuda.synchronize()
    check_prolong(gc.cpu().numpy(), gb.cpu().numpy(), want_c, want_b, want_c, want_b, n, ng)
    rc, rb = cc.copy(), cb.copy()
    orc.restrict(cfg, want_c, want_b, rc, rb, org)
    g2c, g2b = dev(torch, d, cc), dev(torch, d, cb)
    s.restrict(gc, gb, g2c, g2b, o)
    torch.cuda.synchronize()
    # restriction of slightly different interior faces is not read: cells and
    # the coarse faces come from outer faces only, which agree bitwise
    assert np.array_equal(g2c.cpu().numpy(), rc)
    assert np.array_equal(g2b.cpu().numpy(), rb)


def test_level_operator_errors(torch_dev, athmhd):
    torch, d = torch_dev
    n, ng = (8, 8, 8), 2
    N, F = shapes(n, ng)
    a = [torch.zeros((5,) + N, dtype=torch.float64, device=d) for _ in range(2)]
    b = [torch.zeros((3,) + F, dtype=torch.float64, device=d) for _ in range(2)]
    s = solver(athmhd, n, ng)
    with pytest.raises(athmhd.AthmhdError) as e:
        s.prolong(a[0], b[0], a[1], b[1], (0, 2, 0))
    assert e.value.code == athmhd.EINVAL
    with pytest.raises(athmhd.AthmhdError) as e:
        s.restrict(a[0], b[0], a[0], b[1], (0, 0, 0))
    assert e.value.code == athmhd.EINVAL
    odd = athmhd.Solver((8, 7, 8), ng, (0.1,) * 3, 5.0 / 3.0)
    No, Fo = shapes((8, 7, 8), ng)
    ao = [torch.zeros((5,) + No, dtype=torch.float64, device=d) for _ in range(2)]
    bo = [torch.zeros((3,) + Fo, dtype=torch.float64, device=d) for _ in range(2)]
    with pytest.raises(athmhd.AthmhdError) as e:
        odd.restrict(ao[0], bo[0], ao[1], bo[1], (0, 0, 0))
    assert e.value.code == athmhd.EINVAL
    slab = athmhd.Solver(n, ng, (0.1, 0.2, 0.1), 5.0 / 3.0)
    with pytest.raises(athmhd.AthmhdError) as e:
        slab.prolong(a[0], b[0], a[1], b[1], (0, 0, 0))
    assert e.value.code == athmhd.EUNSUP
    slab.restrict(a[0], b[0], a[1], b[1], (0, 0, 0))   # restriction needs no cubic cells
    torch.cuda.synchronize()


def cold_block(N, F, seed, p0=1e-4, gamma=5.0 / 3.0):
    """rho near 1, momenta of order 1 from cell to cell, weak faces, pressure
    p0: prolonging E and M separately leaves some children below p0."""
    rng = np.random.default_rng(seed)
    cells = np.empty((5,) + N)
    cells[0] = 1.0 + 0.2 * rng.random(N)
    cells[1:4] = rng.standard_normal((3,) + N)
    faces = 0.05 * rng.standard_normal((3,) + F)
    b1 = 0.5 * (faces[0][:-1, :-1, :-1] + faces[0][:-1, :-1, 1:])
    b2 = 0.5 * (faces[1][:-1, :-1, :-1] + faces[1][:-1, 1:, :-1])
    b3 = 0.5 * (faces[2][:-1, :-1, :-1] + faces[2][1:, :-1, :-1])
    kin = 0.5 * (cells[1] ** 2 + cells[2] ** 2 + cells[3] ** 2) / cells[0]
    cells[4] = p0 / (gamma - 1.0) + kin + 0.5 * (b1 ** 2 + b2 ** 2 + b3 ** 2)
    return cells, faces


def fine_pressure(cells, faces, n, ng, gamma=5.0 / 3.0):
    a = (slice(ng, ng + n[2]), slice(ng, ng + n[1]), slice(ng, ng + n[0]))
    b1 = faces[0][a[0], a[1], ng:ng + n[0] + 1]
    b2 = faces[1][a[0], ng:ng + n[1] + 1, a[2]]
    b3 = faces[2][ng:ng + n[2] + 1, a[1], a[2]]
    mag = 0.5 * ((0.5 * (b1[..., :-1] + b1[..., 1:])) ** 2 + (0.5 * (b2[:, :-1] + b2[:, 1:])) ** 2
                 + (0.5 * (b3[:-1] + b3[1:])) ** 2)
    kin = 0.5 * (cells[1][a] ** 2 + cells[2][a] ** 2 + cells[3][a] ** 2) / cells[0][a]
    return (gamma - 1.0) * (cells[4][a] - kin - mag)


@pytest.mark.parametrize("o", [(0, 0, 0), (1, 0, 1), (1, 1, 1)])
def test_prolong_with_a_pressure_floor_matches_the_oracle(torch_dev, athmhd, orc, o):
    """Refined cells below the handle's pressure floor get E raised: rho, M
    and the faces bitwise as without the floor, E within 1e-14 of the oracle,
    and one counted activation per floored cell."""
    torch, d = torch_dev
    n, ng, pf = (16, 12, 10), 2, 1e-5
    N, F = shapes(n, ng)
    cc, cb = cold_block(N, F, seed=71)
    org = tuple(o[k] * n[k] // 2 for k in range(3))
    cfg0 = orc.make_cfg(n, ng, (0.1,) * 3, 5.0 / 3.0)
    cfg1 = orc.make_cfg(n, ng, (0.1,) * 3, 5.0 / 3.0, pfloor=pf)
    c0, b0 = np.zeros_like(cc), np.zeros_like(cb)
    orc.prolong(cfg0, cc, cb, c0, b0, org)
    want_c, want_b = np.zeros_like(cc), np.zeros_like(cb)
    orc.prolong(cfg1, cc, cb, want_c, want_b, org)
    expected = int((fine_pressure(c0, b0, n, ng) < pf).sum())
    assert expected >= 3
    s = solver(athmhd, n, ng)
    s.set_floors(0.0, pf)
    assert s.floor_count() == 0
    gc, gb = torch.zeros(cc.shape, dtype=torch.float64, device=d), torch.zeros(cb.shape, dtype=torch.float64, device=d)
    s.prolong(dev(torch, d, cc), dev(torch, d, cb), gc, gb, o)
    got_c, got_b = gc.cpu().numpy(), gb.cpu().numpy()
    assert s.floor_count() == expected
    assert np.array_equal(got_c[:4], want_c[:4])
    assert np.abs(got_c[4] - want_c[4]).max() <= 1e-14 * np.abs(want_c[4]).max()
    check_prolong(got_c[:4], got_b, want_c[:4], want_b, want_c[:4], want_b, n, ng)
    assert fine_pressure(got_c, got_b, n, ng).min() >= pf * (1 - 1e-9)


PRIM_TOL = 1e-13


@pytest.mark.parametrize("n,ng,ns", [((10, 14, 6), 3, 1), ((32, 24, 16), 2, 2), ((16, 16, 16), 2, 0)])
@pytest.mark.parametrize("o", [(0, 0, 0), (1, 0, 0), (0, 1, 1), (1, 1, 1)])
def test_primitive_prolong_matches_the_oracle(torch_dev, athmhd, orc, n, ng, ns, o):
    """Prolongation in primitive variables of a smooth physical state with
    scalars: rho and the faces as in the bitwise cases, every other array
    within 1e-13 of its scale (divisions and the pressure formula round
    differently with FMA contraction)."""
    torch, d = torch_dev
    b = inputs.smooth_random(n=n, seed=9, ng=ng)
    if ns:
        b = inputs.with_scalars(b, ns, seed=19)
    cfg = orc.cfg_for(b, nscalars=ns)
    cc = orc.prim2cons(cfg, b.prim, b.bface)
    org = tuple(o[k] * n[k] // 2 for k in range(3))
    want_c, want_b = np.zeros_like(cc), np.zeros_like(b.bface)
    orc.prolong(cfg, cc, b.bface, want_c, want_b, org, primitive=True)
    s = athmhd.Solver(b.n, b.ng, (0.1,) * 3, b.gamma, nscalars=ns)   # the operators do not read dx
    gc = torch.zeros(cc.shape, dtype=torch.float64, device=d)
    gb = torch.zeros(b.bface.shape, dtype=torch.float64, device=d)
    s.prolong(dev(torch, d, cc), dev(torch, d, b.bface), gc, gb, o, primitive=True)
    got_c, got_b = gc.cpu().numpy(), gb.cpu().numpy()
    assert np.array_equal(got_c[0], want_c[0])
    for v in range(1, cc.shape[0]):
        err = np.abs(got_c[v] - want_c[v]).max() / np.abs(want_c[v]).max()
        assert err <= PRIM_TOL, (v, err)
    check_prolong(got_c[:1], got_b, want_c[:1], want_b, want_c[:1], want_b, n, ng)


def test_primitive_prolong_of_a_cold_state(torch_dev, athmhd, orc):
    """The cold state that conserved prolongation drives negative: positive
    pressure everywhere, and parity with the oracle; the floor counter stays
    at zero with a floor set (primitive prolongation applies none)."""
    torch, d = torch_dev
    n, ng = (16, 12, 10), 2
    N, F = shapes(n, ng)
    cc, cb = cold_block(N, F, seed=73)
    cfg = orc.make_cfg(n, ng, (0.1,) * 3, 5.0 / 3.0)
    s = solver(athmhd, n, ng)
    s.set_floors(0.0, 1e-5)
    s.floor_count()
    for o in [(0, 0, 0), (1, 1, 0)]:
        org = tuple(o[k] * n[k] // 2 for k in range(3))
        want_c, want_b = np.zeros_like(cc), np.zeros_like(cb)
        orc.prolong(cfg, cc, cb, want_c, want_b, org, primitive=True)
        gc = torch.zeros(cc.shape, dtype=torch.float64, device=d)
        gb = torch.zeros(cb.shape, dtype=torch.float64, device=d)
        s.prolong(dev(torch, d, cc), dev(torch, d, cb), gc, gb, o, primitive=True)
        got_c, got_b = gc.cpu().numpy(), gb.cpu().numpy()
        assert fine_pressure(got_c, got_b, n, ng).min() > 0
        for v in range(5):
            err = np.abs(got_c[v] - want_c[v]).max() / np.abs(want_c[v]).max()
            assert err <= PRIM_TOL, (v, err)
    assert s.floor_count() == 0


def test_primitive_flag_is_checked(torch_dev, athmhd):
    torch, d = torch_dev
    import ctypes
    n, ng = (8, 8, 8), 2
    N, F = shapes(n, ng)
    a = [torch.zeros((5,) + N, dtype=torch.float64, device=d) for _ in range(2)]
    b = [torch.zeros((3,) + F, dtype=torch.float64, device=d) for _ in range(2)]
    s = solver(athmhd, n, ng)
    p = [ctypes.c_void_p(x.data_ptr()) for x in (a[0], b[0], a[1], b[1])]
    rc = athmhd.lib().athmhd_prolong(s._h, *p, 0, 0, 0, 2, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == athmhd.EINVAL


def test_level_operators_with_the_maximum_number_of_scalars(torch_dev, athmhd, orc):
    """64 scalar rows: restriction and conserved prolongation bitwise, and
    primitive prolongation within 1e-13, against the oracle."""
    torch, d = torch_dev
    n, ng, ns = (8, 6, 4), 2, 64
    b = inputs.with_scalars(inputs.smooth_random(n=n, seed=81, ng=ng), ns, seed=82)
    cfg = orc.cfg_for(b, nscalars=ns)
    cc = orc.prim2cons(cfg, b.prim, b.bface)
    s = athmhd.Solver(b.n, b.ng, (0.1,) * 3, b.gamma, nscalars=ns)
    o = (1, 0, 1)
    org = tuple(o[k] * n[k] // 2 for k in range(3))
    for primitive in (False, True):
        want_c, want_b = np.zeros_like(cc), np.zeros_like(b.bface)
        orc.prolong(cfg, cc, b.bface, want_c, want_b, org, primitive=primitive)
        gc = torch.zeros(cc.shape, dtype=torch.float64, device=d)
        gb = torch.zeros(b.bface.shape, dtype=torch.float64, device=d)
        s.prolong(dev(torch, d, cc), dev(torch, d, b.bface), gc, gb, o, primitive=primitive)
        got_c, got_b = gc.cpu().numpy(), gb.cpu().numpy()
        if primitive:
            assert np.array_equal(got_c[0], want_c[0])
            for v in range(1, cc.shape[0]):
                assert np.abs(got_c[v] - want_c[v]).max() <= PRIM_TOL * np.abs(want_c[v]).max(), v
            check_prolong(got_c[:1], got_b, want_c[:1], want_b, want_c[:1], want_b, n, ng)
        else:
            check_prolong(got_c, got_b, want_c, want_b, want_c, want_b, n, ng)
    rc, rb = cc.copy(), b.bface.copy()
    orc.restrict(cfg, want_c, want_b, rc, rb, org)
    g2c, g2b = dev(torch, d, cc), dev(torch, d, b.bface)
    s.restrict(dev(torch, d, want_c), dev(torch, d, want_b), g2c, g2b, o)
    assert np.array_equal(g2c.cpu().numpy(), rc) and np.array_equal(g2b.cpu().numpy(), rb)


# ---- boxes (coarse buffers and ghost zones between levels)

def box_face_slices(flo, ext, d, extra):
    e = [0, 0, 0]
    e[d] = 1
    return tuple(slice(flo[k], flo[k] + extra * ext[k] + e[k]) for k in (2, 1, 0))


def check_box(got_c, got_b, want_c, want_b, init_b, flo, ext, fine, bitwise_faces):
    """Cells bitwise (every entry: outside the box both sides are the initial
    values); faces inside the box bitwise on the outer ones (or all, for
    restriction) and within FACE_TOL elsewhere, outside the box untouched."""
    assert np.array_equal(got_c, want_c)
    scale = np.abs(want_b).max()
    for d in range(3):
        sf = box_face_slices(flo, ext, d, 2 if fine else 1)
        m = np.zeros(got_b.shape[1:], bool)
        m[sf] = True
        assert np.array_equal(got_b[d][~m], init_b[d][~m]), d
        g, w = got_b[d][sf], want_b[d][sf]
        if bitwise_faces:
            assert np.array_equal(g, w), d
        else:
            idx = [slice(None)] * 3
            idx[2 - d] = slice(0, None, 2)
            assert np.array_equal(g[tuple(idx)], w[tuple(idx)]), d
            assert np.abs(g - w).max() <= FACE_TOL * scale, d


N_BOX, NG_BOX = (12, 10, 8), 4
RESTRICT_BOXES = [((12, 4, 4), (16, 5, 4), (2, 5, 4)),     # fine boundary layer -> coarse upper x1 ghosts
                  ((0, 0, 0), (0, 0, 0), (2, 2, 2)),       # ghost corner onto ghost corner
                  ((1, 3, 2), (5, 2, 3), (3, 2, 2)),       # odd offsets
                  ((4, 4, 4), (18, 16, 14), (2, 2, 2))]    # coarse box ending at the last stored cell
PROLONG_BOXES = [((0, 4, 4), (5, 3, 6), (2, 4, 3)),        # coarse cells -> fine lower x1 ghosts
                 ((16, 0, 2), (3, 4, 2), (2, 3, 3)),       # fine upper x1 ghosts, ghost rows
                 ((1, 3, 2), (1, 1, 1), (3, 2, 2)),        # coarse box from the first readable cell
                 ((4, 4, 4), (16, 14, 12), (3, 3, 3))]     # coarse box ending at N - 1


@pytest.mark.parametrize("box", RESTRICT_BOXES)
def test_restrict_box_matches_the_oracle(torch_dev, athmhd, orc, box):
    torch, d = torch_dev
    n, ng, ns = N_BOX, NG_BOX, 1
    N, F = shapes(n, ng)
    fc, fb = random_pair(N, F, 6, seed=101)
    cc, cb = random_pair(N, F, 6, seed=102)
    cfg = orc.make_cfg(n, ng, (0.1,) * 3, 5.0 / 3.0, nscalars=ns)
    want_c, want_b = cc.copy(), cb.copy()
    orc.restrict_box(cfg, fc, fb, want_c, want_b, *box)
    s = solver(athmhd, n, ng, ns)
    gc, gb = dev(torch, d, cc), dev(torch, d, cb)
    s.restrict_box(dev(torch, d, fc), dev(torch, d, fb), gc, gb, *box)
    check_box(gc.cpu().numpy(), gb.cpu().numpy(), want_c, want_b, cb, box[1], box[2], fine=False,
              bitwise_faces=True)


@pytest.mark.parametrize("primitive", [False, True])
@pytest.mark.parametrize("box", PROLONG_BOXES)
def test_prolong_box_matches_the_oracle(torch_dev, athmhd, orc, box, primitive):
    torch, d = torch_dev
    n, ng, ns = N_BOX, NG_BOX, 1
    N, F = shapes(n, ng)
    if primitive:      # a physical state: positive density and pressure everywhere, ghosts included
        b = inputs.with_scalars(inputs.smooth_random(n=n, seed=103, ng=ng), ns, seed=104)
        cfg = orc.make_cfg(n, ng, (0.1,) * 3, b.gamma, nscalars=ns)
        cc, cb = orc.prim2cons(cfg, b.prim, b.bface), b.bface
    else:
        cc, cb = random_pair(N, F, 6, seed=105)
        cfg = orc.make_cfg(n, ng, (0.1,) * 3, 5.0 / 3.0, nscalars=ns)
    fc0, fb0 = random_pair(N, F, 6, seed=106)
    want_c, want_b = fc0.copy(), fb0.copy()
    orc.prolong_box(cfg, cc, cb, want_c, want_b, *box, primitive=primitive)
    s = solver(athmhd, n, ng, ns)
    gc, gb = dev(torch, d, fc0), dev(torch, d, fb0)
    s.prolong_box(dev(torch, d, cc), dev(torch, d, cb), gc, gb, *box, primitive=primitive)
    got_c, got_b = gc.cpu().numpy(), gb.cpu().numpy()
    if primitive:
        sc = tuple(slice(box[0][k], box[0][k] + 2 * box[2][k]) for k in (2, 1, 0))
        mask = np.zeros(N, bool)
        mask[sc] = True
        assert np.array_equal(got_c[:, ~mask], fc0[:, ~mask])
        assert np.array_equal(got_c[0], want_c[0])
        for v in range(1, 6):
            assert np.abs(got_c[v] - want_c[v]).max() <= PRIM_TOL * np.abs(want_c[v][mask]).max(), v
        check_box(got_c[:1], got_b, want_c[:1], want_b, fb0, box[0], box[2], fine=True, bitwise_faces=False)
    else:
        check_box(got_c, got_b, want_c, want_b, fb0, box[0], box[2], fine=True, bitwise_faces=False)


def test_box_bounds_are_checked(torch_dev, athmhd):
    """Boxes reaching outside the stored arrays are refused before any launch."""
    torch, d = torch_dev
    n, ng = N_BOX, NG_BOX
    N, F = shapes(n, ng)
    Nx = N[::-1]                                    # stored cells along (x1, x2, x3)
    a = [torch.zeros((5,) + N, dtype=torch.float64, device=d) for _ in range(2)]
    b = [torch.zeros((3,) + F, dtype=torch.float64, device=d) for _ in range(2)]
    s = solver(athmhd, n, ng)
    bad_restrict = [((0, 0, 0), (0, 0, 0), (0, 1, 1)),                       # empty extent
                    ((Nx[0] - 3, 0, 0), (0, 0, 0), (2, 1, 1)),              # fine box past the end
                    ((-1, 0, 0), (0, 0, 0), (1, 1, 1)),                     # negative start
                    ((0, 0, 0), (Nx[0] - 1, 0, 0), (2, 1, 1))]              # coarse box past the end
    for box in bad_restrict:
        with pytest.raises(athmhd.AthmhdError) as e:
            s.restrict_box(a[0], b[0], a[1], b[1], *box)
        assert e.value.code == athmhd.EINVAL, box
    bad_prolong = [((0, 0, 0), (0, 1, 1), (1, 1, 1)),                       # no lower neighbour
                   ((0, 0, 0), (1, 1, Nx[2] - 1), (1, 1, 1)),               # no upper neighbour
                   ((0, 0, Nx[2] - 1), (1, 1, 1), (1, 1, 1))]               # fine box past the end
    for box in bad_prolong:
        with pytest.raises(athmhd.AthmhdError) as e:
            s.prolong_box(a[0], b[0], a[1], b[1], *box)
        assert e.value.code == athmhd.EINVAL, box
    # the largest boxes allowed run
    s.restrict_box(a[0], b[0], a[1], b[1], (0, 0, 0), (Nx[0] // 2, Nx[1] // 2, Nx[2] // 2),
                   (Nx[0] // 2, Nx[1] // 2, Nx[2] // 2))
    s.prolong_box(a[0], b[0], a[1], b[1], (0, 0, 0), (1, 1, 1), (Nx[0] // 2 - 1, Nx[1] // 2 - 1, Nx[2] // 2 - 1))
    torch.cuda.synchronize()


def curl_faces(N, seed):
    """A face field with zero discrete divergence (curl of an edge potential)."""
    rng = np.random.default_rng(seed)
    ax, ay, az = rng.standard_normal((3,) + tuple(m + 2 for m in N))
    s = slice(0, -1)
    bx = (az[s, 1:, s] - az[s, s, s]) - (ay[1:, s, s] - ay[s, s, s])
    by = (ax[1:, s, s] - ax[s, s, s]) - (az[s, s, 1:] - az[s, s, s])
    bz = (ay[s, s, 1:] - ay[s, s, s]) - (ax[s, 1:, s] - ax[s, s, s])
    return np.ascontiguousarray(np.stack([bx, by, bz]))


@pytest.mark.parametrize("keep", [63, 5, 42, 16])
@pytest.mark.parametrize("box", [PROLONG_BOXES[0], ((4, 4, 4), (4, 4, 4), (6, 5, 4))])
def test_prolong_box_with_kept_faces_matches_the_oracle(torch_dev, athmhd, orc, box, keep):
    """Kept sides are read, not written (bitwise the initial fine values on
    both sides), and the interior faces are solved with them."""
    torch, d = torch_dev
    n, ng = N_BOX, NG_BOX
    N, F = shapes(n, ng)
    cc, cb = random_pair(N, F, 5, seed=121)
    fc0, fb0 = random_pair(N, F, 5, seed=122)
    cfg = orc.make_cfg(n, ng, (0.1,) * 3, 5.0 / 3.0)
    want_c, want_b = fc0.copy(), fb0.copy()
    orc.prolong_box(cfg, cc, cb, want_c, want_b, *box, keep=keep)
    s = solver(athmhd, n, ng)
    gc, gb = dev(torch, d, fc0), dev(torch, d, fb0)
    s.prolong_box(dev(torch, d, cc), dev(torch, d, cb), gc, gb, *box, keep=keep)
    check_box(gc.cpu().numpy(), gb.cpu().numpy(), want_c, want_b, fb0, box[0], box[2], fine=True,
              bitwise_faces=False)


def test_kept_faces_keep_a_divergence_free_field_on_the_device(torch_dev, athmhd, orc):
    """A divergence-free fine field restricted onto its parent octant and
    prolonged back with its 6 sides kept stays divergence-free."""
    torch, d = torch_dev
    n, ng = (16, 12, 8), 2
    N, F = shapes(n, ng)
    fb_true = curl_faces(N, seed=123)
    cc, cb = random_pair(N, F, 5, seed=124)
    s = solver(athmhd, n, ng)
    gcc, gcb = dev(torch, d, cc), dev(torch, d, cb)
    s.restrict(torch.zeros_like(gcc), dev(torch, d, fb_true), gcc, gcb, (1, 0, 1))
    box = ((ng,) * 3, (ng + 8, ng, ng + 4), (8, 6, 4))
    gf = dev(torch, d, fb_true)
    s.prolong_box(gcc, gcb, torch.zeros_like(gcc), gf, *box, keep=63)
    got = gf.cpu().numpy()
    div = inputs.divb_metric(got, n, ng, (1.0, 1.0, 1.0))
    assert div <= 1e-13, div
    for k in range(3):       # the 6 sides are the original values
        e = [slice(ng, ng + n[2]), slice(ng, ng + n[1]), slice(ng, ng + n[0])]
        for side in (ng, ng + n[k]):
            sl = list(e)
            sl[2 - k] = side
            assert np.array_equal(got[k][tuple(sl)], fb_true[k][tuple(sl)])


def test_keep_mask_is_checked(torch_dev, athmhd):
    torch, d = torch_dev
    n, ng = N_BOX, NG_BOX
    N, F = shapes(n, ng)
    a = [torch.zeros((5,) + N, dtype=torch.float64, device=d) for _ in range(2)]
    b = [torch.zeros((3,) + F, dtype=torch.float64, device=d) for _ in range(2)]
    s = solver(athmhd, n, ng)
    for keep in (64, -1):
        with pytest.raises(athmhd.AthmhdError) as e:
            s.prolong_box(a[0], b[0], a[1], b[1], (4, 4, 4), (4, 4, 4), (2, 2, 2), keep=keep)
        assert e.value.code == athmhd.EINVAL


def test_level_operators_replay_from_a_graph(torch_dev, athmhd):
    """The level operators allocate nothing and record no memset, so a
    refinement (8 octant prolongations) and a derefinement (8 restrictions)
    can be captured once in a graph: three replays, with eager updates of the
    input between them, each bitwise equal to eager calls on the same data."""
    torch, d = torch_dev
    n, ng = (16, 12, 8), 2
    N, F = shapes(n, ng)
    cc0, cb0 = random_pair(N, F, 5, seed=131)
    cc, cb = dev(torch, d, cc0), dev(torch, d, cb0)
    fcs = [torch.zeros_like(cc) for _ in range(8)]
    fbs = [torch.zeros_like(cb) for _ in range(8)]
    rc, rb = torch.zeros_like(cc), torch.zeros_like(cb)
    s = solver(athmhd, n, ng)

    def refine_and_back():
        for i, o in enumerate(OCTANTS):
            s.prolong(cc, cb, fcs[i], fbs[i], o)
        for i, o in enumerate(OCTANTS):
            s.restrict(fcs[i], fbs[i], rc, rb, o)

    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        refine_and_back()
    torch.cuda.current_stream().wait_stream(side)
    torch.cuda.synchronize()
    # capture in thread-local mode after a collection: a tensor of an earlier
    # test freed by the garbage collector during a global-mode capture can
    # invalidate the capture from outside these calls
    gc.collect()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph, capture_error_mode="thread_local"):
        refine_and_back()
    torch.cuda.synchronize()
    for rep in range(3):
        cc.mul_(1.0 + 0.1 * rep)
        cb.add_(0.05)
        torch.cuda.synchronize()
        graph.replay()
        torch.cuda.synchronize()
        got = [x.clone() for x in fcs + fbs] + [rc.clone(), rb.clone()]
        refine_and_back()
        torch.cuda.synchronize()
        want = fcs + fbs + [rc, rb]
        assert all(torch.equal(a, b) for a, b in zip(got, want)), rep
