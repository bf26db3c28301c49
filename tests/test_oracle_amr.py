"""Pins of the oracle's level operators for block refinement (Sec. 2.1.5):
restriction (volume averages of cells, area averages of faces) and
prolongation (minmod-limited linear cells; faces split on the coarse faces by
the 2D minmod profile, the interior faces from Toth & Roe's divergence and
curl conditions).

None of these re-types the operators.  They check what the definitions and the
mathematics fix:
  * restriction after prolongation is the identity (the children's offsets
    cancel in the average, for cells and for the 4 faces of each coarse face);
  * a linear cell field is prolonged to the exact fine averages, and restriction
    of a linear fine field gives the exact coarse averages;
  * a cell at a local extremum has flat children (minmod);
  * any linear face field with zero divergence, whatever its curl, is prolonged
    to the exact fine face averages, interior faces included (the field then
    satisfies every condition, and the conditions have one solution);
  * every fine cell has its parent's divergence, for arbitrary face data;
    restricted faces have the mean divergence of the children;
  * the operators commute with mirroring an axis and with cycling the axes
    (a wrong weighting of the two outer planes in the curl estimate, or a
    transposed index, breaks one of them);
  * only the named octant of the coarse block is written by restriction;
  * with a pressure floor, every refined cell ends at or above it, and only E
    of the cells below it changes (mass, momentum and faces bitwise as
    without the floor).
"""
import itertools

import numpy as np
import pytest

OCTANTS = list(itertools.product((0, 1), repeat=3))


def geom(orc, n=(8, 6, 4), ng=2, ns=0):
    cfg = orc.make_cfg(n, ng, (0.1, 0.1, 0.1), 5.0 / 3.0, nscalars=ns)
    N = (n[2] + 2 * ng, n[1] + 2 * ng, n[0] + 2 * ng)
    return cfg, N


def random_block(N, nv, seed):
    rng = np.random.default_rng(seed)
    return rng.standard_normal((nv,) + N), rng.standard_normal((3,) + tuple(x + 1 for x in N))


def oct_origin(n, o):
    return tuple(o[d] * n[d] // 2 for d in range(3))


def prolong(orc, cfg, cc, cb, o):
    fc, fb = np.zeros_like(cc), np.zeros_like(cb)
    orc.prolong(cfg, cc, cb, fc, fb, o)
    return fc, fb


def divergence(bf, ng, n, h):
    """Flux divergence of every active cell of a face field (unit-free h)."""
    a = bf[0][ng:ng + n[2], ng:ng + n[1], ng:ng + n[0] + 1]
    b = bf[1][ng:ng + n[2], ng:ng + n[1] + 1, ng:ng + n[0]]
    c = bf[2][ng:ng + n[2] + 1, ng:ng + n[1], ng:ng + n[0]]
    return (np.diff(a, axis=2) + np.diff(b, axis=1) + np.diff(c, axis=0)) / h


def octant_slices(n, ng, o, extra=(0, 0, 0)):
    """(k, j, i) slices of octant o of the coarse block, with `extra` entries
    appended along (x, y, z)."""
    h = [n[d] // 2 for d in range(3)]
    s = [slice(ng + o[d] * h[d], ng + o[d] * h[d] + h[d] + extra[d]) for d in range(3)]
    return (s[2], s[1], s[0])


@pytest.mark.parametrize("o", OCTANTS)
def test_restriction_undoes_prolongation(orc, o):
    n = (8, 6, 4)
    cfg, N = geom(orc, n, ns=1)
    cc, cb = random_block(N, 6, seed=11)
    org = oct_origin(n, o)
    fc, fb = prolong(orc, cfg, cc, cb, org)
    rc, rb = np.full_like(cc, np.nan), np.full_like(cb, np.nan)
    orc.restrict(cfg, fc, fb, rc, rb, org)
    s = octant_slices(n, 2, o)
    assert np.abs(rc[(slice(None),) + s] - cc[(slice(None),) + s]).max() <= 4e-15
    for d in range(3):
        e = [0, 0, 0]
        e[d] = 1
        sf = octant_slices(n, 2, o, e)
        assert np.abs(rb[d][sf] - cb[d][sf]).max() <= 4e-15, d


def test_restriction_writes_only_its_octant(orc):
    n = (8, 6, 4)
    cfg, N = geom(orc, n)
    fc, fb = random_block(N, 5, seed=2)
    rc, rb = np.full((5,) + N, 7.0), np.full((3,) + tuple(x + 1 for x in N), 7.0)
    o = (1, 0, 1)
    orc.restrict(cfg, fc, fb, rc, rb, oct_origin(n, o))
    mask = np.zeros(N, bool)
    mask[octant_slices(n, 2, o)] = True
    assert np.all(rc[:, ~mask] == 7.0) and not np.any(rc[:, mask] == 7.0)
    for d in range(3):
        e = [0, 0, 0]
        e[d] = 1
        m = np.zeros(rb.shape[1:], bool)
        m[octant_slices(n, 2, o, e)] = True
        assert np.all(rb[d][~m] == 7.0) and not np.any(rb[d][m] == 7.0)


def cell_centres(N, ng, h):
    z, y, x = np.meshgrid(*[(np.arange(m) - ng + 0.5) * h for m in N], indexing="ij")
    return x, y, z


@pytest.mark.parametrize("o", OCTANTS)
def test_linear_cells_prolong_exactly(orc, o):
    """U = a + b.x: cell averages are centre values; both minmod arguments are
    the same slope, so the children get U at their own centres."""
    n = (8, 6, 4)
    cfg, N = geom(orc, n)
    coef = np.array([[0.3, 1.5, -2.0, 0.7], [-1.0, 0.2, 0.9, -0.4], [2.0, -0.3, 0.0, 1.1], [0.5, 0.0, 0.0, 0.0],
                     [1.0, 3.0, 2.0, 1.0]])
    xc, yc, zc = cell_centres(N, 2, 1.0)           # coarse spacing 1
    cc = np.stack([c[0] + c[1] * xc + c[2] * yc + c[3] * zc for c in coef])
    _, cb = random_block(N, 5, seed=1)
    org = oct_origin(n, o)
    fc, _ = prolong(orc, cfg, cc, cb, org)
    xf, yf, zf = cell_centres(N, 2, 0.5)           # fine spacing 1/2 ...
    off = [org[d] for d in range(3)]               # ... starting at the octant's corner
    want = np.stack([c[0] + c[1] * (xf + off[0]) + c[2] * (yf + off[1]) + c[3] * (zf + off[2]) for c in coef])
    a = (slice(None), slice(2, 2 + n[2]), slice(2, 2 + n[1]), slice(2, 2 + n[0]))
    assert np.abs(fc[a] - want[a]).max() <= 1e-13


def test_extremum_cell_has_flat_children(orc):
    n = (8, 8, 8)
    cfg, N = geom(orc, n)
    cc = np.zeros((5,) + N)
    cc[:, 4, 4, 4] = 1.0      # a peak in every variable, inside octant (0, 0, 0)
    cc[:, 5, 4, 4] = 0.5      # one side rising, the other falling in z: minmod is 0
    _, cb = random_block(N, 5, seed=1)
    fc, _ = prolong(orc, cfg, cc, cb, (0, 0, 0))
    # coarse cell (4, 4, 4) is active cell (2, 2, 2): fine cells 4..5 + ng
    kids = fc[:, 6:8, 6:8, 6:8]
    assert np.all(kids == 1.0)


def linear_faces(N, ng, h, M, b0, shift=(0, 0, 0)):
    """Face averages of the linear field B = b0 + M x (trace M = 0), with x
    measured from the block's first active corner plus `shift`."""
    F = tuple(m + 1 for m in N)
    out = np.empty((3,) + F)
    for d in range(3):
        idx = np.meshgrid(*[np.arange(m) for m in F], indexing="ij")   # (k, j, i)
        x = [(idx[2] - ng) * h, (idx[1] - ng) * h, (idx[0] - ng) * h]
        x = [x[e] + (0.0 if e == d else 0.5 * h) + shift[e] for e in range(3)]   # face centres
        out[d] = b0[d] + M[d][0] * x[0] + M[d][1] * x[1] + M[d][2] * x[2]
    return out


@pytest.mark.parametrize("o", OCTANTS)
def test_divergence_free_linear_field_prolongs_exactly(orc, o):
    n = (8, 6, 4)
    cfg, N = geom(orc, n)
    M = np.array([[0.7, -1.3, 0.4], [2.1, -0.2, 0.9], [-0.6, 1.7, -0.5]])   # curl != 0, trace 0
    b0 = np.array([0.3, -0.8, 1.2])
    cb = linear_faces(N, 2, 1.0, M, b0)
    cc, _ = random_block(N, 5, seed=4)
    org = oct_origin(n, o)
    _, fb = prolong(orc, cfg, cc, cb, org)
    want = linear_faces(N, 2, 0.5, M, b0, shift=org)
    for d in range(3):
        e = [0, 0, 0]
        e[d] = 1
        s = (slice(2, 2 + n[2] + e[2]), slice(2, 2 + n[1] + e[1]), slice(2, 2 + n[0] + e[0]))
        assert np.abs(fb[d][s] - want[d][s]).max() <= 2e-14, d


@pytest.mark.parametrize("o", OCTANTS[::3])
def test_fine_cells_keep_the_parent_divergence(orc, o):
    n = (8, 6, 4)
    cfg, N = geom(orc, n)
    cc, cb = random_block(N, 5, seed=8)     # arbitrary faces: nonzero divergence
    org = oct_origin(n, o)
    _, fb = prolong(orc, cfg, cc, cb, org)
    df = divergence(fb, 2, n, 0.5)
    dc = divergence(cb, 2, n, 1.0)
    h = [n[d] // 2 for d in range(3)]
    parent = dc[org[2]:org[2] + h[2], org[1]:org[1] + h[1], org[0]:org[0] + h[0]]
    want = np.repeat(np.repeat(np.repeat(parent, 2, 0), 2, 1), 2, 2)
    assert np.abs(df - want).max() <= 1e-13 * np.abs(dc).max()


def test_divergence_free_smooth_field_stays_divergence_free(orc):
    from paper_2005_06651_amd import inputs
    b = inputs.smooth_random(n=(8, 8, 8), seed=6, ng=2)
    cfg = orc.cfg_for(b)
    cc = orc.prim2cons(cfg, b.prim, b.bface)
    scale = np.abs(b.bface).max() / b.dx[0]
    for o in OCTANTS:
        _, fb = prolong(orc, cfg, cc, b.bface, oct_origin(b.n, o))
        assert np.abs(divergence(fb, 2, b.n, b.dx[0] / 2)).max() <= 1e-12 * scale


def test_restricted_faces_carry_the_mean_child_divergence(orc):
    n = (8, 6, 4)
    cfg, N = geom(orc, n)
    fc, fb = random_block(N, 5, seed=9)
    cc, cb = random_block(N, 5, seed=10)
    o = (1, 1, 0)
    org = oct_origin(n, o)
    orc.restrict(cfg, fc, fb, cc, cb, org)
    df = divergence(fb, 2, n, 0.5)
    mean = df.reshape(n[2] // 2, 2, n[1] // 2, 2, n[0] // 2, 2).mean(axis=(1, 3, 5))
    h = [n[d] // 2 for d in range(3)]
    dc = divergence(cb, 2, n, 1.0)[org[2]:org[2] + h[2], org[1]:org[1] + h[1], org[0]:org[0] + h[0]]
    assert np.abs(dc - mean).max() <= 1e-13 * np.abs(mean).max()


def test_linear_fine_field_restricts_exactly(orc):
    n = (8, 8, 8)
    cfg, N = geom(orc, n)
    M = np.array([[0.7, -1.3, 0.4], [2.1, -0.2, 0.9], [-0.6, 1.7, -0.5]])
    b0 = np.array([0.3, -0.8, 1.2])
    o = (0, 1, 1)
    org = oct_origin(n, o)
    fb = linear_faces(N, 2, 0.5, M, b0, shift=org)
    xf, yf, zf = cell_centres(N, 2, 0.5)
    fc = np.stack([1.0 + 0.5 * (xf + org[0]) - 2.0 * (yf + org[1]) + 0.25 * (zf + org[2])] * 5)
    cc, cb = np.zeros((5,) + N), np.zeros((3,) + tuple(m + 1 for m in N))
    orc.restrict(cfg, fc, fb, cc, cb, org)
    xc, yc, zc = cell_centres(N, 2, 1.0)
    wantc = 1.0 + 0.5 * xc - 2.0 * yc + 0.25 * zc
    s = octant_slices(n, 2, o)
    assert np.abs(cc[0][s] - wantc[s]).max() <= 1e-13
    wantb = linear_faces(N, 2, 1.0, M, b0)
    for d in range(3):
        e = [0, 0, 0]
        e[d] = 1
        sf = octant_slices(n, 2, o, e)
        assert np.abs(cb[d][sf] - wantb[d][sf]).max() <= 1e-13


def mirror_x(cells, faces):
    """Reflect x -> L - x: cells reverse along i; the x faces reverse over all
    N1 + 1 entries and change sign; the y and z faces reverse like cells."""
    c = cells[..., ::-1].copy()
    f = np.zeros_like(faces)
    f[0] = -faces[0][..., ::-1]
    f[1][..., :-1] = faces[1][..., :-1][..., ::-1]
    f[2][..., :-1] = faces[2][..., :-1][..., ::-1]
    return c, f


@pytest.mark.parametrize("o", [(0, 0, 0), (1, 0, 1)])
def test_prolongation_commutes_with_a_mirror(orc, o):
    n = (8, 6, 4)
    cfg, N = geom(orc, n)
    cc, cb = random_block(N, 5, seed=12)
    org = oct_origin(n, o)
    fc, fb = prolong(orc, cfg, cc, cb, org)
    mc, mb = mirror_x(cc, cb)
    morg = (n[0] // 2 - org[0],) + org[1:]
    gc, gb = prolong(orc, cfg, mc, mb, morg)
    wc, wb = mirror_x(fc, fb)
    a = (slice(None), slice(2, 2 + n[2]), slice(2, 2 + n[1]), slice(2, 2 + n[0]))
    assert np.abs(gc[a] - wc[a]).max() <= 1e-14
    for d in range(3):
        e = [0, 0, 0]
        e[d] = 1
        s = (slice(2, 2 + n[2] + e[2]), slice(2, 2 + n[1] + e[1]), slice(2, 2 + n[0] + e[0]))
        assert np.abs(gb[d][s] - wb[d][s]).max() <= 1e-13, d


def cycle(cells, faces):
    """Relabel axes (x, y, z) -> (z, x, y): the new x is the old y, the new y
    the old z, the new z the old x."""
    c = np.ascontiguousarray(cells.transpose(0, 3, 1, 2))
    f = np.stack([faces[1].transpose(2, 0, 1), faces[2].transpose(2, 0, 1), faces[0].transpose(2, 0, 1)])
    return c, np.ascontiguousarray(f)


@pytest.mark.parametrize("o", [(0, 0, 0), (1, 0, 1), (0, 1, 1)])
def test_prolongation_commutes_with_cycling_the_axes(orc, o):
    n = (8, 8, 8)
    cfg, N = geom(orc, n)
    cc, cb = random_block(N, 5, seed=13)
    org = oct_origin(n, o)
    fc, fb = prolong(orc, cfg, cc, cb, org)
    rc, rb = cycle(cc, cb)
    gc, gb = prolong(orc, cfg, rc, rb, (org[1], org[2], org[0]))
    wc, wb = cycle(fc, fb)
    a = (slice(None), slice(2, 10), slice(2, 10), slice(2, 10))
    assert np.abs(gc[a] - wc[a]).max() <= 1e-14
    for d in range(3):
        e = [0, 0, 0]
        e[d] = 1
        s = (slice(2, 10 + e[2]), slice(2, 10 + e[1]), slice(2, 10 + e[0]))
        assert np.abs(gb[d][s] - wb[d][s]).max() <= 1e-13, d


def pressure(cells, faces, n, ng, gamma):
    """Pressure of every active cell from U and the mean of its two bounding faces."""
    a = (slice(ng, ng + n[2]), slice(ng, ng + n[1]), slice(ng, ng + n[0]))
    b1 = faces[0][a[0], a[1], ng:ng + n[0] + 1]
    b2 = faces[1][a[0], ng:ng + n[1] + 1, a[2]]
    b3 = faces[2][ng:ng + n[2] + 1, a[1], a[2]]
    bc = [0.5 * (b1[..., :-1] + b1[..., 1:]), 0.5 * (b2[:, :-1] + b2[:, 1:]), 0.5 * (b3[:-1] + b3[1:])]
    rho = cells[0][a]
    kin = 0.5 * (cells[1][a] ** 2 + cells[2][a] ** 2 + cells[3][a] ** 2) / rho
    return (gamma - 1.0) * (cells[4][a] - kin - 0.5 * (bc[0] ** 2 + bc[1] ** 2 + bc[2] ** 2))


def cold_state(N, F, seed):
    """rho near 1, momenta of order 1 varying from cell to cell, pressure 1e-4:
    linear interpolation of E and M separately then leaves some children with
    less E than their kinetic energy (M^2 / 2 rho is convex)."""
    rng = np.random.default_rng(seed)
    cells = np.empty((5,) + N)
    cells[0] = 1.0 + 0.2 * rng.random(N)
    cells[1:4] = rng.standard_normal((3,) + N)
    faces = 0.05 * rng.standard_normal((3,) + F)
    bc = [0.5 * (faces[0][..., :-1][:, :-1, :] + faces[0][..., 1:][:, :-1, :])[:-1],
          0.5 * (faces[1][:, :-1][..., :-1] + faces[1][:, 1:][..., :-1])[:-1],
          0.5 * (faces[2][:-1][:, :-1, :-1] + faces[2][1:][:, :-1, :-1])]
    kin = 0.5 * (cells[1] ** 2 + cells[2] ** 2 + cells[3] ** 2) / cells[0]
    cells[4] = 1e-4 / (5.0 / 3.0 - 1.0) + kin + 0.5 * sum(b ** 2 for b in bc)
    return cells, faces


@pytest.mark.parametrize("o", [(0, 0, 0), (1, 1, 0)])
def test_pressure_floor_on_refined_cells(orc, o):
    """With a pressure floor, every refined cell has P >= pfloor; only E of the
    cells below it changes (upwards), and mass, momentum and faces are those
    of the prolongation without the floor, bitwise."""
    n, ng, pf = (8, 6, 4), 2, 1e-5
    N = (n[2] + 2 * ng, n[1] + 2 * ng, n[0] + 2 * ng)
    F = tuple(x + 1 for x in N)
    cc, cb = cold_state(N, F, seed=61)
    org = oct_origin(n, o)
    cfg0 = orc.make_cfg(n, ng, (0.1,) * 3, 5.0 / 3.0)
    cfg1 = orc.make_cfg(n, ng, (0.1,) * 3, 5.0 / 3.0, pfloor=pf)
    c0, b0 = prolong(orc, cfg0, cc, cb, org)
    c1, b1 = prolong(orc, cfg1, cc, cb, org)
    p0 = pressure(c0, b0, n, ng, 5.0 / 3.0)
    p1 = pressure(c1, b1, n, ng, 5.0 / 3.0)
    low = p0 < pf
    assert low.sum() >= 3                          # the floor is exercised
    assert np.array_equal(c1[:4], c0[:4]) and np.array_equal(b1, b0)
    a = (slice(ng, ng + n[2]), slice(ng, ng + n[1]), slice(ng, ng + n[0]))
    assert np.array_equal(c1[4][a][~low], c0[4][a][~low])
    assert np.all(c1[4][a][low] > c0[4][a][low])
    assert np.all(p1 >= pf * (1 - 1e-9)), p1.min()
    assert np.abs(p1[low] - pf).max() <= 1e-9 * np.abs(c1[4][a]).max()


def prims_of(cells, faces, n, ng, gamma=5.0 / 3.0):
    """(rho, v1, v2, v3, P, C...) of every active cell from U and its
    bounding faces."""
    a = (slice(ng, ng + n[2]), slice(ng, ng + n[1]), slice(ng, ng + n[0]))
    rho = cells[0][a]
    out = [rho] + [cells[k][a] / rho for k in (1, 2, 3)]
    out.append(pressure(cells, faces, n, ng, gamma))
    out += [cells[k][a] / rho for k in range(5, cells.shape[0])]
    return np.stack(out)


def linear_prims(N, ng, h, coef, shift=(0, 0, 0)):
    x, y, z = cell_centres(N, ng, h)
    return np.stack([c[0] + c[1] * (x + shift[0]) + c[2] * (y + shift[1]) + c[3] * (z + shift[2]) for c in coef])


PRIM_COEF = np.array([[1.0, 0.05, -0.03, 0.02], [0.3, 0.02, 0.01, -0.04], [-0.2, 0.01, 0.03, 0.02],
                      [0.1, -0.02, 0.02, 0.01], [0.8, 0.03, 0.01, -0.02], [0.5, 0.04, -0.01, 0.03]])


def cons_from_prims(w, faces, gamma=5.0 / 3.0):
    """Conserved variables of every stored cell (ghosts included) from
    primitives and the mean of the two stored faces bounding the cell."""
    b1 = 0.5 * (faces[0][:-1, :-1, :-1] + faces[0][:-1, :-1, 1:])
    b2 = 0.5 * (faces[1][:-1, :-1, :-1] + faces[1][:-1, 1:, :-1])
    b3 = 0.5 * (faces[2][:-1, :-1, :-1] + faces[2][1:, :-1, :-1])
    rho, v = w[0], w[1:4]
    u = np.empty_like(w)
    u[0] = rho
    u[1:4] = rho * v
    u[4] = w[4] / (gamma - 1.0) + 0.5 * rho * (v ** 2).sum(0) + 0.5 * (b1 ** 2 + b2 ** 2 + b3 ** 2)
    u[5:] = rho * w[5:]
    return u


@pytest.mark.parametrize("o", [(0, 0, 0), (1, 0, 1), (0, 1, 1), (1, 1, 1)])
def test_primitive_prolongation_of_linear_primitives_is_exact(orc, o):
    """Linear rho, v, P and C with a linear divergence-free field: the
    primitives of the fine cells (recovered from their U and fine faces) are
    the linear fields at the fine centres."""
    n, ng = (8, 6, 4), 2
    cfg, N = geom(orc, n, ns=1)
    M = np.array([[0.07, -0.13, 0.04], [0.21, -0.02, 0.09], [-0.06, 0.17, -0.05]])
    b0 = np.array([0.3, -0.2, 0.25])
    cb = linear_faces(N, ng, 1.0, M, b0)
    cc = cons_from_prims(linear_prims(N, ng, 1.0, PRIM_COEF), cb)
    org = oct_origin(n, o)
    fc, fb = np.zeros_like(cc), np.zeros_like(cb)
    orc.prolong(cfg, cc, cb, fc, fb, org, primitive=True)
    got = prims_of(fc, fb, n, ng)
    a = (slice(None), slice(ng, ng + n[2]), slice(ng, ng + n[1]), slice(ng, ng + n[0]))
    want = linear_prims(N, ng, 0.5, PRIM_COEF, shift=org)[a]
    assert np.abs(got - want).max() <= 1e-13


def test_primitive_prolongation_keeps_pressure_positive(orc):
    """The cold state whose conserved prolongation gives negative pressure:
    prolonging P itself (minmod) keeps every refined cell positive; density
    and faces are bitwise those of the conserved prolongation."""
    n, ng = (8, 6, 4), 2
    N = (n[2] + 2 * ng, n[1] + 2 * ng, n[0] + 2 * ng)
    F = tuple(x + 1 for x in N)
    cc, cb = cold_state(N, F, seed=61)
    cfg = orc.make_cfg(n, ng, (0.1,) * 3, 5.0 / 3.0)
    for o in [(0, 0, 0), (1, 1, 0)]:
        org = oct_origin(n, o)
        c0, b0 = prolong(orc, cfg, cc, cb, org)
        c1, b1 = np.zeros_like(cc), np.zeros_like(cb)
        orc.prolong(cfg, cc, cb, c1, b1, org, primitive=True)
        assert (pressure(c0, b0, n, ng, 5.0 / 3.0) < 0).any()
        assert pressure(c1, b1, n, ng, 5.0 / 3.0).min() > 0
        assert np.array_equal(c1[0], c0[0]) and np.array_equal(b1, b0)


# ---- boxes: the same operators between any even-aligned fine box and a
# coarse box, ghost zones included (coarse buffers, ghost-zone prolongation)

def test_octant_calls_are_boxes(orc):
    n, ng = (8, 6, 4), 2
    cfg, N = geom(orc, n, ns=1)
    cc, cb = random_block(N, 6, seed=91)
    o = (1, 0, 1)
    org = oct_origin(n, o)
    a = prolong(orc, cfg, cc, cb, org)
    fc, fb = np.zeros_like(cc), np.zeros_like(cb)
    orc.prolong_box(cfg, cc, cb, fc, fb, (ng,) * 3, tuple(ng + x for x in org), tuple(x // 2 for x in n))
    assert np.array_equal(fc, a[0]) and np.array_equal(fb, a[1])
    r1c, r1b = cc.copy(), cb.copy()
    r2c, r2b = cc.copy(), cb.copy()
    orc.restrict(cfg, a[0], a[1], r1c, r1b, org)
    orc.restrict_box(cfg, a[0], a[1], r2c, r2b, (ng,) * 3, tuple(ng + x for x in org), tuple(x // 2 for x in n))
    assert np.array_equal(r1c, r2c) and np.array_equal(r1b, r2b)


def coarse_linear(N, coef):
    """Linear cell fields of the stored index (coarse cell C has centre C + 1/2)."""
    z, y, x = np.meshgrid(*[np.arange(m) + 0.5 for m in N], indexing="ij")
    return np.stack([c[0] + c[1] * x + c[2] * y + c[3] * z for c in coef])


def test_restriction_into_the_coarse_ghost_zone(orc):
    """A fine boundary layer (4 fine cells thick) restricted into the coarse
    block's upper x1 ghost zone (2 cells), as for a coarse buffer: linear
    fields exact, nothing outside the box written."""
    n, ng = (8, 8, 8), 4
    cfg, N = geom(orc, n, ng=ng)
    coef = [[0.3, 1.5, -2.0, 0.7], [1.0, 0.2, 0.9, -0.4], [2.0, -0.3, 0.1, 1.1], [0.5, 0.0, 0.3, 0.0],
            [1.0, 3.0, 2.0, 1.0]]
    flo, clo, ext = (ng + n[0] - 4, ng, ng), (ng + n[0], ng + 2, ng), (2, 4, 4)
    # fine fields: linear in the coarse coordinate of each fine centre
    z, y, x = np.meshgrid(*[np.arange(m) for m in N], indexing="ij")
    xf = [clo[d] + ([x, y, z][d] - flo[d]) / 2.0 + 0.25 for d in range(3)]
    fc = np.stack([c[0] + c[1] * xf[0] + c[2] * xf[1] + c[3] * xf[2] for c in coef])
    _, fb = random_block(N, 5, seed=92)
    cc = np.full((5,) + N, 7.0)
    cb = np.full((3,) + tuple(m + 1 for m in N), 7.0)
    orc.restrict_box(cfg, fc, fb, cc, cb, flo, clo, ext)
    want = coarse_linear(N, coef)
    s = (slice(clo[2], clo[2] + ext[2]), slice(clo[1], clo[1] + ext[1]), slice(clo[0], clo[0] + ext[0]))
    assert np.abs(cc[(slice(None),) + s] - want[(slice(None),) + s]).max() <= 1e-13
    mask = np.zeros(N, bool)
    mask[s] = True
    assert np.all(cc[:, ~mask] == 7.0)


def test_prolongation_into_the_fine_ghost_zone(orc):
    """Coarse cells (ghosts of the coarse neighbour included) prolonged into
    the fine block's lower x1 ghost zone: linear cells and divergence-free
    linear faces exact, each fine cell with its parent's divergence, nothing
    outside the box written."""
    n, ng = (8, 8, 8), 4
    cfg, N = geom(orc, n, ng=ng)
    F = tuple(m + 1 for m in N)
    coef = [[0.3, 1.5, -2.0, 0.7], [1.0, 0.2, 0.9, -0.4], [2.0, -0.3, 0.1, 1.1], [0.5, 0.0, 0.3, 0.0],
            [1.0, 3.0, 2.0, 1.0]]
    cc = coarse_linear(N, coef)
    M = np.array([[0.7, -1.3, 0.4], [2.1, -0.2, 0.9], [-0.6, 1.7, -0.5]])
    b0 = np.array([0.3, -0.8, 1.2])
    cb = linear_faces(N, 0, 1.0, M, b0)          # coarse face positions: stored index
    flo, clo, ext = (0, ng, ng), (5, 3, 6), (2, 4, 3)
    fc = np.full((5,) + N, 7.0)
    fb = np.full((3,) + F, 7.0)
    orc.prolong_box(cfg, cc, cb, fc, fb, flo, clo, ext)
    s = tuple(slice(flo[d], flo[d] + 2 * ext[d]) for d in (2, 1, 0))
    z, y, x = np.meshgrid(*[np.arange(m) for m in N], indexing="ij")
    xf = [clo[d] + ([x, y, z][d] - flo[d]) / 2.0 + 0.25 for d in range(3)]
    want = np.stack([c[0] + c[1] * xf[0] + c[2] * xf[1] + c[3] * xf[2] for c in coef])
    assert np.abs(fc[(slice(None),) + s] - want[(slice(None),) + s]).max() <= 1e-13
    mask = np.zeros(N, bool)
    mask[s] = True
    assert np.all(fc[:, ~mask] == 7.0)
    # faces: the fine face at fine index i along d sits at coarse coordinate
    # clo_d + (i - flo_d) / 2; transverse centres as for cells
    zf, yf, xf_ = np.meshgrid(*[np.arange(m) for m in F], indexing="ij")
    idx = [xf_, yf, zf]
    for d in range(3):
        pos = [clo[e] + (idx[e] - flo[e]) / 2.0 + (0.0 if e == d else 0.25) for e in range(3)]
        wantd = b0[d] + M[d][0] * pos[0] + M[d][1] * pos[1] + M[d][2] * pos[2]
        e = [0, 0, 0]
        e[d] = 1
        sf = tuple(slice(flo[k], flo[k] + 2 * ext[k] + e[k]) for k in (2, 1, 0))
        assert np.abs(fb[d][sf] - wantd[sf]).max() <= 2e-14, d
        m = np.zeros(F, bool)
        m[sf] = True
        assert np.all(fb[d][~m] == 7.0)


def _sin_avg(lo, h, k):
    """Average of sin(k x) over [lo, lo + h]."""
    return (np.cos(k * lo) - np.cos(k * (lo + h))) / (k * h)


def _prolong_l1_error(orc, n):
    """L1 error of the prolonged cells of octant (0, 0, 0) against the exact
    fine-cell averages of U = 2 + sin(2 pi x) + sin(2 pi (y + 0.1)) / 2 +
    0.3 sin(2 pi (z + 0.3)) on the unit cube (n coarse cells per side)."""
    ng, hc = 2, 1.0 / n
    cfg = orc.make_cfg((n, n, n), ng, (hc,) * 3, 5.0 / 3.0)
    N = n + 2 * ng
    idx = np.arange(N) - ng
    k = 2.0 * np.pi

    def field(h):
        ax, ay, az = _sin_avg(idx * h, h, k), _sin_avg(idx * h + 0.1, h, k), _sin_avg(idx * h + 0.3, h, k)
        return 2.0 + ax[None, None, :] + 0.5 * ay[None, :, None] + 0.3 * az[:, None, None]

    cc = np.stack([field(hc)] * 5)
    cb = np.zeros((3, N + 1, N + 1, N + 1))
    fc, fb = np.zeros_like(cc), np.zeros_like(cb)
    orc.prolong(cfg, cc, cb, fc, fb, (0, 0, 0))
    a = (slice(ng, ng + n),) * 3
    return float(np.abs(fc[0][a] - field(hc / 2)[a]).mean())


def test_cell_prolongation_is_second_order_on_smooth_data(orc):
    """Minmod-limited linear prolongation is second-order accurate in L1 on
    a smooth field (the limiter clips only near extrema)."""
    e = [_prolong_l1_error(orc, n) for n in (8, 16, 32)]
    rates = [np.log2(e[i] / e[i + 1]) for i in range(2)]
    assert min(rates) >= 1.9, (e, rates)


def curl_faces(N, seed, scale=1.0):
    """A face field with zero discrete divergence: the discrete curl of a
    random edge potential (forward differences commute)."""
    rng = np.random.default_rng(seed)
    ax, ay, az = scale * rng.standard_normal((3,) + tuple(m + 2 for m in N))
    s = slice(0, -1)
    bx = (az[s, 1:, s] - az[s, s, s]) - (ay[1:, s, s] - ay[s, s, s])
    by = (ax[1:, s, s] - ax[s, s, s]) - (az[s, s, 1:] - az[s, s, s])
    bz = (ay[s, s, 1:] - ay[s, s, s]) - (ax[s, 1:, s] - ax[s, s, s])
    return np.ascontiguousarray(np.stack([bx, by, bz]))


@pytest.mark.parametrize("o", [(0, 0, 0), (1, 0, 1)])
def test_kept_fine_faces_are_used_and_keep_the_field_divergence_free(orc, o):
    """Fine faces that already exist on the box's sides are kept (bitwise)
    and the interior faces are solved with them: a divergence-free fine field,
    restricted to the coarse level and prolonged back with all 6 sides kept,
    stays divergence-free; without keeping, the sides change."""
    n, ng = (8, 6, 4), 2
    cfg, N = geom(orc, n)
    fb_true = curl_faces(N, seed=111)
    assert np.abs(divergence(fb_true, ng, n, 1.0)).max() <= 1e-13
    cc, cb = random_block(N, 5, seed=112)
    org = oct_origin(n, o)
    orc.restrict(cfg, np.zeros_like(cc), fb_true, cc, cb, org)      # coarse faces of the octant
    box = ((ng,) * 3, tuple(ng + x for x in org), tuple(x // 2 for x in n))
    sides = np.zeros((3,) + fb_true.shape[1:], bool)                 # faces on the box's 6 sides
    for d in range(3):
        idx = [slice(ng, ng + n[k] + (1 if k == d else 0)) for k in range(3)]
        for side in (ng, ng + n[d]):
            sl = list(idx)
            sl[d] = side
            sides[d][sl[2], sl[1], sl[0]] = True
    fc = np.zeros_like(cc)
    fb = np.where(sides, fb_true, 7.0)
    orc.prolong_box(cfg, cc, cb, fc, fb, *box, keep=63)
    assert np.array_equal(fb[sides], fb_true[sides])
    assert np.abs(divergence(fb, ng, n, 1.0)).max() <= 1e-12 * np.abs(fb_true).max()
    fb0 = np.where(sides, fb_true, 7.0)
    orc.prolong_box(cfg, cc, cb, np.zeros_like(cc), fb0, *box, keep=0)
    assert not np.array_equal(fb0[sides], fb_true[sides])
    assert np.abs(divergence(fb0, ng, n, 1.0)).max() <= 1e-12 * np.abs(fb_true).max()
