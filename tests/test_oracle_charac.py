"""Pins of the oracle's characteristic reconstruction (Sec. 3.2.1: PLM and
PPM on the characteristic variables C = L W of the primitive system).

The eigenvectors are checked against the primitive-variable form of the ideal
MHD equations (Eq. (cons) with the ideal-gas law), written out here as the
quasi-linear matrix A of W_t + A W_x = 0 in the face frame: L A R must be
diagonal with the seven wave speeds, and L R = I, also where speeds coincide
(no transverse field, no normal field).  The reconstruction itself is pinned
by what projecting, limiting per family and projecting back must give:
exact linear profiles, independent limiting of two families (a family at an
extremum gets no slope while the other keeps its van Leer slope), unchanged
donor-cell states, and at the step level uniform states, conservation,
div B, direction independence and the paper's motivation: fewer
oscillations at MHD discontinuities (Brio & Wu).
"""
import math

import numpy as np
import pytest

from test_oracle_pins import _line_problem

G = 5.0 / 3.0


def prim_matrix(w, bn, g):
    """A of W_t + A W_x = 0 for W = (rho, vn, vt1, vt2, P, Bt1, Bt2), normal
    field bn: continuity, momentum with the magnetic pressure and tension
    terms, the adiabatic pressure equation and the induction equation."""
    rho, u, v, ww, p, b1, b2 = w
    return np.array([
        [u, rho, 0, 0, 0, 0, 0],
        [0, u, 0, 0, 1 / rho, b1 / rho, b2 / rho],
        [0, 0, u, 0, 0, -bn / rho, 0],
        [0, 0, 0, u, 0, 0, -bn / rho],
        [0, g * p, 0, 0, u, 0, 0],
        [0, b1, -bn, 0, 0, u, 0],
        [0, b2, 0, -bn, 0, 0, u],
    ], dtype=float)


def wave_speeds(w, bn, g):
    rho, p = w[0], w[4]
    a2, ca2 = g * p / rho, bn * bn / rho
    b2 = ca2 + (w[5] ** 2 + w[6] ** 2) / rho
    d = math.sqrt(max((a2 + b2) ** 2 - 4 * a2 * ca2, 0.0))
    cf, cs = math.sqrt(0.5 * (a2 + b2 + d)), math.sqrt(max(0.5 * (a2 + b2 - d), 0.0))
    return np.array([-cf, -math.sqrt(ca2), -cs, 0.0, cs, math.sqrt(ca2), cf]) + w[1]


def states():
    rng = np.random.default_rng(11)
    out = [(np.array([1.0, 0.3, -0.2, 0.1, 0.7, 0.5, -0.4]), 0.8),
           (np.array([1.3, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0]), 0.9),      # no transverse field
           (np.array([0.7, 0.1, 0.0, 0.0, 0.5, 0.0, 0.0]), 0.0),      # no field at all
           (np.array([1.0, 0.0, 0.0, 0.0, 0.6, 0.2, 0.3]), -0.5),     # negative normal field
           (np.array([1.0, 0.0, 0.0, 0.0, 0.6, 1.1, 0.0]), 0.0)]      # transverse field only
    for _ in range(12):
        out.append((np.array([rng.uniform(0.2, 2), *rng.normal(size=3), rng.uniform(0.1, 2), *rng.normal(size=2)]),
                    float(rng.normal())))
    return out


@pytest.mark.parametrize("case", range(17))
def test_eigenvectors_diagonalise_the_primitive_system(orc, case):
    w, bn = states()[case]
    R, L = orc.prim_eigen(G, w, bn)
    assert np.abs(L @ R - np.eye(7)).max() < 1e-13
    D = L @ prim_matrix(w, bn, G) @ R
    scale = np.abs(np.diag(D)).max() + 1.0
    assert np.abs(D - np.diag(np.diag(D))).max() < 1e-13 * scale
    assert np.abs(np.diag(D) - wave_speeds(w, bn, G)).max() < 1e-12 * scale
    assert np.linalg.cond(R) < 1e3  # the normalisation keeps R well conditioned


def test_linear_profile_is_reconstructed_exactly(orc):
    w0, bn = states()[0]
    dw = np.array([0.01, -0.02, 0.03, 0.005, -0.01, 0.02, -0.015])
    left, right = orc.char_plm(G, w0 - dw, w0, w0 + dw, bn)
    assert np.allclose(left, w0 - 0.5 * dw, rtol=0, atol=1e-15)
    assert np.allclose(right, w0 + 0.5 * dw, rtol=0, atol=1e-15)


@pytest.mark.parametrize("case", [0, 3, 6])
def test_each_wave_family_is_limited_on_its_own(orc, case):
    """Left difference a1 r_f- + b r_f+, right difference a2 r_f- - b r_f+:
    the fast family moving left keeps the van Leer slope of (a1, a2), the one
    moving right is at an extremum and gets none.  Limiting the primitive
    variables instead would mix the two."""
    w0, bn = states()[case]
    R, _ = orc.prim_eigen(G, w0, bn)
    a1, a2, b = 0.02, 0.05, 0.03
    dl = a1 * R[:, 0] + b * R[:, 6]
    dr = a2 * R[:, 0] - b * R[:, 6]
    left, right = orc.char_plm(G, w0 - dl, w0, w0 + dr, bn)
    slope = 2 * a1 * a2 / (a1 + a2) * R[:, 0]
    assert np.allclose(left, w0 - 0.5 * slope, rtol=0, atol=1e-14)
    assert np.allclose(right, w0 + 0.5 * slope, rtol=0, atol=1e-14)


def _blk(orc, recon, integ="vl2", **kw):
    from paper_2005_06651_amd import inputs
    ng = 2
    b = inputs.smooth_random(n=(12, 10, 8), seed=21, ng=ng)
    cfg = orc.cfg_for(b, recon=recon, integrator=integ, **kw)
    return b, cfg, orc.prim2cons(cfg, b.prim, b.bface)


def test_donor_cell_is_unchanged(orc):
    b, cfg0, cons = _blk(orc, "dc", integ="rk2")
    _, cfg1, _ = _blk(orc, "dc", integ="rk2", charac=True)
    c0, b0, _, _ = orc.run(cfg0, cons, b.bface, 2, dt=0.004)
    c1, b1, _, _ = orc.run(cfg1, cons, b.bface, 2, dt=0.004)
    assert np.array_equal(c0, c1) and np.array_equal(b0, b1)


def test_characteristic_step_invariants(orc):
    """Uniform state preserved to rounding, totals of U conserved, div B at
    round-off, and a different result from primitive PLM on smooth data."""
    from paper_2005_06651_amd import inputs
    u = inputs.uniform(n=(8, 6, 4), ng=2)
    cfg = orc.cfg_for(u, recon="plm", charac=True)
    cons = orc.prim2cons(cfg, u.prim, u.bface)
    c, bf, _, _ = orc.run(cfg, cons, u.bface, 3, dt=0.01)
    a = u.active
    assert np.abs(c[(slice(None),) + a] - cons[(slice(None),) + a]).max() < 1e-14
    b, cfg1, cons = _blk(orc, "plm", charac=True)
    c1, b1, _, _ = orc.run(cfg1, cons, b.bface, 3)
    a = b.active
    for v in range(5):
        t0, t1 = cons[v][a].sum(), c1[v][a].sum()
        assert abs(t1 - t0) <= 1e-13 * max(abs(t0), 1.0)
    orc.fill_ghosts(cfg1, c1, b1)
    assert inputs.divb_metric(b1, b.n, b.ng, b.dx) < 1e-13
    _, cfg0, _ = _blk(orc, "plm")
    c0, _, _, _ = orc.run(cfg0, cons, b.bface, 3)
    assert np.abs(c0[0][a] - c1[0][a]).max() > 1e-8


def test_characteristic_1d_problem_is_direction_independent(orc):
    n, ng = 24, 2
    outs = []
    for axis in range(3):
        dims, prim, bf = _line_problem(n, axis, ng)
        cfg = orc.make_cfg(dims, ng, (1.0 / n,) * 3, G, recon="plm", riemann="hlld", integrator="vl2",
                           charac=True)
        cons = orc.prim2cons(cfg, prim, bf)
        c, b, _, _ = orc.run(cfg, cons, bf, 5, dt=0.004)
        t1 = (axis + 1) % 3
        sl = [slice(ng + 1, ng + 2)] * 3
        sl[2 - axis] = slice(ng, ng + n)
        sl = tuple(sl)
        outs.append(np.stack([c[0][sl].ravel(), c[1 + axis][sl].ravel(), c[1 + t1][sl].ravel(), c[4][sl].ravel(),
                              b[t1][sl].ravel()]))
    assert np.array_equal(outs[0], outs[1])
    assert np.array_equal(outs[0], outs[2])


def _brio_wu(n, ng=2):
    """Brio & Wu's shock tube (gamma 2, B_n = 0.75; left rho 1, P 1, B_t 1;
    right rho 0.125, P 0.1, B_t -1) as the two interfaces of a periodic
    domain along x1."""
    x = (np.arange(n) + 0.5) / n
    left = (x > 0.25) & (x < 0.75)
    rho = np.where(left, 1.0, 0.125)
    p = np.where(left, 1.0, 0.1)
    bt = np.where(left, 1.0, -1.0)
    N1 = n + 2 * ng
    N = (4 + 2 * ng, 4 + 2 * ng, N1)
    idx = np.mod(np.arange(N1) - ng, n)
    prim = np.zeros((5,) + N)
    bf = np.zeros((3, N[0] + 1, N[1] + 1, N1 + 1))
    prim[0][...] = rho[idx]
    prim[4][...] = p[idx]
    bf[0][...] = 0.75
    bf[1][:, :, :N1] = bt[idx]
    bf[1][:, :, N1] = bt[idx[0]]
    return (n, 4, 4), prim, bf


def test_characteristic_plm_oscillates_less_on_brio_wu(orc):
    """The paper's motivation for characteristic variables (Sec. 3.2.1): fewer
    oscillations in MHD solutions.  On Brio & Wu's tube the total variation of
    rho and of the transverse velocity at t = 0.08 is lower than with PLM on
    the primitive variables."""
    n, g = 256, 2
    dims, prim, bf = _brio_wu(n)
    tv = {}
    for ch in (False, True):
        cfg = orc.make_cfg(dims, g, (1.0 / n, 0.25, 0.25), 2.0, recon="plm", riemann="hlld", integrator="vl2",
                           cfl=0.4, charac=ch)
        c, _, _, _ = orc.run(cfg, orc.prim2cons(cfg, prim, bf), bf, 0, t_end=0.08)
        rho = c[0][g, g, g:g + n]
        vt = c[2][g, g, g:g + n] / rho
        tv[ch] = (np.abs(np.diff(rho)).sum(), np.abs(np.diff(vt)).sum())
    assert tv[True][0] < tv[False][0] and tv[True][1] < tv[False][1], tv


def _scalar_ppm_edges(orc, f):
    """Left and right edges of the middle cell of the 5 values f by the
    oracle's scalar PPM (pinned in test_oracle_pins)."""
    line = np.concatenate([[2 * f[0] - f[1]], f, [2 * f[4] - f[3]]])  # cells -3 .. 3
    ql, qr = orc.recon_line("ppm", line)
    return qr[3], ql[4]


@pytest.mark.parametrize("case", [0, 3, 6])
def test_ppm_reconstructs_each_wave_family_on_its_own(orc, case):
    """W = W_c + f r_a + g r_b with r_a, r_b two right eigenvectors of W_c and
    f, g two profiles vanishing at the middle cell (one monotone, one with an
    extremum): the characteristic PPM edges are W_c + ppm(f) r_a + ppm(g) r_b,
    each family reconstructed by the scalar PPM."""
    w0, bn = states()[case]
    R, _ = orc.prim_eigen(G, w0, bn)
    f = np.array([-0.03, -0.012, 0.0, 0.01, 0.025])     # monotone
    h = np.array([0.02, 0.015, 0.0, 0.012, 0.03])       # minimum at the middle cell
    ra, rb = R[:, 0], R[:, 4]
    stencil = np.array([w0 + f[o] * ra + h[o] * rb for o in range(5)])
    left, right = orc.char_ppm(G, stencil, bn)
    fl, fr = _scalar_ppm_edges(orc, f)
    hl, hr = _scalar_ppm_edges(orc, h)
    assert np.allclose(left, w0 + fl * ra + hl * rb, rtol=0, atol=1e-14)
    assert np.allclose(right, w0 + fr * ra + hr * rb, rtol=0, atol=1e-14)


def test_ppm_of_one_profile_equals_primitive_ppm(orc):
    """All components following one profile (W = W_c + f v): limiting is
    homogeneous, so the characteristic edges equal PPM on each primitive."""
    w0, bn = states()[0]
    v = np.array([0.1, -0.2, 0.05, 0.3, -0.1, 0.2, 0.15])
    f = np.array([-0.05, -0.02, 0.0, 0.03, 0.04])
    left, right = orc.char_ppm(G, np.array([w0 + f[o] * v for o in range(5)]), bn)
    fl, fr = _scalar_ppm_edges(orc, f)
    assert np.allclose(left, w0 + fl * v, rtol=0, atol=1e-14)
    assert np.allclose(right, w0 + fr * v, rtol=0, atol=1e-14)


def test_characteristic_ppm_step_invariants_and_symmetry(orc):
    from paper_2005_06651_amd import inputs
    u = inputs.uniform(n=(8, 6, 4), ng=3)
    cfg = orc.cfg_for(u, recon="ppm", integrator="rk3", charac=True)
    cons = orc.prim2cons(cfg, u.prim, u.bface)
    c, _, _, _ = orc.run(cfg, cons, u.bface, 2, dt=0.01)
    a = (slice(None),) + u.active
    assert np.abs(c[a] - cons[a]).max() < 1e-14
    b = inputs.smooth_random(n=(12, 10, 8), seed=23, ng=3)
    cfg = orc.cfg_for(b, recon="ppm", integrator="rk3", charac=True)
    cons = orc.prim2cons(cfg, b.prim, b.bface)
    c1, b1, _, _ = orc.run(cfg, cons, b.bface, 2)
    for v in range(5):
        t0, t1 = cons[v][b.active].sum(), c1[v][b.active].sum()
        assert abs(t1 - t0) <= 1e-13 * max(abs(t0), 1.0)
    orc.fill_ghosts(cfg, c1, b1)
    assert inputs.divb_metric(b1, b.n, b.ng, b.dx) < 1e-13
    n, ng = 24, 3
    outs = []
    for axis in range(3):
        dims, prim, bf = _line_problem(n, axis, ng)
        cfg = orc.make_cfg(dims, ng, (1.0 / n,) * 3, G, recon="ppm", riemann="hlld", integrator="rk3", charac=True)
        c, bb, _, _ = orc.run(cfg, orc.prim2cons(cfg, prim, bf), bf, 4, dt=0.004)
        t1 = (axis + 1) % 3
        sl = [slice(ng + 1, ng + 2)] * 3
        sl[2 - axis] = slice(ng, ng + n)
        sl = tuple(sl)
        outs.append(np.stack([c[0][sl].ravel(), c[1 + axis][sl].ravel(), c[1 + t1][sl].ravel(), c[4][sl].ravel(),
                              bb[t1][sl].ravel()]))
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])


def test_characteristic_ppm_oscillates_less_on_brio_wu(orc):
    """As for PLM: RK3 + characteristic PPM on Brio & Wu's tube has lower
    total variation of rho and v_t at t = 0.08 than PPM on the primitives."""
    n, g = 256, 3
    dims, prim, bf = _brio_wu(n, ng=g)
    tv = {}
    for ch in (False, True):
        cfg = orc.make_cfg(dims, g, (1.0 / n, 0.25, 0.25), 2.0, recon="ppm", riemann="hlld", integrator="rk3",
                           cfl=0.4, charac=ch)
        c, _, _, _ = orc.run(cfg, orc.prim2cons(cfg, prim, bf), bf, 0, t_end=0.08)
        rho = c[0][g, g, g:g + n]
        vt = c[2][g, g, g:g + n] / rho
        tv[ch] = (np.abs(np.diff(rho)).sum(), np.abs(np.diff(vt)).sum())
    assert tv[True][0] < tv[False][0] and tv[True][1] < tv[False][1], tv
