"""Pins of the oracle's two-level composite (Sec. 2.1.3 communication between
levels, Sec. 2.1.4 flux and EMF correction, Sec. 3.4.1 linear wave with mesh
refinement; reading R-35): one coarse block beside a 2 x 2 x 2 region of fine
blocks on a periodic domain.

What the paper fixes: the totals of U over both levels are conserved exactly
(the coarse flux through an interface is the area integral of the fine
fluxes), div B stays at round-off on every block (the coarse EMFs on an
interface are the line integrals of the fine ones, Eq. emfcorr), a uniform
state is preserved, and the linear wave converges at second order with an
error no larger than on the unrefined root grid.
"""
import math

import numpy as np
import pytest

from paper_2005_06651_amd import inputs

N3 = (8, 8, 8)
BOX = (2.0, 1.0, 1.0)


def composite(orc, seed=5, ng=2, n=N3, **kw):
    cg = inputs.analytic_state((2 * n[0], n[1], n[2]), ng, BOX, seed=seed)
    fg = inputs.analytic_state((4 * n[0], 2 * n[1], 2 * n[2]), ng, BOX, seed=seed)
    prim, bf = inputs.two_level(cg, fg, n)
    cfg = orc.make_cfg(n, ng, cg.dx, cg.gamma, **kw)
    cons = np.ascontiguousarray(np.stack([orc.prim2cons(cfg, prim[b], bf[b]) for b in range(9)]))
    bf = np.ascontiguousarray(bf)
    assert orc.two_level_fill(cfg, cons, bf) == 0
    return cfg, cons, bf, cg.dx


def totals(cons, n, ng, dx):
    a = (slice(None), slice(ng, ng + n[2]), slice(ng, ng + n[1]), slice(ng, ng + n[0]))
    dv = dx[0] * dx[1] * dx[2]
    t = cons[0][a].sum(axis=(1, 2, 3)) * dv
    for b in range(1, 9):
        t = t + cons[b][a].sum(axis=(1, 2, 3)) * dv / 8.0
    return t


def divb_all(bf, n, ng, dx):
    return max(inputs.divb_metric(bf[b], n, ng, dx if b == 0 else tuple(x / 2 for x in dx)) for b in range(9))


def test_two_level_preserves_a_uniform_state(orc):
    """A uniform state stays uniform to round-off on both levels."""
    n, ng = N3, 2
    u = inputs.uniform(n=n, ng=ng, dx=(0.25, 0.125, 0.125))
    cfg = orc.make_cfg(n, ng, u.dx, u.gamma, integrator="vl2", recon="plm", riemann="hlld")
    c1 = orc.prim2cons(cfg, u.prim, u.bface)
    cons = np.ascontiguousarray(np.stack([c1] * 9))
    bf = np.ascontiguousarray(np.stack([u.bface] * 9))
    ref_c, ref_b = cons.copy(), bf.copy()
    for _ in range(3):
        assert orc.two_level_step(cfg, cons, bf, 0.01) == 0
    # restriction sums eight equal values, which rounds: round-off, not bits
    assert np.max(np.abs(cons - ref_c)) <= 2e-15 and np.max(np.abs(bf - ref_b)) <= 2e-15


@pytest.mark.parametrize("integ,recon,rs,ng", [("vl2", "plm", "hlld", 2), ("rk3", "ppm", "hlle", 4),
                                               ("rk1", "dc", "roe", 2)])
def test_two_level_conserves_totals_and_div_b(orc, integ, recon, rs, ng):
    """Totals of rho, M and E over both levels constant to round-off, and the
    div B metric at round-off on every block, over several steps."""
    n = N3 if ng == 2 else (8, 8, 8)
    cfg, cons, bf, dx = composite(orc, seed=6, ng=ng, n=n, integrator=integ, recon=recon, riemann=rs)
    t0 = totals(cons, n, ng, dx)
    assert divb_all(bf, n, ng, dx) <= 1e-14
    for _ in range(5):
        dt, bad = orc.two_level_newdt(cfg, cons, bf)
        assert bad == 0
        assert orc.two_level_step(cfg, cons, bf, dt) == 0
    t = totals(cons, n, ng, dx)
    assert np.max(np.abs(t - t0)) <= 1e-14 * np.max(np.abs(t0))
    assert divb_all(bf, n, ng, dx) <= 1e-14


def test_two_level_coarse_interface_faces_are_fine_averages(orc):
    """After a step (which ends with the composite ghost fill), the coarse
    block's x1 boundary faces are the area averages of the four fine faces on
    them (restriction, Sec. 2.1.5), and the coarse x1 ghost cells are the
    volume averages of the eight fine cells."""
    n, ng = N3, 2
    cfg, cons, bf, dx = composite(orc, seed=7, ng=ng, integrator="vl2", recon="plm", riemann="hlld")
    dt, _ = orc.two_level_newdt(cfg, cons, bf)
    assert orc.two_level_step(cfg, cons, bf, dt) == 0
    for side in range(2):
        ci = ng if side == 0 else ng + n[0]
        fi = ng + n[0] if side == 0 else ng
        fa = 1 if side == 0 else 0
        for k in range(ng, ng + n[2]):
            for j in range(ng, ng + n[1]):
                s = 0.0
                for dk in range(2):
                    for dj in range(2):
                        gj, gk = 2 * (j - ng) + dj, 2 * (k - ng) + dk
                        blk = 1 + fa + 2 * (gj // n[1]) + 4 * (gk // n[2])
                        s += bf[blk, 0, ng + gk % n[2], ng + gj % n[1], fi]
                assert abs(bf[0, 0, k, j, ci] - 0.25 * s) <= 1e-15 * max(1.0, abs(s))
    # a coarse ghost cell on the lower x1 side: eight fine cells of the a = 1 blocks
    j, k = ng + 1, ng + 2
    s = 0.0
    for dk in range(2):
        for dj in range(2):
            for di in range(2):
                gj, gk = 2 * (j - ng) + dj, 2 * (k - ng) + dk
                blk = 1 + 1 + 2 * (gj // n[1]) + 4 * (gk // n[2])
                s += cons[blk, 0, ng + gk % n[2], ng + gj % n[1], ng + n[0] - 2 + di]
    assert abs(cons[0, 0, k, j, ng - 1] - s / 8.0) <= 1e-15 * abs(s)


def _linear_wave_error(orc, N, refined):
    lw = inputs.linear_wave(N)
    cfg_kw = dict(integrator="vl2", recon="plm", riemann="hlld", cfl=0.3)
    if not refined:
        cfg = orc.cfg_for(lw, **cfg_kw)
        c, bf, t, _ = orc.run(cfg, lw.cons, lw.bface, 0, t_end=0.5)
        a = lw.active
        vol = np.prod(lw.meta["box"])
        dv = np.prod(lw.dx)
        return math.sqrt(sum((np.abs(c[v][a] - lw.cons[v][a]).sum() * dv / vol) ** 2 for v in range(5)))
    fine = inputs.linear_wave(2 * N)
    n = (N, N, N)
    cons, bf = inputs.two_level(lw, fine, n)
    cfg = orc.make_cfg(n, lw.ng, lw.dx, lw.gamma, **cfg_kw)
    assert orc.two_level_fill(cfg, cons, bf) == 0
    c0 = cons.copy()
    t = 0.0
    while t < 0.5 * (1 - 1e-14):
        dt, bad = orc.two_level_newdt(cfg, cons, bf)
        assert bad == 0
        dt = min(dt, 0.5 - t)
        assert orc.two_level_step(cfg, cons, bf, dt) == 0
        t += dt
    g = lw.ng
    a = (slice(g, g + N), slice(g, g + N), slice(g, g + N))
    vol = np.prod(lw.meta["box"])
    dv = np.prod(lw.dx)
    err = 0.0
    for v in range(5):
        e = np.abs(cons[0][v][a] - c0[0][v][a]).sum() * dv
        for b in range(1, 9):
            e += np.abs(cons[b][v][a] - c0[b][v][a]).sum() * dv / 8.0
        err += (e / vol) ** 2
    return math.sqrt(err)


@pytest.mark.slow
def test_two_level_linear_wave_second_order(orc):
    """Sec. 3.4.1: the fast linear wave through a static two-level composite
    (half of the box refined) converges at second order (N = 8 -> 16), and its
    error is no larger than on the unrefined root grid of the same N."""
    e8, e16 = _linear_wave_error(orc, 8, True), _linear_wave_error(orc, 16, True)
    u16 = _linear_wave_error(orc, 16, False)
    order = math.log2(e8 / e16)
    assert order >= 1.8, (e8, e16, order)
    assert e16 <= u16, (e16, u16)
