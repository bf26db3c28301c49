"""Pins of the oracle's passive scalars (Sec. 3.2.6, "Additional Physics":
Eq. (passive_scalars), d(rho C_i)/dt + div(rho v C_i) = 0, with the specific
density C_i as the primitive and rho C_i as the conserved variable).

None of these re-types the oracle's scalar flux.  They check what the transport
equation and its upwind discretisation fix:
  * C_i = 1 turns the scalar equation into the continuity equation, so rho C_i
    must follow rho exactly, bitwise;
  * the MHD variables do not see the scalars;
  * C -> a C + b maps rho C to a rho C + b rho (the transport equation is
    linear in C and reconstruction of a primitive commutes with affine maps);
  * in a uniform flow the donor-cell step is the textbook first-order upwind
    scheme, in closed form, for either sign of the velocity;
  * the first-order upwind step keeps C inside its initial range (mass-flux
    upwinding is a convex combination), which a central or downwind flux
    breaks;
  * total scalar mass is conserved;
  * smooth advection in a uniform flow converges at the order of the
    reconstruction (second order for PLM, third for PPM with RK3; the paper's
    scalar-advection tests show the same orders).
"""
import math

import numpy as np
import pytest

from paper_2005_06651_amd import inputs

COMBOS = [
    dict(integrator="vl2", recon="plm", riemann="hlld"),
    dict(integrator="rk3", recon="ppm", riemann="hlle"),
    dict(integrator="rk2", recon="dc", riemann="hlld", ct_eps=1e-3),
    dict(integrator="rk1", recon="plm", riemann="hlle"),
]


def act(b):
    g = b.ng
    n1, n2, n3 = b.n
    return (slice(None), slice(g, g + n3), slice(g, g + n2), slice(g, g + n1))


def scalar_block(n=(12, 10, 8), seed=3, ng=2, ns=2):
    return inputs.with_scalars(inputs.smooth_random(n=n, seed=seed, ng=ng), ns, seed=seed + 100)


def run(orc, cfg, cons, bf, nsteps):
    cons, bf = cons.copy(), bf.copy()
    for _ in range(nsteps):
        dt, bad = orc.newdt(cfg, cons, bf)
        assert bad == 0
        assert orc.step(cfg, cons, bf, dt) == 0
    return cons, bf


@pytest.mark.parametrize("kw", COMBOS)
def test_unit_concentration_follows_density_bitwise(orc, kw):
    ng = 3 if kw["recon"] == "ppm" else 2
    b = scalar_block(ng=ng)
    prim = b.prim.copy()
    prim[5] = 1.0
    cfg = orc.cfg_for(b, nscalars=2, **kw)
    c, _ = run(orc, cfg, orc.prim2cons(cfg, prim, b.bface), b.bface, 3)
    assert np.array_equal(c[5], c[0])


@pytest.mark.parametrize("kw", COMBOS[:2])
def test_scalars_leave_the_mhd_state_alone(orc, kw):
    ng = 3 if kw["recon"] == "ppm" else 2
    b = scalar_block(ng=ng)
    cfg2 = orc.cfg_for(b, nscalars=2, **kw)
    cfg0 = orc.cfg_for(b, **kw)
    c2, f2 = run(orc, cfg2, orc.prim2cons(cfg2, b.prim, b.bface), b.bface, 2)
    c0, f0 = run(orc, cfg0, orc.prim2cons(cfg0, np.ascontiguousarray(b.prim[:5]), b.bface), b.bface, 2)
    assert np.array_equal(c2[:5], c0)
    assert np.array_equal(f2, f0)


@pytest.mark.parametrize("kw", COMBOS)
@pytest.mark.parametrize("a,off", [(-0.7, 2.3), (3.0, -0.4)])
def test_affine_map_of_the_concentration(orc, kw, a, off):
    ng = 3 if kw["recon"] == "ppm" else 2
    b = scalar_block(ng=ng, ns=1)
    cfg = orc.cfg_for(b, nscalars=1, **kw)
    c, _ = run(orc, cfg, orc.prim2cons(cfg, b.prim, b.bface), b.bface, 2)
    prim = b.prim.copy()
    prim[5] = a * prim[5] + off
    c2, _ = run(orc, cfg, orc.prim2cons(cfg, prim, b.bface), b.bface, 2)
    want = a * c[5] + off * c[0]
    s = act(b)[1:]
    err = np.abs(c2[5][s] - want[s]).max() / np.abs(want[s]).max()
    assert err <= 1e-13, err


@pytest.mark.parametrize("rs", ["hlld", "hlle"])
@pytest.mark.parametrize("vel", [(0.6, 0.0, 0.0), (-0.45, 0.0, 0.0), (0.3, -0.5, 0.25)])
def test_donor_cell_step_is_first_order_upwind(orc, rs, vel):
    """Uniform rho, v, p, B: one RK1 step with donor-cell states is
    s_i - dt sum_d rho u_d (C_up(i+1/2) - C_up(i-1/2)) / dx_d with the upwind
    cell on the side the flow comes from."""
    n = (10, 8, 6)
    dx = (0.1, 0.125, 1.0 / 6.0)
    b = inputs.uniform(n=n, ng=2, rho=1.3, v=vel, p=0.8, B=(0.4, -0.3, 0.2), dx=dx)
    b = inputs.with_scalars(b, 1, seed=7)
    cfg = orc.cfg_for(b, nscalars=1, integrator="rk1", recon="dc", riemann=rs)
    cons = orc.prim2cons(cfg, b.prim, b.bface)
    dt = 0.02
    c1, _ = cons.copy(), None
    bf = b.bface.copy()
    assert orc.step(cfg, c1, bf, dt) == 0
    g = b.ng
    C = b.prim[5][g:g + n[2], g:g + n[1], g:g + n[0]]
    rho = 1.3
    want = rho * C
    for d, ax in ((0, 2), (1, 1), (2, 0)):
        u = vel[d]
        if u == 0.0:
            continue
        # flux through the lower face of each cell, from the upwind side
        lower = rho * u * (np.roll(C, 1, axis=ax) if u > 0 else C)
        upper = np.roll(lower, -1, axis=ax)
        want = want - dt * (upper - lower) / dx[d]
    got = c1[5][g:g + n[2], g:g + n[1], g:g + n[0]]
    assert np.abs(got - want).max() <= 1e-14 * rho


@pytest.mark.parametrize("kw", [dict(riemann="hlld"), dict(riemann="hlle")])
def test_first_order_step_keeps_concentration_in_range(orc, kw):
    """RK1 + donor cell in a general flow: C after each step lies within the
    range of C before it (the dye starts in [0, 1])."""
    b = scalar_block(n=(12, 10, 8), seed=5, ns=1)
    cfg = orc.cfg_for(b, nscalars=1, integrator="rk1", recon="dc", cfl=0.3, **kw)
    cons = orc.prim2cons(cfg, b.prim, b.bface)
    bf = b.bface.copy()
    a = act(b)
    lo, hi = b.prim[5][a[1:]].min(), b.prim[5][a[1:]].max()
    for _ in range(4):
        dt, bad = orc.newdt(cfg, cons, bf)
        assert orc.step(cfg, cons, bf, dt) == 0
        C = cons[5][a[1:]] / cons[0][a[1:]]
        assert C.min() >= lo - 1e-14 and C.max() <= hi + 1e-14, (C.min(), C.max(), lo, hi)
        lo, hi = C.min(), C.max()


@pytest.mark.parametrize("kw", COMBOS)
def test_total_scalar_mass_is_conserved(orc, kw):
    ng = 3 if kw["recon"] == "ppm" else 2
    b = scalar_block(ng=ng)
    cfg = orc.cfg_for(b, nscalars=2, **kw)
    c0 = orc.prim2cons(cfg, b.prim, b.bface)
    c1, _ = run(orc, cfg, c0, b.bface, 3)
    a = act(b)
    for v in (5, 6):
        m0, m1 = c0[v][a[1:]].sum(), c1[v][a[1:]].sum()
        assert abs(m1 - m0) <= 1e-13 * abs(m0), (v, m0, m1)


def advect_error(orc, n1, recon, integrator):
    """L1 error of C after advecting a sine along x1 for a quarter period in a
    uniform flow (u = 1, unit box), against the exact shifted cell averages."""
    ng = 3 if recon == "ppm" else 2
    n = (n1, 4, 4)
    dx = (1.0 / n1, 1.0 / 4, 1.0 / 4)
    b = inputs.uniform(n=n, ng=ng, rho=1.0, v=(1.0, 0.0, 0.0), p=0.6, B=(0.0, 0.0, 0.0), dx=dx)
    h = dx[0]
    xl = (np.arange(b.shape[2]) - ng) * h  # lower face of every stored cell (periodic images agree)

    def cell_avg(t):
        # exact average over each cell of 0.5 + 0.4 sin(2 pi (x - t))
        k = 2.0 * math.pi
        return 0.5 - 0.4 * (np.cos(k * (xl + h - t)) - np.cos(k * (xl - t))) / (k * h)

    prim = np.concatenate([b.prim, np.broadcast_to(cell_avg(0.0), b.shape)[None]], axis=0)
    prim = np.ascontiguousarray(prim)
    cfg = orc.make_cfg(n, ng, dx, b.gamma, recon=recon, riemann="hlle", integrator=integrator, cfl=0.4,
                       nscalars=1)
    cons = orc.prim2cons(cfg, prim, b.bface)
    t_end = 0.25
    cons, _, t, _ = orc.run(cfg, cons, b.bface, 0, t_end=t_end)
    g = ng
    got = cons[5][g, g, g:g + n1] / cons[0][g, g, g:g + n1]
    want = cell_avg(t)[g:g + n1]
    return float(np.mean(np.abs(got - want)))


@pytest.mark.parametrize("recon,integrator,order", [("plm", "vl2", 1.8), ("ppm", "rk3", 2.6)])
def test_smooth_advection_converges_at_the_reconstruction_order(orc, recon, integrator, order):
    e = [advect_error(orc, n1, recon, integrator) for n1 in (32, 64, 128)]
    rates = [math.log2(e[i] / e[i + 1]) for i in range(2)]
    assert min(rates) >= order, (e, rates)
