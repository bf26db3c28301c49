"""Pins of the oracle's Roe solver (Sec. 3.2.2 names Roe's linearised solver;
reading R-34 for its averages).

A Roe matrix A of a pair of states is defined by three properties: it maps
the jump of the conserved state onto the jump of the flux,
A (U_R - U_L) = F_R - F_L; it is diagonalisable with real eigenvalues; and it
reduces to the flux Jacobian when U_L = U_R.  The first property makes the
solver resolve any isolated discontinuity that satisfies the
Rankine-Hugoniot conditions of Eq. (cons) exactly.  The physical fluxes here
are written out from Eq. (cons), independently of the oracle.
"""
import math

import numpy as np
import pytest

from test_oracle_pins import exact_cons, exact_flux, random_state

GAM = 5.0 / 3.0


def pair(rng, bx_zero=False, bt_zero=False):
    wl, wr = random_state(rng), random_state(rng)
    if bt_zero:
        wl[5:] = 0.0
        wr[5:] = 0.0
    bx = 0.0 if bx_zero else rng.uniform(-1.5, 1.5)
    return wl, wr, bx


@pytest.mark.parametrize("bx_zero,bt_zero", [(False, False), (True, False), (False, True), (True, True)])
def test_roe_matrix_maps_state_jump_to_flux_jump(orc, bx_zero, bt_zero):
    """A (U_R - U_L) = F_R - F_L on random pairs, including a vanishing normal
    or transverse field."""
    rng = np.random.default_rng(31 + 2 * bx_zero + bt_zero)
    for _ in range(400):
        wl, wr, bx = pair(rng, bx_zero, bt_zero)
        A = orc.roe_matrix(GAM, wl, wr, bx)
        du = exact_cons(wr, bx) - exact_cons(wl, bx)
        df = exact_flux(wr, bx) - exact_flux(wl, bx)
        assert np.max(np.abs(A @ du - df)) <= 1e-14 * (np.max(np.abs(A)) * np.max(np.abs(du)) + np.max(np.abs(df)))


def test_roe_matrix_is_the_jacobian_for_equal_states(orc):
    """U_L = U_R: A is the flux Jacobian dF/dU, checked by central differences
    of the physical flux in the conserved variables."""
    rng = np.random.default_rng(35)
    for _ in range(50):
        w = random_state(rng)
        bx = rng.uniform(-1.5, 1.5)
        A = orc.roe_matrix(GAM, w, w, bx)
        u0 = exact_cons(w, bx)
        J = np.zeros((7, 7))
        for c in range(7):
            h = 1e-6 * max(1.0, abs(u0[c]))
            cols = []
            for sgn in (1.0, -1.0):
                u = u0.copy()
                u[c] += sgn * h
                rho, m, e, bt = u[0], u[1:4], u[4], u[5:7]
                v = m / rho
                p = (GAM - 1) * (e - 0.5 * rho * v @ v - 0.5 * (bx * bx + bt @ bt))
                cols.append(exact_flux(np.array([rho, *v, p, *bt]), bx))
            J[:, c] = (cols[0] - cols[1]) / (2 * h)
        assert np.max(np.abs(A - J)) <= 1e-7 * max(1.0, np.max(np.abs(J)))


def test_roe_matrix_is_hyperbolic_with_the_averaged_wave_speeds(orc):
    """Real eigenvalues: u, u +- b_x, u +- c_f, u +- c_s of the averaged state,
    c_f and c_s the fast and slow speeds for the sound speed
    a^2 = (gamma-1)(H - |v|^2/2 - |B|^2/rho) - (gamma-2) X and b = B/sqrt(rho)
    (the averages of reading R-34).  numpy's eigenvalue routine is the
    reference."""
    rng = np.random.default_rng(36)
    for it in range(300):
        wl, wr, bx = pair(rng, bt_zero=(it % 5 == 0))
        A = orc.roe_matrix(GAM, wl, wr, bx)
        ev = np.linalg.eigvals(A)
        sl, sr = math.sqrt(wl[0]), math.sqrt(wr[0])
        D = sl + sr
        rho = sl * sr
        v = (sl * wl[1:4] + sr * wr[1:4]) / D
        hl = (exact_cons(wl, bx)[4] + wl[4] + 0.5 * (bx * bx + wl[5:] @ wl[5:])) / wl[0]
        hr = (exact_cons(wr, bx)[4] + wr[4] + 0.5 * (bx * bx + wr[5:] @ wr[5:])) / wr[0]
        H = (sl * hl + sr * hr) / D
        bt = (sr * wl[5:] + sl * wr[5:]) / D
        X = (wr[5:] - wl[5:]) @ (wr[5:] - wl[5:]) / (2 * D * D)
        a2 = (GAM - 1) * (H - 0.5 * v @ v - (bx * bx + bt @ bt) / rho) - (GAM - 2) * X
        assert a2 > 0
        bx2, bt2 = bx * bx / rho, bt @ bt / rho
        s = a2 + bx2 + bt2
        disc = math.sqrt(max(s * s - 4 * a2 * bx2, 0.0))
        cf, cs = math.sqrt(0.5 * (s + disc)), math.sqrt(max(0.5 * (s - disc), 0.0))
        lam = np.sort([v[0], v[0] - math.sqrt(bx2), v[0] + math.sqrt(bx2), v[0] - cf, v[0] + cf, v[0] - cs, v[0] + cs])
        assert np.max(np.abs(ev.imag)) <= 1e-7 * cf
        assert np.max(np.abs(np.sort(ev.real) - lam)) <= 1e-7 * cf


def test_roe_consistency(orc):
    rng = np.random.default_rng(37)
    for _ in range(300):
        w = random_state(rng)
        bx = rng.uniform(-1.5, 1.5)
        f, _ = orc.riemann("roe", GAM, w, w, bx)
        assert np.max(np.abs(f - exact_flux(w, bx))) <= 1e-14 * np.max(np.abs(exact_flux(w, bx)))


def test_roe_supersonic_is_upwind(orc):
    """Every eigenvalue of the Roe matrix positive (negative): |A| = A (-A), so
    the flux is F_L (F_R) up to rounding."""
    rng = np.random.default_rng(38)
    n = 0
    for _ in range(400):
        wl, wr, bx = pair(rng)
        sgn = rng.choice([-1.0, 1.0])
        wl[1] = sgn * (abs(wl[1]) + 4.0)
        wr[1] = sgn * (abs(wr[1]) + 4.0)
        ev = np.linalg.eigvals(orc.roe_matrix(GAM, wl, wr, bx)).real
        if not (np.all(ev > 0) or np.all(ev < 0)):
            continue
        n += 1
        f, _ = orc.riemann("roe", GAM, wl, wr, bx)
        up = wl if ev[0] > 0 else wr
        ref = exact_flux(up, bx)
        assert np.max(np.abs(f - ref)) <= 1e-12 * np.max(np.abs(ref))
    assert n > 300


@pytest.mark.parametrize("u", [0.0, 0.37, -0.52])
def test_roe_resolves_contact(orc, u):
    wl = np.array([1.7, u, 0.3, -0.2, 0.9, 0.6, -0.4])
    wr = wl.copy()
    wr[0] = 0.45
    for bx in (0.8, -1.3, 0.0):
        f, _ = orc.riemann("roe", GAM, wl, wr, bx)
        up = wl if u >= 0 else wr
        ref = exact_flux(up, bx)
        assert np.max(np.abs(f - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("u", [0.21, -0.33])
def test_roe_resolves_tangential_discontinuity(orc, u):
    wl = np.array([1.3, u, 0.4, -0.1, 1.0, 0.8, 0.2])
    wr = np.array([0.6, u, -0.7, 0.5, 0.0, -0.3, 0.9])
    wr[4] = wl[4] + 0.5 * (wl[5] ** 2 + wl[6] ** 2) - 0.5 * (wr[5] ** 2 + wr[6] ** 2)
    f, _ = orc.riemann("roe", GAM, wl, wr, 0.0)
    up = wl if u >= 0 else wr
    ref = exact_flux(up, 0.0)
    assert np.max(np.abs(f - ref)) <= 1e-13 * np.max(np.abs(ref))


@pytest.mark.parametrize("bx", [1.1, -0.7])
@pytest.mark.parametrize("side", [-1, 1])
@pytest.mark.parametrize("u", [0.4, -0.9])
def test_roe_resolves_rotational_discontinuity(orc, bx, side, u):
    """The rotational discontinuity of the HLLD pins: it satisfies the jump
    conditions, so it is an eigenvector of the Roe matrix and the flux is the
    upwind one."""
    rho, p, bt = 1.4, 0.8, 0.9
    th_l, th_r = 0.3, 2.1
    byl, bzl = bt * math.cos(th_l), bt * math.sin(th_l)
    byr, bzr = bt * math.cos(th_r), bt * math.sin(th_r)
    vyl, vzl = 0.2, -0.3
    s_minus_u = side * abs(bx) / math.sqrt(rho)
    vyr = vyl - s_minus_u * (byr - byl) / bx
    vzr = vzl - s_minus_u * (bzr - bzl) / bx
    wl = np.array([rho, u, vyl, vzl, p, byl, bzl])
    wr = np.array([rho, u, vyr, vzr, p, byr, bzr])
    S = u + s_minus_u
    f, _ = orc.riemann("roe", GAM, wl, wr, bx)
    ref = exact_flux(wl if S > 0 else wr, bx)
    assert np.max(np.abs(f - ref)) <= 1e-13 * np.max(np.abs(ref))


def test_roe_mirror_symmetry(orc):
    rng = np.random.default_rng(39)
    M = np.array([1, -1, 1, 1, 1, 1, 1.0])
    for _ in range(300):
        wl, wr, bx = pair(rng)
        f, _ = orc.riemann("roe", GAM, wl, wr, bx)
        ml, mr = wl.copy(), wr.copy()
        ml[1] *= -1
        mr[1] *= -1
        g, _ = orc.riemann("roe", GAM, mr, ml, -bx)
        assert np.max(np.abs(g + M * f)) <= 1e-13 * max(1.0, np.max(np.abs(f)))


@pytest.mark.slow
def test_roe_linear_wave_converges(orc):
    """Fast linear wave (Sec. 3.3.1, Eq. RMS-error) with VL2 + PLM + Roe: the
    error after one period falls by at least 2^1.8 from N = 8 to N = 16."""
    from paper_2005_06651_amd import inputs
    errs = []
    for N in (8, 16):
        b = inputs.linear_wave(N)
        cfg = orc.cfg_for(b, integrator="vl2", recon="plm", riemann="roe", cfl=0.3)
        c, bf, t, _ = orc.run(cfg, b.cons, b.bface, 0, t_end=0.5)
        a = b.active
        errs.append(math.sqrt(sum(np.mean(np.abs(c[v][a] - b.cons[v][a])) ** 2 for v in range(5))))
    order = math.log2(errs[0] / errs[1])
    assert order >= 1.8, (errs, order)
