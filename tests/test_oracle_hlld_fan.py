"""Pins of the oracle's HLLD solver away from the special states where its
intermediate-state corrections vanish (Sec. 3.2.2; Miyoshi & Kusano 2005).

The HLLD fan is defined by jump conditions, not by a closed formula: four
intermediate states separated by the waves S_L < S*_L <= S_M <= S*_R < S_R,
with one normal velocity S_M and one total pressure p_T* across the whole fan,
density unchanged across the rotational waves S*_L, S*_R, which move at the
Alfven speed of the density beside them, and transverse velocity and field
continuous across the contact S_M.  Across every wave the Rankine-Hugoniot
conditions of Eq. (cons) hold.  These tests check exactly those relations on
random general states (B_x != 0, sheared transverse velocity and field,
different densities and pressures), where every correction term of the star
and double-star states is active; the physical fluxes are written out here
from Eq. (cons), independently of the oracle.
"""
import math

import numpy as np
import pytest

GAM = 5.0 / 3.0


def cons_of(w, bx, g=GAM):
    rho, u, v, ww, p, by, bz = w
    e = p / (g - 1) + 0.5 * rho * (u * u + v * v + ww * ww) + 0.5 * (bx * bx + by * by + bz * bz)
    return np.array([rho, rho * u, rho * v, rho * ww, e, by, bz])


def flux_of(u, bx, ptot):
    """Flux of Eq. (cons) in the face frame for a conserved state u = (rho,
    M_n, M_t1, M_t2, E, B_t1, B_t2) whose total pressure is ptot."""
    rho, mn, m1, m2, e, by, bz = u
    vn, v1, v2 = mn / rho, m1 / rho, m2 / rho
    vb = vn * bx + v1 * by + v2 * bz
    return np.array([mn, mn * vn + ptot - bx * bx, mn * v1 - bx * by, mn * v2 - bx * bz,
                     (e + ptot) * vn - bx * vb, by * vn - bx * v1, bz * vn - bx * v2])


def ptot_of(w, bx):
    return w[4] + 0.5 * (bx * bx + w[5] ** 2 + w[6] ** 2)


def general_pair(rng):
    wl = np.array([rng.uniform(0.3, 3.0), rng.uniform(-0.8, 0.8), rng.uniform(-1, 1), rng.uniform(-1, 1),
                   rng.uniform(0.2, 3.0), rng.uniform(-1.5, 1.5), rng.uniform(-1.5, 1.5)])
    wr = np.array([rng.uniform(0.3, 3.0), rng.uniform(-0.8, 0.8), rng.uniform(-1, 1), rng.uniform(-1, 1),
                   rng.uniform(0.2, 3.0), rng.uniform(-1.5, 1.5), rng.uniform(-1.5, 1.5)])
    bx = rng.choice([-1.0, 1.0]) * rng.uniform(0.2, 1.6)
    return wl, wr, bx


def jump_residual(s, ua, ub, fa, fb):
    """max |S (U_b - U_a) - (F_b - F_a)| relative to the size of its terms"""
    res = s * (ub - ua) - (fb - fa)
    scale = np.max(np.abs(s) * (np.abs(ua) + np.abs(ub)) + np.abs(fa) + np.abs(fb))
    return float(np.max(np.abs(res)) / scale)


def fan_residuals(orc, wl, wr, bx):
    """Every defining relation of the HLLD fan of (wl, wr, bx); returns the
    worst relative residual per relation, or None if no fan forms."""
    f, sp, st = orc.hlld_fan(GAM, wl, wr, bx)
    if sp is None:
        return None
    sl, ssl, sm, ssr, sr, pts = sp
    usl, ussl, ussr, usr = st
    ul, ur = cons_of(wl, bx), cons_of(wr, bx)
    fl, fr = flux_of(ul, bx, ptot_of(wl, bx)), flux_of(ur, bx, ptot_of(wr, bx))
    fsl, fssl, fssr, fsr = (flux_of(u, bx, pts) for u in (usl, ussl, ussr, usr))
    out = {}
    # ordering of the waves (the rotational waves may coincide with the outer
    # ones, or with the contact when B_x = 0)
    vscale = abs(sl) + abs(sr)
    slack = 1e-13 * vscale
    out["order"] = 0.0 if (sl - slack <= ssl <= sm <= ssr <= sr + slack and sl < sm < sr) else 1.0
    # one normal velocity in the fan
    out["normal velocity"] = max(abs(u[1] / u[0] - sm) for u in st) / vscale
    # density unchanged across the rotational waves, which move at the Alfven
    # speed of that density
    out["rho across S*"] = max(abs(ussl[0] - usl[0]) / usl[0], abs(ussr[0] - usr[0]) / usr[0])
    out["Alfven speeds"] = max(abs(ssl - (sm - abs(bx) / math.sqrt(usl[0]))),
                               abs(ssr - (sm + abs(bx) / math.sqrt(usr[0])))) / vscale
    # transverse velocity and field continuous across the contact
    vt = [np.array([u[2] / u[0], u[3] / u[0]]) for u in (ussl, ussr)]
    bt = [ussl[5:7], ussr[5:7]]
    out["contact"] = float(max(np.max(np.abs(vt[0] - vt[1])) / vscale,
                               np.max(np.abs(bt[0] - bt[1])) / (np.max(np.abs(bt)) + abs(bx))))
    # Rankine-Hugoniot across each of the five waves
    out["RH S_L"] = jump_residual(sl, ul, usl, fl, fsl)
    out["RH S*_L"] = jump_residual(ssl, usl, ussl, fsl, fssl)
    out["RH S_M"] = jump_residual(sm, ussl, ussr, fssl, fssr)
    out["RH S*_R"] = jump_residual(ssr, ussr, usr, fssr, fsr)
    out["RH S_R"] = jump_residual(sr, usr, ur, fsr, fr)
    # the flux is that of the state found at x/t = 0
    if ssl >= 0.0:
        fz = fsl
    elif ssr <= 0.0:
        fz = fsr
    elif sm >= 0.0:
        fz = fssl
    else:
        fz = fssr
    out["flux at x/t=0"] = float(np.max(np.abs(f - fz)) / np.max(np.abs(fl) + np.abs(fr)))
    # integral consistency: the fan's width-weighted states sum to the HLL
    # average times the fan's width
    lhs = (ssl - sl) * usl + (sm - ssl) * ussl + (ssr - sm) * ussr + (sr - ssr) * usr
    rhs = sr * ur - sl * ul - (fr - fl)
    out["integral"] = float(np.max(np.abs(lhs - rhs)) / np.max(np.abs(sr * ur) + np.abs(sl * ul) + np.abs(fr - fl)))
    return out


TOL = 1e-13


def test_hlld_fan_jump_conditions_general_states(orc):
    """All defining relations of the HLLD fan hold on 600 random general
    states; every region of the fan occurs among them."""
    rng = np.random.default_rng(2024)
    worst = {}
    regions = set()
    n = 0
    while n < 600:
        wl, wr, bx = general_pair(rng)
        res = fan_residuals(orc, wl, wr, bx)
        if res is None:
            continue
        n += 1
        for k, v in res.items():
            worst[k] = max(worst.get(k, 0.0), v)
        _, sp, _ = orc.hlld_fan(GAM, wl, wr, bx)
        sl, ssl, sm, ssr, sr, _ = sp
        regions.add("*L" if ssl >= 0 else "*R" if ssr <= 0 else "**L" if sm >= 0 else "**R")
    bad = {k: v for k, v in worst.items() if not v <= TOL}
    assert not bad, bad
    assert regions == {"*L", "*R", "**L", "**R"}, regions


@pytest.mark.parametrize("side", ["left", "right"])
def test_hlld_outer_star_state_from_flux(orc, side):
    """In the outer star regions (S_L < 0 <= S*_L, and its mirror) the returned
    flux alone fixes the star state through the jump condition across the
    outer wave, U* = U_a + (F - F_a)/S_a, with S_a from the wave-speed
    estimate S_L = min(u_L, u_R) - max(c_fL, c_fR) (mirror: S_R).  That state
    must then carry the flux itself: mass flux rho* S_M with S_M its normal
    velocity, transverse momentum and field fluxes and the energy flux of
    Eq. (cons) at the total pressure p_T* implied by the normal-momentum flux,
    and the same p_T* must follow from the jump conditions on the other side
    (uniform total pressure across the fan)."""
    rng = np.random.default_rng(77 if side == "left" else 78)
    hits = 0
    worst = 0.0
    for _ in range(3000):
        wl, wr, bx = general_pair(rng)
        if side == "left":
            wl[1], wr[1] = abs(wl[1]) + 0.3, abs(wr[1]) + 0.3  # fan mostly to the right
        else:
            wl[1], wr[1] = -abs(wl[1]) - 0.3, -abs(wr[1]) - 0.3
        f, _ = orc.riemann("hlld", GAM, wl, wr, bx)
        cl = orc.fast_speed(wl[0], wl[4], bx, wl[5], wl[6], GAM)
        cr = orc.fast_speed(wr[0], wr[4], bx, wr[5], wr[6], GAM)
        sl = min(wl[1], wr[1]) - max(cl, cr)
        sr = max(wl[1], wr[1]) + max(cl, cr)
        if not (sl < 0.0 < sr):
            continue
        wa, wb, sa, sb = (wl, wr, sl, sr) if side == "left" else (wr, wl, sr, sl)
        ua = cons_of(wa, bx)
        fa = flux_of(ua, bx, ptot_of(wa, bx))
        us = ua + (f - fa) / sa
        rho_s = us[0]
        sm = us[1] / rho_s
        # the outer star state lies between the outer wave and the rotational
        # wave on its side: keep the cases where x/t = 0 is in it
        ss = sm - abs(bx) / math.sqrt(rho_s) if side == "left" else sm + abs(bx) / math.sqrt(rho_s)
        if not ((ss >= 0.0) if side == "left" else (ss <= 0.0)):
            continue
        hits += 1
        pts = f[1] - rho_s * sm * sm + bx * bx
        # the other side: mass and normal momentum jump at S_b with the same
        # S_M give its star density and p_T*
        rho_b = wb[0] * (sb - wb[1]) / (sb - sm)
        pts_b = sb * (rho_b * sm - wb[0] * wb[1]) - rho_b * sm * sm + wb[0] * wb[1] ** 2 + ptot_of(wb, bx)
        fs = flux_of(us, bx, pts)
        scale = np.max(np.abs(f)) + np.max(np.abs(fa))
        worst = max(worst, float(np.max(np.abs(fs - f)) / scale), abs(pts - pts_b) / abs(pts))
    assert hits >= 200, hits
    assert worst <= TOL, worst


@pytest.mark.parametrize("bx", [2.5, -3.0])
@pytest.mark.parametrize("u", [0.15, -0.2])
def test_hlld_degenerate_shear_is_linear_alfven(orc, bx, u):
    """A field along the normal with c_A > a and no transverse field, and a jump
    in the transverse velocity only: the star denominators
    rho (S - u)(S - S_M) - B_x^2 vanish (the fast and Alfven waves coincide), so
    the degenerate branch is taken.  The transverse momentum and field fluxes
    must equal those of the linear Alfven-wave solution of this shear (middle
    state v_t = (v_L + v_R)/2, B_t = sign(B_x) sqrt(rho) (v_R - v_L)/2), and
    every jump condition of the fan must hold."""
    rho, p = 1.2, 0.3
    assert bx * bx / rho > GAM * p / rho
    for amp in (1e-3, 0.1, 0.4):
        wl = np.array([rho, u, 0.2 + amp, -0.1 - 0.5 * amp, p, 0.0, 0.0])
        wr = np.array([rho, u, 0.2 - amp, -0.1 + 0.5 * amp, p, 0.0, 0.0])
        res = fan_residuals(orc, wl, wr, bx)
        bad = {k: v for k, v in res.items() if not v <= TOL}
        assert not bad, (amp, bad)
        f, _ = orc.riemann("hlld", GAM, wl, wr, bx)
        vm = 0.5 * (wl[2:4] + wr[2:4])
        bm = math.copysign(1.0, bx) * math.sqrt(rho) * 0.5 * (wr[2:4] - wl[2:4])
        lin_m = rho * u * vm - bx * bm
        lin_b = bm * u - bx * vm
        assert np.max(np.abs(f[2:4] - lin_m)) < 1e-14 * (1 + abs(bx))
        assert np.max(np.abs(f[5:7] - lin_b)) < 1e-14 * (1 + abs(bx))


@pytest.mark.parametrize("seed", [5, 6])
def test_hlld_vanishing_normal_field(orc, seed):
    """B_x = 0 with jumping transverse fields: the rotational waves collapse
    onto the contact and the fan has three waves; the jump conditions still
    hold with the double-star states equal to the single-star ones.  The
    contact is then a tangential discontinuity, across which the transverse
    velocity and field may jump."""
    rng = np.random.default_rng(seed)
    for _ in range(200):
        wl, wr, _ = general_pair(rng)
        res = fan_residuals(orc, wl, wr, 0.0)
        if res is None:
            continue
        res.pop("order")  # S*_L = S_M = S*_R here
        res.pop("contact")
        bad = {k: v for k, v in res.items() if not v <= TOL}
        assert not bad, bad
