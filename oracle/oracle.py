"""ctypes front end of the CPU oracle (athmhd_oracle.cpp).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark.  The product library never imports it.
Arrays use the block layout of paper_2005_06651_amd.inputs (float64, C order).
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "athmhd_oracle.cpp")
LIB = os.path.join(HERE, "liboracle.so")

RECON = {"dc": 0, "plm": 1, "ppm": 2}
RIEMANN = {"hlle": 0, "hlld": 1, "roe": 2}
INTEGRATOR = {"rk1": 0, "vl2": 1, "rk2": 2, "rk3": 3}


def build(force: bool = False) -> str:
    """Compile the oracle with g++ (plain C++17, no FMA contraction)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        cmd = ["g++", "-std=c++17", "-O2", "-ffp-contract=off", "-fPIC", "-shared",
               "-o", LIB + ".tmp", SRC]
        subprocess.check_call(cmd)
        os.replace(LIB + ".tmp", LIB)
    return LIB


class Cfg(C.Structure):
    _fields_ = [("n1", C.c_int32), ("n2", C.c_int32), ("n3", C.c_int32), ("ng", C.c_int32),
                ("gamma", C.c_double), ("dx1", C.c_double), ("dx2", C.c_double), ("dx3", C.c_double),
                ("recon", C.c_int32), ("riemann", C.c_int32), ("integrator", C.c_int32), ("nscalars", C.c_int32),
                ("cfl", C.c_double), ("ct_eps", C.c_double), ("dfloor", C.c_double), ("pfloor", C.c_double),
                ("charac", C.c_int32), ("pad_", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        P = C.POINTER(C.c_double)
        cp = C.POINTER(Cfg)
        _lib.orc_fill_ghosts.argtypes = [cp, P, P]
        _lib.orc_cons2prim.argtypes = [cp, P, P, P, P]
        _lib.orc_prim2cons.argtypes = [cp, P, P, P]
        _lib.orc_step.argtypes = [cp, P, P, C.c_double]
        _lib.orc_step_jvp.argtypes = [cp, P, P, P, P, C.c_double]
        _lib.orc_newdt.argtypes = [cp, P, P, P]
        _lib.orc_count_ops.argtypes = [cp, P, P, C.c_double, C.POINTER(C.c_ulonglong)]
        _lib.orc_riemann.argtypes = [C.c_int, C.c_double, P, P, C.c_double, P, P]
        _lib.orc_phys_flux.argtypes = [C.c_double, P, C.c_double, P, P]
        _lib.orc_hlld_fan.argtypes = [C.c_double, P, P, C.c_double, P, P]
        _lib.orc_roe_matrix.argtypes = [C.c_double, P, P, C.c_double, P]
        _lib.orc_two_level_step.argtypes = [cp, P, P, C.c_double]
        _lib.orc_two_level_fill.argtypes = [cp, P, P]
        _lib.orc_two_level_newdt.argtypes = [cp, P, P, P]
        _lib.orc_fast_speed.argtypes = [C.c_double] * 6
        _lib.orc_fast_speed.restype = C.c_double
        _lib.orc_recon_line.argtypes = [C.c_int, C.c_int, P, P, P]
        _lib.orc_prim_eigen.argtypes = [C.c_double, P, C.c_double, P, P]
        _lib.orc_char_plm.argtypes = [C.c_double, P, P, P, C.c_double, P, P]
        _lib.orc_char_ppm.argtypes = [C.c_double, P, C.c_double, P, P]
        _lib.orc_restrict.argtypes = [cp, P, P, P, P, C.c_int, C.c_int, C.c_int]
        _lib.orc_prolong.argtypes = [cp, P, P, P, P, C.c_int, C.c_int, C.c_int, C.c_int]
        I3 = C.POINTER(C.c_int)
        _lib.orc_restrict_box.argtypes = [cp, P, P, P, P, I3, I3, I3]
        _lib.orc_prolong_box.argtypes = [cp, P, P, P, P, I3, I3, I3, C.c_int, C.c_int]
        _lib.orc_drive_scalar.argtypes = [C.c_int, C.c_double, C.c_double, C.c_double, C.c_int,
                                          P, P]
        _lib.orc_take_floor_count.restype = C.c_longlong
    return _lib


def _p(a: np.ndarray):
    assert a.dtype == np.float64 and a.flags.c_contiguous
    return a.ctypes.data_as(C.POINTER(C.c_double))


def make_cfg(n, ng, dx, gamma, recon="plm", riemann="hlld", integrator="vl2", cfl=0.3, ct_eps=0.0,
             dfloor=0.0, pfloor=0.0, nscalars=0, charac=False) -> Cfg:
    assert nscalars >= 0
    return Cfg(int(n[0]), int(n[1]), int(n[2]), int(ng), float(gamma), float(dx[0]), float(dx[1]),
               float(dx[2]), RECON[recon], RIEMANN[riemann], INTEGRATOR[integrator], int(nscalars), float(cfl),
               float(ct_eps), float(dfloor), float(pfloor), int(bool(charac)), 0)


def _check(cfg: Cfg, cells: np.ndarray, bface: np.ndarray | None = None) -> None:
    """The C routines index the arrays by the configuration alone: check their
    shapes first (5 MHD variables plus the passive scalars, padded faces)."""
    N = (cfg.n3 + 2 * cfg.ng, cfg.n2 + 2 * cfg.ng, cfg.n1 + 2 * cfg.ng)
    assert cells.shape == (5 + cfg.nscalars,) + N, (cells.shape, cfg.nscalars, N)
    if bface is not None:
        assert bface.shape == (3,) + tuple(x + 1 for x in N), bface.shape


def take_floor_count() -> int:
    """Floor activations (cells and face states) since the previous call."""
    return int(lib().orc_take_floor_count())


def cfg_for(block, **kw) -> Cfg:
    return make_cfg(block.n, block.ng, block.dx, block.gamma, **kw)


def fill_ghosts(cfg: Cfg, cons: np.ndarray, bface: np.ndarray) -> None:
    _check(cfg, cons, bface)
    lib().orc_fill_ghosts(C.byref(cfg), _p(cons), _p(bface))


def prim2cons(cfg: Cfg, prim: np.ndarray, bface: np.ndarray) -> np.ndarray:
    _check(cfg, prim, bface)
    cons = np.empty_like(prim)
    lib().orc_prim2cons(C.byref(cfg), _p(prim), _p(bface), _p(cons))
    return cons


def cons2prim(cfg: Cfg, cons: np.ndarray, bface: np.ndarray):
    _check(cfg, cons, bface)
    prim = np.empty_like(cons)
    bcc = np.empty((3,) + cons.shape[1:])
    bad = lib().orc_cons2prim(C.byref(cfg), _p(cons), _p(bface), _p(prim), _p(bcc))
    return prim, bcc, bad


def step(cfg: Cfg, cons: np.ndarray, bface: np.ndarray, dt: float) -> int:
    """Advance (cons, bface) in place by one step; returns the count of
    non-physical cells met (0 normally), negative on a bad configuration."""
    _check(cfg, cons, bface)
    return lib().orc_step(C.byref(cfg), _p(cons), _p(bface), float(dt))


def step_jvp(cfg: Cfg, cons, bface, dcons, dbface, dt: float) -> int:
    _check(cfg, cons, bface)
    _check(cfg, dcons, dbface)
    return lib().orc_step_jvp(C.byref(cfg), _p(cons), _p(bface), _p(dcons), _p(dbface), float(dt))


def count_ops(cfg: Cfg, cons: np.ndarray, bface: np.ndarray, dt: float):
    """(adds, multiplies, divides, square roots) of one step on this state."""
    _check(cfg, cons, bface)
    out = (C.c_ulonglong * 4)()
    r = lib().orc_count_ops(C.byref(cfg), _p(cons), _p(bface), float(dt), out)
    assert r >= 0
    return tuple(int(x) for x in out)


def newdt(cfg: Cfg, cons: np.ndarray, bface: np.ndarray):
    _check(cfg, cons, bface)
    out = np.zeros(1)
    bad = lib().orc_newdt(C.byref(cfg), _p(cons), _p(bface), _p(out))
    return float(out[0]), bad


def riemann(rs: str, gamma: float, wl, wr, bn: float):
    wl = np.ascontiguousarray(wl, dtype=np.float64)
    wr = np.ascontiguousarray(wr, dtype=np.float64)
    f = np.zeros(7)
    smax = np.zeros(1)
    lib().orc_riemann(RIEMANN[rs], float(gamma), _p(wl), _p(wr), float(bn), _p(f), _p(smax))
    return f, float(smax[0])


def hlld_fan(gamma: float, wl, wr, bn: float):
    """HLLD flux and its fan: (flux, speeds, states) with speeds = (S_L, S*_L,
    S_M, S*_R, S_R, p_T*) and states = (U*_L, U**_L, U**_R, U*_R) in the face
    frame; speeds and states are None when an outer state is upwind."""
    wl = np.ascontiguousarray(wl, dtype=np.float64)
    wr = np.ascontiguousarray(wr, dtype=np.float64)
    f = np.zeros(7)
    out = np.zeros(34)
    rc = lib().orc_hlld_fan(float(gamma), _p(wl), _p(wr), float(bn), _p(f), _p(out))
    if rc:
        return f, None, None
    return f, out[:6].copy(), out[6:].reshape(4, 7).copy()


def two_level_step(cfg: Cfg, cons, bface, dt: float) -> int:
    """One step of the two-level composite (nine blocks, in place); cfg is the
    coarse block's configuration."""
    assert cons.flags.c_contiguous and bface.flags.c_contiguous
    return lib().orc_two_level_step(C.byref(cfg), _p(cons), _p(bface), float(dt))


def two_level_fill(cfg: Cfg, cons, bface) -> int:
    return lib().orc_two_level_fill(C.byref(cfg), _p(cons), _p(bface))


def two_level_newdt(cfg: Cfg, cons, bface):
    out = np.zeros(1)
    bad = lib().orc_two_level_newdt(C.byref(cfg), _p(cons), _p(bface), _p(out))
    return float(out[0]), bad


def roe_matrix(gamma: float, wl, wr, bn: float):
    """Roe matrix of the pair (7 x 7, face frame)."""
    wl = np.ascontiguousarray(wl, dtype=np.float64)
    wr = np.ascontiguousarray(wr, dtype=np.float64)
    a = np.zeros(49)
    lib().orc_roe_matrix(float(gamma), _p(wl), _p(wr), float(bn), _p(a))
    return a.reshape(7, 7)


def phys_flux(gamma: float, w, bn: float):
    w = np.ascontiguousarray(w, dtype=np.float64)
    u = np.zeros(7)
    f = np.zeros(7)
    lib().orc_phys_flux(float(gamma), _p(w), float(bn), _p(u), _p(f))
    return u, f


def fast_speed(rho, p, bn, bt1, bt2, gamma) -> float:
    return lib().orc_fast_speed(rho, p, bn, bt1, bt2, gamma)


def recon_line(recon: str, q):
    q = np.ascontiguousarray(q, dtype=np.float64)
    ql = np.full_like(q, np.nan)
    qr = np.full_like(q, np.nan)
    lib().orc_recon_line(RECON[recon], len(q), _p(q), _p(ql), _p(qr))
    return ql, qr


def prim_eigen(gamma: float, w, bn: float):
    """(R, L): right eigenvectors as columns and their inverse, for the
    face-frame primitive state w = (rho, vn, vt1, vt2, P, Bt1, Bt2)."""
    w = np.ascontiguousarray(w, dtype=np.float64)
    R = np.zeros((7, 7))
    L = np.zeros((7, 7))
    lib().orc_prim_eigen(float(gamma), _p(w), float(bn), _p(R), _p(L))
    return R, L


def char_plm(gamma: float, wm, w0, wp, bn: float):
    """Characteristic PLM (left, right) edge states of the cell w0."""
    wm, w0, wp = (np.ascontiguousarray(x, dtype=np.float64) for x in (wm, w0, wp))
    left, right = np.zeros(7), np.zeros(7)
    lib().orc_char_plm(float(gamma), _p(wm), _p(w0), _p(wp), float(bn), _p(left), _p(right))
    return left, right


def char_ppm(gamma: float, stencil, bn: float):
    """Characteristic PPM (left, right) edge states of the middle cell of a
    five-cell stencil (5 x 7 face-frame primitives)."""
    st = np.ascontiguousarray(stencil, dtype=np.float64)
    assert st.shape == (5, 7)
    left, right = np.zeros(7), np.zeros(7)
    lib().orc_char_ppm(float(gamma), _p(st), float(bn), _p(left), _p(right))
    return left, right


def restrict(cfg: Cfg, fcons, fbface, ccons, cbface, octant) -> None:
    """Restrict the fine block into octant (ox, oy, oz) of the coarse block
    (in place in ccons, cbface)."""
    for x, y in ((fcons, fbface), (ccons, cbface)):
        _check(cfg, x, y)
    lib().orc_restrict(C.byref(cfg), _p(fcons), _p(fbface), _p(ccons), _p(cbface), *[int(v) for v in octant])


def prolong(cfg: Cfg, ccons, cbface, fcons, fbface, octant, primitive: bool = False) -> None:
    """Prolong octant (ox, oy, oz) of the coarse block into the fine block (in
    place in fcons, fbface); primitive=True prolongs the primitives and
    converts back."""
    for x, y in ((fcons, fbface), (ccons, cbface)):
        _check(cfg, x, y)
    lib().orc_prolong(C.byref(cfg), _p(ccons), _p(cbface), _p(fcons), _p(fbface), *[int(v) for v in octant],
                      int(bool(primitive)))


def _box(flo, clo, ext, cfg=None, prolong=False):
    """The three boxes as C arrays, after checking that every index the C
    routine touches lies in the stored arrays (the C code does not check)."""
    if cfg is not None:
        N = (cfg.n1 + 2 * cfg.ng, cfg.n2 + 2 * cfg.ng, cfg.n3 + 2 * cfg.ng)
        for d in range(3):
            assert ext[d] >= 1 and flo[d] >= 0 and flo[d] + 2 * ext[d] <= N[d], (flo, ext, N)
            lo, hi = (1, N[d] - 1) if prolong else (0, N[d])
            assert clo[d] >= lo and clo[d] + ext[d] <= hi, (clo, ext, N, prolong)
    return [(C.c_int * 3)(*[int(x) for x in v]) for v in (flo, clo, ext)]


def restrict_box(cfg: Cfg, fcons, fbface, ccons, cbface, flo, clo, ext) -> None:
    """Restrict fine cells [flo, flo + 2 ext) (stored (x1, x2, x3) indices,
    ghosts included) onto coarse cells [clo, clo + ext), in place."""
    for x, y in ((fcons, fbface), (ccons, cbface)):
        _check(cfg, x, y)
    lib().orc_restrict_box(C.byref(cfg), _p(fcons), _p(fbface), _p(ccons), _p(cbface), *_box(flo, clo, ext, cfg))


def prolong_box(cfg: Cfg, ccons, cbface, fcons, fbface, flo, clo, ext, primitive: bool = False,
                keep: int = 0) -> None:
    """Prolong coarse cells [clo, clo + ext) onto fine cells [flo, flo + 2 ext)
    and their faces, in place; keep bit 2 d + S keeps the fine faces already
    on side S of the box along direction d."""
    for x, y in ((fcons, fbface), (ccons, cbface)):
        _check(cfg, x, y)
    assert 0 <= keep <= 63, keep
    lib().orc_prolong_box(C.byref(cfg), _p(ccons), _p(cbface), _p(fcons), _p(fbface),
                          *_box(flo, clo, ext, cfg, prolong=True), int(bool(primitive)), int(keep))


def drive_scalar(integrator: str, lam: complex, dt: float, nsteps: int) -> complex:
    re = np.zeros(1)
    im = np.zeros(1)
    r = lib().orc_drive_scalar(INTEGRATOR[integrator], lam.real, lam.imag, dt, nsteps, _p(re), _p(im))
    assert r == 0
    return complex(re[0], im[0])


def run(cfg: Cfg, cons, bface, nsteps: int, dt: float | None = None, t_end: float | None = None):
    """Advance nsteps (or up to t_end) with dt from newdt unless dt is given.
    Returns (cons, bface, t, steps)."""
    cons = np.array(cons, dtype=np.float64, order="C", copy=True)
    bface = np.array(bface, dtype=np.float64, order="C", copy=True)
    t = 0.0
    it = 0
    while True:
        if t_end is not None and t >= t_end * (1 - 1e-14):
            break
        if t_end is None and it >= nsteps:
            break
        h = dt
        if h is None:
            h, bad = newdt(cfg, cons, bface)
            assert bad == 0
        if t_end is not None:
            h = min(h, t_end - t)
        bad = step(cfg, cons, bface, h)
        if bad != 0:
            raise FloatingPointError(f"oracle step reported {bad} non-physical cells")
        t += h
        it += 1
    return cons, bface, t, it
