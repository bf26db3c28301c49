"""Seeded synthetic inputs for the MHD step.

This module only builds initial states: primitive or conserved cell fields and
face-averaged magnetic fields on the block layout.  It holds none of the
solver's arithmetic (no reconstruction, Riemann solver, EMF or update), so both
the HIP library and the CPU oracle can be fed from it.

Layout (shared by every producer and consumer of block data):
  cell arrays  [v][k][j][i], shape (nv, N3, N2, N1), N_d = n_d + 2*ng, i fastest
  face arrays  [c][k][j][i], shape (3, N3+1, N2+1, N1+1); component c at index
               (k, j, i) is the face on the lower side of cell (k, j, i) along c.
Ghost entries are the periodic images of active entries: every value is
evaluated at the coordinates of the image, so ghosts match their source bitwise.

Face fields come from a vector potential: each face value is the circulation of
A around the face (Stokes) divided by the face area, with every edge integral
computed once and shared by the faces that meet at that edge.  The discrete
divergence then telescopes to round-off.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np


@dataclass
class Block:
    n: tuple            # active cells (n1, n2, n3)
    ng: int
    dx: tuple           # (dx1, dx2, dx3)
    gamma: float
    bface: np.ndarray   # (3, N3+1, N2+1, N1+1)
    prim: np.ndarray | None = None   # (5 + ns, N3, N2, N1): rho, v1, v2, v3, p, then scalars C_i
    cons: np.ndarray | None = None   # (5 + ns, N3, N2, N1): rho, M1, M2, M3, E, then rho C_i
    meta: dict = field(default_factory=dict)

    @property
    def shape(self):
        n1, n2, n3 = self.n
        return (n3 + 2 * self.ng, n2 + 2 * self.ng, n1 + 2 * self.ng)

    @property
    def active(self):
        """Slices of the active cells of a cell array (last three axes)."""
        g = self.ng
        n1, n2, n3 = self.n
        return (slice(g, g + n3), slice(g, g + n2), slice(g, g + n1))


def _wrapped_index(N: int, n: int, ng: int) -> np.ndarray:
    """Active index of the periodic image of every stored index 0..N-1."""
    idx = np.arange(N)
    return ng + np.mod(idx - ng, n)


def _cell_centres(n: int, ng: int, h: float, extra: int = 0) -> np.ndarray:
    """Coordinate of the cell centre of the periodic image of every stored index
    (extra=1 adds the padded entry of face arrays)."""
    N = n + 2 * ng + extra
    return (_wrapped_index(N, n, ng) - ng + 0.5) * h


def _lower_faces(n: int, ng: int, h: float, extra: int = 1) -> np.ndarray:
    N = n + 2 * ng + extra
    return (_wrapped_index(N, n, ng) - ng) * h


# ---------------------------------------------------------------------------
# Face fields from a vector potential given as a sum of Fourier modes
#   A(x) = sum_m  a_m * sin(k_m . x + phi_m)
# Edge integrals of each mode are closed-form.
# ---------------------------------------------------------------------------
def _edge_integral(kd, x0, h, theta):
    """Integral over [x0, x0+h] of sin(kd*x + theta) dx (arrays broadcast)."""
    if abs(kd) < 1e-300:
        return h * np.sin(theta + 0.0 * x0)
    return (np.cos(kd * x0 + theta) - np.cos(kd * (x0 + h) + theta)) / kd


def faces_from_modes(n, ng, dx, modes):
    """Face-averaged B of curl A for A = sum a sin(k.x + phi) (modes = list of
    (k(3), a(3), phi)).  Returns (3, N3+1, N2+1, N1+1)."""
    n1, n2, n3 = n
    h1, h2, h3 = dx
    # coordinates along each axis, padded length N+1, of the periodic images
    xc = [_cell_centres(n1, ng, h1, 1), _cell_centres(n2, ng, h2, 1), _cell_centres(n3, ng, h3, 1)]
    xf = [_lower_faces(n1, ng, h1), _lower_faces(n2, ng, h2), _lower_faces(n3, ng, h3)]
    shp = (n3 + 2 * ng + 1, n2 + 2 * ng + 1, n1 + 2 * ng + 1)
    # G1: integral of A_x along x over cell i, at (y_{j-1/2}, z_{k-1/2}); G2, G3 alike
    G1 = np.zeros(shp)
    G2 = np.zeros(shp)
    G3 = np.zeros(shp)
    X1f, X2f, X3f = xf[0][None, None, :], xf[1][None, :, None], xf[2][:, None, None]
    for k, a, phi in modes:
        k1, k2, k3 = k
        if a[0] != 0.0:
            G1 += a[0] * _edge_integral(k1, X1f, h1, k2 * X2f + k3 * X3f + phi)
        if a[1] != 0.0:
            G2 += a[1] * _edge_integral(k2, X2f, h2, k1 * X1f + k3 * X3f + phi)
        if a[2] != 0.0:
            G3 += a[2] * _edge_integral(k3, X3f, h3, k1 * X1f + k2 * X2f + phi)
    return _faces_from_edges(G1, G2, G3, n, ng, dx)


def _faces_from_edges(G1, G2, G3, n, ng, dx):
    """Circulation around each face / area.  The G arrays live on the padded
    grid; neighbours one index up are taken at the periodic image index so the
    last padded entry stays consistent."""
    n1, n2, n3 = n
    h1, h2, h3 = dx
    N1, N2, N3 = n1 + 2 * ng, n2 + 2 * ng, n3 + 2 * ng
    up1 = _wrapped_index(N1 + 2, n1, ng)[1:N1 + 2]   # image of index+1
    up2 = _wrapped_index(N2 + 2, n2, ng)[1:N2 + 2]
    up3 = _wrapped_index(N3 + 2, n3, ng)[1:N3 + 2]
    B = np.zeros((3,) + G1.shape)
    # B1 at (i-1/2, j, k): G3(i-1/2, j+1/2, k) - G3(i-1/2, j-1/2, k) - G2(i-1/2, j, k+1/2) + G2(i-1/2, j, k-1/2)
    B[0] = (G3[:, up2, :] - G3 - G2[up3, :, :] + G2) / (h2 * h3)
    # B2 at (i, j-1/2, k): G1(k+1/2) - G1(k-1/2) - G3(i+1/2) + G3(i-1/2)
    B[1] = (G1[up3, :, :] - G1 - G3[:, :, up1] + G3) / (h3 * h1)
    # B3 at (i, j, k-1/2): G2(i+1/2) - G2(i-1/2) - G1(j+1/2) + G1(j-1/2)
    B[2] = (G2[:, :, up1] - G2 - G1[:, up2, :] + G1) / (h1 * h2)
    return B


def _spectral_edges(n, ng, dx, L, Ahat):
    """Edge integrals of a real periodic vector potential given by its rfft
    spectrum on the active grid (Ahat: 3 complex arrays from rfftn of point
    values at cell centres).  Evaluated exactly for the band-limited field."""
    n1, n2, n3 = n
    h1, h2, h3 = dx
    k1 = np.fft.rfftfreq(n1, d=1.0 / n1)[None, None, :]
    k2 = np.fft.fftfreq(n2, d=1.0 / n2)[None, :, None]
    k3 = np.fft.fftfreq(n3, d=1.0 / n3)[:, None, None]
    w1, w2, w3 = 2 * np.pi * k1 / L[0], 2 * np.pi * k2 / L[1], 2 * np.pi * k3 / L[2]

    def sinc_int(w, h):  # integral over a cell of e^{i w x} relative to the centre value, times h
        with np.errstate(invalid="ignore", divide="ignore"):
            s = np.where(np.abs(w) > 0, np.sin(0.5 * w * h) / (0.5 * w * h + 1e-300), 1.0)
        return h * s

    # shift from cell centre (grid of Ahat) to lower face: e^{-i w h/2}
    s1, s2, s3 = np.exp(-0.5j * w1 * h1), np.exp(-0.5j * w2 * h2), np.exp(-0.5j * w3 * h3)
    G1 = np.fft.irfftn(Ahat[0] * sinc_int(w1, h1) * s2 * s3, s=(n3, n2, n1), axes=(0, 1, 2))
    G2 = np.fft.irfftn(Ahat[1] * sinc_int(w2, h2) * s1 * s3, s=(n3, n2, n1), axes=(0, 1, 2))
    G3 = np.fft.irfftn(Ahat[2] * sinc_int(w3, h3) * s1 * s2, s=(n3, n2, n1), axes=(0, 1, 2))
    return [_pad_periodic(G, ng, extra=1) for G in (G1, G2, G3)]


def _pad_periodic(a_active: np.ndarray, ng: int, extra: int = 0) -> np.ndarray:
    """Stored array (ghosts + optional padded entry) of periodic images."""
    n3, n2, n1 = a_active.shape
    i1 = _wrapped_index(n1 + 2 * ng + extra, n1, ng) - ng
    i2 = _wrapped_index(n2 + 2 * ng + extra, n2, ng) - ng
    i3 = _wrapped_index(n3 + 2 * ng + extra, n3, ng) - ng
    return a_active[np.ix_(i3, i2, i1)]


def _band_modes(rng, n, kmin, kmax):
    """Random complex spectrum on integer wavevectors kmin <= |k| <= kmax, as
    rfft-shaped arrays for a grid of n = (n1, n2, n3) cells on a unit-period box."""
    n1, n2, n3 = n
    k1 = np.fft.rfftfreq(n1, d=1.0 / n1)[None, None, :]
    k2 = np.fft.fftfreq(n2, d=1.0 / n2)[None, :, None]
    k3 = np.fft.fftfreq(n3, d=1.0 / n3)[:, None, None]
    kk = np.sqrt(k1 ** 2 + k2 ** 2 + k3 ** 2)
    band = (kk >= kmin) & (kk <= kmax)
    shp = (n3, n2, n1 // 2 + 1)
    spec = np.zeros((3,) + shp, complex)
    for c in range(3):
        re = rng.standard_normal(shp)
        im = rng.standard_normal(shp)
        spec[c] = np.where(band, re + 1j * im, 0.0)
    return spec, (k1, k2, k3)


def _project_solenoidal(spec, kvec):
    k1, k2, k3 = kvec
    kk = k1 ** 2 + k2 ** 2 + k3 ** 2
    kk = np.where(kk == 0, 1.0, kk)
    dot = (spec[0] * k1 + spec[1] * k2 + spec[2] * k3) / kk
    return np.stack([spec[0] - dot * k1, spec[1] - dot * k2, spec[2] - dot * k3])


# ---------------------------------------------------------------------------
# Workloads
# ---------------------------------------------------------------------------
def linear_wave(N: int = 16, gamma: float = 5.0 / 3.0, amp: float = 1.0e-6, ng: int = 2) -> Block:
    """Fast magnetosonic eigenmode along the grid diagonal (Sec. 3.3.1): box
    3 x 1.5 x 1.5 on 2N x N x N cells, wavelength 1, amplitude amp.  Wave frame
    n1 = (1,2,2)/3, n2 = (-2,1,0)/sqrt5, n3 = n1 x n2.  Background rho = 1,
    p = 1/gamma, v = 0, B = (1, sqrt2, 1/2) in the wave frame, so a = 1 and the
    fast speed is 2.  Conserved state U = U0 + amp * R cos(k.x) with the fast
    right eigenvector R (normalised to drho = 1); B from a vector potential."""
    n = (2 * N, N, N)
    L = (3.0, 1.5, 1.5)
    dx = tuple(L[d] / n[d] for d in range(3))
    e1 = np.array([1.0, 2.0, 2.0]) / 3.0
    e2 = np.array([-2.0, 1.0, 0.0]) / math.sqrt(5.0)
    e3 = np.cross(e1, e2)
    r2 = math.sqrt(2.0)
    b_wave = (1.0, r2, 0.5)
    B0 = b_wave[0] * e1 + b_wave[1] * e2 + b_wave[2] * e3
    # R = (drho, dMn, dMt1, dMt2, dE, dBt1, dBt2)
    R = (1.0, 2.0, -2.0 * r2 / 3.0, -1.0 / 3.0, 4.5, 4.0 * r2 / 3.0, 2.0 / 3.0)
    dM = R[1] * e1 + R[2] * e2 + R[3] * e3
    dB = R[5] * e2 + R[6] * e3
    p0 = 1.0 / gamma
    E0 = p0 / (gamma - 1.0) + 0.5 * float(B0 @ B0)
    kvec = 2.0 * math.pi * e1  # wavelength 1

    x1 = _cell_centres(n[0], ng, dx[0])[None, None, :]
    x2 = _cell_centres(n[1], ng, dx[1])[None, :, None]
    x3 = _cell_centres(n[2], ng, dx[2])[:, None, None]
    phase = np.cos(kvec[0] * x1 + kvec[1] * x2 + kvec[2] * x3)
    shape = (n[2] + 2 * ng, n[1] + 2 * ng, n[0] + 2 * ng)
    cons = np.empty((5,) + shape)
    cons[0] = 1.0 + amp * R[0] * phase
    cons[1] = amp * dM[0] * phase
    cons[2] = amp * dM[1] * phase
    cons[3] = amp * dM[2] * phase
    cons[4] = E0 + amp * R[4] * phase
    # perturbation potential a sin(k.x) with curl = amp * dB cos(k.x)
    a = amp * np.cross(dB, kvec) / float(kvec @ kvec)
    bf = faces_from_modes(n, ng, dx, [(tuple(kvec), tuple(a), 0.0)])
    for c in range(3):
        bf[c] += B0[c]
    return Block(n=n, ng=ng, dx=dx, gamma=gamma, bface=bf, cons=cons,
                 meta=dict(workload="linear_wave_fast", N=N, amp=amp, t_end=0.5, cfl=0.3,
                           fast_speed=2.0, box=L))


def turbulence(n: int = 256, seed: int = 1, mach: float = 1.0, brms: float = 0.1, bx0: float = 0.5,
               gamma: float = 5.0 / 3.0, ng: int = 2, kmin: float = 1.0, kmax: float = 4.0) -> Block:
    """Decaying-turbulence initial state on the unit periodic cube with n^3
    cells: rho = 1, p = 1, solenoidal velocity with power on 1 <= |k| <= 4
    scaled to rms |v| = mach * sqrt(gamma p / rho), point-sampled at cell
    centres; B = (bx0, 0, 0) + curl A with A on the same band, scaled so the
    rms of the face values of curl A is brms."""
    rng = np.random.default_rng(seed)
    nn = (n, n, n)
    dx = (1.0 / n,) * 3
    vspec, kv = _band_modes(rng, nn, kmin, kmax)
    vspec = _project_solenoidal(vspec, kv)
    vel = np.stack([np.fft.irfftn(vspec[c], s=(n, n, n), axes=(0, 1, 2)) for c in range(3)])
    vrms = math.sqrt(float(np.mean(np.sum(vel ** 2, axis=0))))
    vel *= mach * math.sqrt(gamma) / vrms
    aspec, _ = _band_modes(rng, nn, kmin, kmax)
    # aspec holds the rfft of point values of A at cell centres
    G = _spectral_edges(nn, ng, dx, (1.0, 1.0, 1.0), aspec)
    dB = _faces_from_edges(G[0], G[1], G[2], nn, ng, dx)
    g = ng
    act = dB[:, g:g + n, g:g + n, g:g + n]
    brms_now = math.sqrt(float(np.mean(np.sum(act ** 2, axis=0))))
    bf = dB * (brms / brms_now)
    bf[0] += bx0
    prim = np.empty((5,) + (n + 2 * ng,) * 3)
    prim[0] = 1.0
    for c in range(3):
        prim[1 + c] = _pad_periodic(vel[c], ng)
    prim[4] = 1.0
    return Block(n=nn, ng=ng, dx=dx, gamma=gamma, bface=bf, prim=prim,
                 meta=dict(workload="turbulence", seed=seed, mach=mach, brms=brms, bx0=bx0, cfl=0.3))


def blast(n: int = 512, seed: int = 1, gamma: float = 5.0 / 3.0, ng: int = 3, p_amb: float = 0.1,
          p_in: float = 10.0, radius: float = 0.1, edge: float = 0.0) -> Block:
    """MHD blast on the unit periodic cube: rho = 1, p = p_amb, p = p_in where
    the (periodic, minimum-image) distance to a seeded random centre is below
    radius (sampled at cell centres); uniform B = (1/sqrt2, 1/sqrt2, 0).
    edge > 0 replaces the step by p_amb + (p_in - p_amb) (1 - tanh((r - radius)
    / (edge dx))) / 2, a sphere whose surface is smoothed over ~edge cells."""
    rng = np.random.default_rng(seed)
    c = rng.random(3)
    nn = (n, n, n)
    h = 1.0 / n
    x = [_cell_centres(n, ng, h)] * 3
    d1 = np.abs(x[0][None, None, :] - c[0]); d1 = np.minimum(d1, 1.0 - d1)
    d2 = np.abs(x[1][None, :, None] - c[1]); d2 = np.minimum(d2, 1.0 - d2)
    d3 = np.abs(x[2][:, None, None] - c[2]); d3 = np.minimum(d3, 1.0 - d3)
    r2 = d1 ** 2 + d2 ** 2 + d3 ** 2
    prim = np.zeros((5,) + (n + 2 * ng,) * 3)
    prim[0] = 1.0
    if edge > 0.0:
        prim[4] = p_amb + (p_in - p_amb) * 0.5 * (1.0 - np.tanh((np.sqrt(r2) - radius) / (edge * h)))
    else:
        prim[4] = np.where(r2 < radius * radius, p_in, p_amb)
    bf = np.zeros((3,) + (n + 2 * ng + 1,) * 3)
    bf[0] = 1.0 / math.sqrt(2.0)
    bf[1] = 1.0 / math.sqrt(2.0)
    return Block(n=nn, ng=ng, dx=(h, h, h), gamma=gamma, bface=bf, prim=prim,
                 meta=dict(workload="blast", seed=seed, centre=c.tolist(), cfl=0.3, edge=edge))


def uniform(n=(8, 8, 8), ng=2, rho=1.0, v=(0.3, -0.2, 0.1), p=0.7, B=(0.5, -0.4, 0.3),
            gamma=5.0 / 3.0, dx=(0.1, 0.1, 0.1)) -> Block:
    """Spatially uniform state."""
    n1, n2, n3 = n
    shape = (n3 + 2 * ng, n2 + 2 * ng, n1 + 2 * ng)
    prim = np.empty((5,) + shape)
    prim[0] = rho
    for c in range(3):
        prim[1 + c] = v[c]
    prim[4] = p
    bf = np.empty((3, shape[0] + 1, shape[1] + 1, shape[2] + 1))
    for c in range(3):
        bf[c] = B[c]
    return Block(n=tuple(n), ng=ng, dx=tuple(dx), gamma=gamma, bface=bf, prim=prim,
                 meta=dict(workload="uniform"))


def smooth_random(n=(16, 16, 16), seed=0, ng=2, gamma=5.0 / 3.0, vmax=0.9, kmax=2.0,
                  rho_range=(0.5, 2.0), p_range=(0.5, 2.0), B0=(0.3, 0.2, -0.1), brms=0.2,
                  dx=None) -> Block:
    """Smooth periodic random state on a block of n cells (unit-period box
    unless dx is given): rho, p in the given ranges via 1.25 + 0.75 f/max|f|
    (for the default ranges), |v| < vmax, B = B0 + curl A."""
    rng = np.random.default_rng(seed)
    n1, n2, n3 = n
    if dx is None:
        dx = (1.0 / n1, 1.0 / n2, 1.0 / n3)
    L = (dx[0] * n1, dx[1] * n2, dx[2] * n3)

    def field_(spec):
        return np.fft.irfftn(spec, s=(n3, n2, n1), axes=(0, 1, 2))

    spec, kv = _band_modes(rng, (n1, n2, n3), 1.0, kmax)
    f_rho = field_(spec[0]); f_p = field_(spec[1])
    vspec, _ = _band_modes(rng, (n1, n2, n3), 1.0, kmax)
    vel = np.stack([field_(vspec[c]) for c in range(3)])
    vmag = np.sqrt(np.sum(vel ** 2, axis=0)).max()
    vel *= vmax / vmag
    mid_r, half_r = 0.5 * (rho_range[0] + rho_range[1]), 0.5 * (rho_range[1] - rho_range[0])
    mid_p, half_p = 0.5 * (p_range[0] + p_range[1]), 0.5 * (p_range[1] - p_range[0])
    rho = mid_r + half_r * f_rho / np.abs(f_rho).max()
    pr = mid_p + half_p * f_p / np.abs(f_p).max()
    aspec, _ = _band_modes(rng, (n1, n2, n3), 1.0, kmax)
    G = _spectral_edges((n1, n2, n3), ng, dx, L, aspec)
    dB = _faces_from_edges(G[0], G[1], G[2], (n1, n2, n3), ng, dx)
    g = ng
    act = dB[:, g:g + n3, g:g + n2, g:g + n1]
    scale = brms / max(math.sqrt(float(np.mean(np.sum(act ** 2, axis=0)))), 1e-300)
    bf = dB * scale
    for c in range(3):
        bf[c] += B0[c]
    prim = np.empty((5, n3 + 2 * ng, n2 + 2 * ng, n1 + 2 * ng))
    prim[0] = _pad_periodic(rho, ng)
    for c in range(3):
        prim[1 + c] = _pad_periodic(vel[c], ng)
    prim[4] = _pad_periodic(pr, ng)
    return Block(n=(n1, n2, n3), ng=ng, dx=tuple(dx), gamma=gamma, bface=bf, prim=prim,
                 meta=dict(workload="smooth_random", seed=seed))


def x1_profile(n=(32, 6, 5), seed=0, ng=2, gamma=5.0 / 3.0, base=(1.0, 0.0, 0.0, 0.0, 1.0, 0.0, 0.0),
               amp=(0.0, 0.0, 0.3, 0.3, 0.0, 0.0, 0.0), b1=1.0, dx=None) -> Block:
    """State that varies along x1 only: each of (rho, v1, v2, v3, P, B2, B3) is
    base + amp * f(x1), f a seeded smooth periodic profile (modes 1..3, max
    |f| = 1) sampled at cell centres, and B1 = b1 everywhere.  B2 and B3 are
    the same on every face of a column, so the discrete div B is zero."""
    rng = np.random.default_rng(seed)
    n1, n2, n3 = n
    if dx is None:
        dx = (1.0 / n1, 1.0 / n1, 1.0 / n1)
    L = dx[0] * n1
    xs = (np.arange(n1) + 0.5) * dx[0]
    prof = []
    for q in range(7):
        f = np.zeros(n1)
        for m in range(1, 4):
            f += rng.normal() * np.sin(2 * math.pi * m * xs / L + rng.uniform(0, 2 * math.pi))
        prof.append(base[q] + amp[q] * f / np.abs(f).max())
    shape = (n3 + 2 * ng, n2 + 2 * ng, n1 + 2 * ng)
    cells = _wrapped_index(shape[2], n1, ng) - ng        # active column of every stored x1 index
    faces = _wrapped_index(shape[2] + 1, n1, ng) - ng    # same for the padded face arrays
    prim = np.empty((5,) + shape)
    for q in range(5):
        prim[q] = prof[q][cells][None, None, :]
    bf = np.zeros((3, shape[0] + 1, shape[1] + 1, shape[2] + 1))
    bf[0] = b1
    bf[1] = prof[5][faces][None, None, :]
    bf[2] = prof[6][faces][None, None, :]
    return Block(n=(n1, n2, n3), ng=ng, dx=tuple(dx), gamma=gamma, bface=bf, prim=prim,
                 meta=dict(workload="x1_profile", seed=seed))


def with_scalars(block: Block, nscalars: int, seed: int = 0, width: float = 0.1) -> Block:
    """The block with nscalars passive-scalar rows appended to its primitives:
    specific densities C_i of seeded tracer patterns on the block's periodic
    box.  Scalar 0 is a dye, 0.5 + 0.5 tanh(f / width) of a smooth random level
    function f scaled to max |f| = 1, so it is 0 or 1 away from fronts a few
    cells wide; further scalars are smooth fields 1 + 0.9 f in [0.1, 1.9]."""
    rng = np.random.default_rng(seed)
    n1, n2, n3 = block.n
    ng = block.ng
    rows = []
    for i in range(nscalars):
        spec, _ = _band_modes(rng, (n1, n2, n3), 1.0, 3.0)
        f = np.fft.irfftn(spec[0], s=(n3, n2, n1), axes=(0, 1, 2))
        f /= np.abs(f).max()
        c = 0.5 + 0.5 * np.tanh(f / width) if i == 0 else 1.0 + 0.9 * f
        rows.append(_pad_periodic(c, ng))
    prim = np.concatenate([block.prim[:5]] + [r[None] for r in rows], axis=0) if rows else block.prim[:5].copy()
    meta = dict(block.meta, nscalars=nscalars, scalar_seed=seed)
    return Block(n=block.n, ng=ng, dx=block.dx, gamma=block.gamma, bface=block.bface, prim=np.ascontiguousarray(prim),
                 meta=meta)


def divb_metric(bf: np.ndarray, n, ng, dx) -> float:
    """max over active cells of |sum_d (B_d+ - B_d-)/dx_d| * min dx / max|B|."""
    g = ng
    n1, n2, n3 = n
    a = (slice(g, g + n3), slice(g, g + n2), slice(g, g + n1))
    b1 = bf[0][a[0], a[1], g:g + n1 + 1]
    b2 = bf[1][a[0], g:g + n2 + 1, a[2]]
    b3 = bf[2][g:g + n3 + 1, a[1], a[2]]
    div = (np.diff(b1, axis=2) / dx[0] + np.diff(b2, axis=1) / dx[1] + np.diff(b3, axis=0) / dx[2])
    bmax = max(np.abs(b1).max(), np.abs(b2).max(), np.abs(b3).max(), 1e-300)
    return float(np.abs(div).max() * min(dx) / bmax)


# ---------------------------------------------------------------------------
# Batched AMR-shaped workload: leaves of a seeded 2:1-balanced octree
# ---------------------------------------------------------------------------
def _morton3(x: int, y: int, z: int, bits: int = 10) -> int:
    key = 0
    for b in range(bits):
        key |= ((x >> b) & 1) << (3 * b) | ((y >> b) & 1) << (3 * b + 1) | ((z >> b) & 1) << (3 * b + 2)
    return key


def balanced_octree(nleaves: int, seed: int = 0, root_level: int = 2, max_level: int = 6):
    """Leaves (level, i, j, k) of a periodic octree on the unit cube, grown by
    refining seeded random leaves while keeping every pair of touching leaves
    (faces, edges, corners, periodic) within one level; at least nleaves
    leaves, returned in Morton order of their lower corner."""
    rng = np.random.default_rng(seed)
    leaves = {(root_level, i, j, k) for i in range(1 << root_level) for j in range(1 << root_level)
              for k in range(1 << root_level)}

    def level_at(lev, i, j, k):
        # level of the leaf covering the fine cell (i, j, k) at level lev
        n = 1 << lev
        i, j, k = i % n, j % n, k % n
        for L in range(lev, -1, -1):
            s = lev - L
            key = (L, i >> s, j >> s, k >> s)
            if key in leaves:
                return L
        return None

    def neighbours_ok(leaf):
        L, i, j, k = leaf
        for di in (-1, 0, 1):
            for dj in (-1, 0, 1):
                for dk in (-1, 0, 1):
                    if di == dj == dk == 0:
                        continue
                    lv = level_at(L, i + di, j + dj, k + dk)
                    if lv is not None and lv < L:
                        return False
        return True

    while len(leaves) < nleaves:
        cand = sorted(leaves)
        leaf = cand[int(rng.integers(len(cand)))]
        L, i, j, k = leaf
        if L >= max_level or not neighbours_ok(leaf):
            continue
        leaves.remove(leaf)
        for a in (0, 1):
            for b in (0, 1):
                for c in (0, 1):
                    leaves.add((L + 1, 2 * i + a, 2 * j + b, 2 * k + c))
    out = sorted(leaves, key=lambda t: _morton3(t[1] << (max_level - t[0]), t[2] << (max_level - t[0]),
                                                 t[3] << (max_level - t[0])))
    return out


def amr_batch(nblocks: int = 1024, seed: int = 3, sizes=(16, 24, 32), fractions=(0.4, 0.4, 0.2), ng: int = 2,
              gamma: float = 5.0 / 3.0):
    """Blocks of uneven sizes shaped like an AMR mesh: the first nblocks leaves
    (Morton order) of a seeded 2:1-balanced octree give each block a level and
    a physical edge 2^-level; block sizes follow the given mix (seeded
    shuffle) and dx = edge / n.  Each block carries its own smooth periodic
    state: rho, p in [0.5, 2], |v| < 0.9, B = B0 + curl A."""
    rng = np.random.default_rng(seed)
    leaves = balanced_octree(nblocks, seed=seed)[:nblocks]
    counts = [int(round(f * nblocks)) for f in fractions]
    counts[-1] = nblocks - sum(counts[:-1])
    size_list = np.concatenate([np.full(c, s) for c, s in zip(counts, sizes)])
    rng.shuffle(size_list)
    blocks = []
    for b, (leaf, n) in enumerate(zip(leaves, size_list)):
        edge = 2.0 ** (-leaf[0])
        n = int(n)
        blk = smooth_random(n=(n, n, n), seed=seed * 100003 + b, ng=ng, gamma=gamma, vmax=0.9,
                            dx=(edge / n,) * 3, B0=tuple(0.3 * rng.standard_normal(3)), brms=0.2)
        blk.meta.update(level=leaf[0], morton=leaf[1:])
        blocks.append(blk)
    return blocks


def split_mesh(cells: np.ndarray, faces: np.ndarray, ng: int, n_block, mesh):
    """Cut a periodic domain (one block of mesh[d] * n_block[d] cells, with ng
    ghost layers: cells (nv, N3, N2, N1), faces (3, N3+1, N2+1, N1+1)) into the
    blocks of a coupled mesh, block b = bx + nbx (by + nby bz), each with its
    own ng ghost layers taken from the periodic domain.  Returns arrays of
    shape (nb, nv, ...) and (nb, 3, ...).  Index arithmetic only."""
    n1, n2, n3 = n_block
    L = (mesh[0] * n1, mesh[1] * n2, mesh[2] * n3)
    M = (n1 + 2 * ng, n2 + 2 * ng, n3 + 2 * ng)
    out_c, out_f = [], []
    for bz in range(mesh[2]):
        for by in range(mesh[1]):
            for bx in range(mesh[0]):
                o = (bx * n1, by * n2, bz * n3)
                ci = [ng + (np.arange(M[d]) + o[d] - ng) % L[d] for d in range(3)]
                fi = [ng + (np.arange(M[d] + 1) + o[d] - ng) % L[d] for d in range(3)]
                out_c.append(cells[:, ci[2][:, None, None], ci[1][None, :, None], ci[0][None, None, :]])
                out_f.append(faces[:, fi[2][:, None, None], fi[1][None, :, None], fi[0][None, None, :]])
    return np.ascontiguousarray(np.stack(out_c)), np.ascontiguousarray(np.stack(out_f))


def join_mesh(cells: np.ndarray, faces: np.ndarray, ng: int, n_block, mesh):
    """Inverse of split_mesh on the active entries: the blocks' active cells and
    the lower faces of their active cells, placed into a periodic domain
    block of (mesh[d] * n_block[d]) cells with ng ghost layers (ghost and image
    entries left zero)."""
    n1, n2, n3 = n_block
    nb, nv = cells.shape[:2]
    L = (mesh[0] * n1, mesh[1] * n2, mesh[2] * n3)
    dc = np.zeros((nv, L[2] + 2 * ng, L[1] + 2 * ng, L[0] + 2 * ng))
    df = np.zeros((3, L[2] + 2 * ng + 1, L[1] + 2 * ng + 1, L[0] + 2 * ng + 1))
    a = (slice(ng, ng + n3), slice(ng, ng + n2), slice(ng, ng + n1))
    b = 0
    for bz in range(mesh[2]):
        for by in range(mesh[1]):
            for bx in range(mesh[0]):
                d = (slice(ng + bz * n3, ng + (bz + 1) * n3), slice(ng + by * n2, ng + (by + 1) * n2),
                     slice(ng + bx * n1, ng + (bx + 1) * n1))
                dc[(slice(None),) + d] = cells[b][(slice(None),) + a]
                df[(slice(None),) + d] = faces[b][(slice(None),) + a]
                b += 1
    return dc, df


def brick_layout(slabs, cross: int):
    """Blocks of uneven cube sizes tiling one periodic domain at one cell
    width: the domain of cross x cross x sum(slabs) cells is cut along x3 into
    slabs of the given thicknesses, and each slab is tiled by cubes of its
    thickness (cross must be a multiple of every thickness).  Across a slab
    boundary the blocks' faces do not line up, so a block's ghost cells along
    x3 come from several neighbours.  Returns (dims, origins, domain): block b
    has dims[b] cells and its first active cell at origins[b] (x1 first).
    Index arithmetic only."""
    dims, origins = [], []
    z = 0
    for s in slabs:
        s = int(s)
        if cross % s:
            raise ValueError(f"cross section {cross} is not a multiple of {s}")
        for y in range(0, cross, s):
            for x in range(0, cross, s):
                dims.append((s, s, s))
                origins.append((x, y, z))
        z += s
    return dims, origins, (cross, cross, z)


def brick_slabs(nblocks: int = 1024, sizes=(16, 24, 32), fractions=(0.4, 0.4, 0.2), cross: int = 192,
                seed: int = 3):
    """Slab thicknesses for brick_layout whose cube counts come closest to
    nblocks blocks in the given size mix (per size, the nearest whole number
    of slabs), in a seeded order along x3."""
    rng = np.random.default_rng(seed)
    slabs = []
    for s, f in zip(sizes, fractions):
        per = (cross // s) ** 2
        slabs += [s] * max(1, int(round(f * nblocks / per)))
    rng.shuffle(slabs)
    return [int(x) for x in slabs]


def split_boxes(cells: np.ndarray, faces: np.ndarray, ng: int, dims, origins):
    """Cut a periodic domain (one block of L[d] cells with ng ghost layers:
    cells (nv, N3, N2, N1), faces (3, N3+1, N2+1, N1+1)) into blocks of their
    own sizes, block b with dims[b] active cells from origins[b], each with
    its own ng ghost layers and face entries taken from the periodic domain.
    Returns two lists of per-block arrays.  Index arithmetic only."""
    L = tuple(cells.shape[3 - d] - 2 * ng for d in range(3))
    out_c, out_f = [], []
    for n, o in zip(dims, origins):
        M = tuple(n[d] + 2 * ng for d in range(3))
        ci = [ng + (np.arange(M[d]) + o[d] - ng) % L[d] for d in range(3)]
        fi = [ng + (np.arange(M[d] + 1) + o[d] - ng) % L[d] for d in range(3)]
        out_c.append(np.ascontiguousarray(cells[:, ci[2][:, None, None], ci[1][None, :, None], ci[0][None, None, :]]))
        out_f.append(np.ascontiguousarray(faces[:, fi[2][:, None, None], fi[1][None, :, None], fi[0][None, None, :]]))
    return out_c, out_f


def join_boxes(cells, faces, ng: int, dims, origins, domain):
    """Inverse of split_boxes on the active entries: each block's active cells
    and the lower faces of its active cells, placed into a periodic domain of
    domain[d] cells with ng ghost layers (other entries left zero)."""
    nv = cells[0].shape[0]
    L = tuple(int(x) for x in domain)
    dc = np.zeros((nv, L[2] + 2 * ng, L[1] + 2 * ng, L[0] + 2 * ng))
    df = np.zeros((3, L[2] + 2 * ng + 1, L[1] + 2 * ng + 1, L[0] + 2 * ng + 1))
    for c, f, n, o in zip(cells, faces, dims, origins):
        a = (slice(None), slice(ng, ng + n[2]), slice(ng, ng + n[1]), slice(ng, ng + n[0]))
        d = (slice(None), slice(ng + o[2], ng + o[2] + n[2]), slice(ng + o[1], ng + o[1] + n[1]),
             slice(ng + o[0], ng + o[0] + n[0]))
        dc[d] = c[a]
        df[d] = f[a]
    return dc, df


def analytic_state(n, ng=2, box=(2.0, 1.0, 1.0), seed=0, gamma=5.0 / 3.0, amp=0.2, vamp=0.4, bamp=0.15,
                   B0=(0.6, 0.3, -0.2), modes=3) -> Block:
    """Smooth periodic state on an n-cell uniform grid of the given box, from
    seeded analytic Fourier modes, so that grids of different resolution over
    the same box sample the same continuous fields: rho, p = 1 + amp f, v =
    vamp g (cell-centre values), B = B0 + curl A with A a sum of modes (face
    values from exact edge integrals).  Wave vectors are integer multiples of
    2 pi / box along each direction."""
    rng = np.random.default_rng(seed)
    dx = tuple(box[d] / n[d] for d in range(3))
    x = [_cell_centres(n[d], ng, dx[d]) for d in range(3)]
    X1, X2, X3 = x[0][None, None, :], x[1][None, :, None], x[2][:, None, None]

    def field():
        f = 0.0
        for _ in range(modes):
            k = [2 * math.pi * rng.integers(-2, 3) / box[d] for d in range(3)]
            f = f + rng.normal() * np.cos(k[0] * X1 + k[1] * X2 + k[2] * X3 + rng.uniform(0, 2 * math.pi))
        return f

    shape = (n[2] + 2 * ng, n[1] + 2 * ng, n[0] + 2 * ng)
    prim = np.empty((5,) + shape)
    f = field() + np.zeros(shape)
    prim[0] = 1.0 + amp * f / max(np.abs(f).max(), 1e-300)
    for c in range(3):
        g = field() + np.zeros(shape)
        prim[1 + c] = vamp * g / max(np.abs(g).max(), 1e-300)
    f = field() + np.zeros(shape)
    prim[4] = 1.0 + amp * f / max(np.abs(f).max(), 1e-300)
    amodes = []
    for _ in range(modes):
        k = [2 * math.pi * rng.integers(-2, 3) / box[d] for d in range(3)]
        if k[0] == k[1] == k[2] == 0.0:
            continue
        a = tuple(bamp * rng.normal(size=3) / math.sqrt(k[0] ** 2 + k[1] ** 2 + k[2] ** 2))
        amodes.append((tuple(k), a, rng.uniform(0, 2 * math.pi)))
    bf = faces_from_modes(tuple(n), ng, dx, amodes) if amodes else np.zeros((3,) + tuple(s + 1 for s in shape))
    for c in range(3):
        bf[c] += B0[c]
    return Block(n=tuple(n), ng=ng, dx=dx, gamma=gamma, bface=bf, prim=prim,
                 meta=dict(workload="analytic_state", seed=seed, box=box))


def two_level(coarse: Block, fine: Block, n):
    """The nine blocks of a two-level composite from two uniform periodic grids
    of the same box: coarse with (2 n1, n2, n3) cells, fine with
    (4 n1, 2 n2, 2 n3).  Block 0 is the coarse grid's upper half along x1;
    block 1 + a + 2 b + 4 c is the fine grid's block (a, b, c) of n cells in
    its lower half along x1.  Returns (cells, faces) of shape (9, nv, ...),
    (9, 3, ...), from the grids' prim (or cons when prim is None).  Index
    arithmetic only."""
    ng = coarse.ng
    cc = coarse.prim if coarse.prim is not None else coarse.cons
    fc = fine.prim if fine.prim is not None else fine.cons
    c_cells, c_faces = split_mesh(cc, coarse.bface, ng, n, (2, 1, 1))
    f_cells, f_faces = split_mesh(fc, fine.bface, ng, n, (4, 2, 2))
    cells = [c_cells[1]]
    faces = [c_faces[1]]
    for c in range(2):
        for b in range(2):
            for a in range(2):
                q = a + 4 * (b + 2 * c)
                cells.append(f_cells[q])
                faces.append(f_faces[q])
    return np.ascontiguousarray(np.stack(cells)), np.ascontiguousarray(np.stack(faces))


def pack(arrays) -> np.ndarray:
    """Concatenate per-block arrays into the flat batched layout."""
    return np.concatenate([np.ascontiguousarray(a).reshape(-1) for a in arrays])
