"""Sub-blocks ("windows") of a periodic block, for checking full-size results
against the oracle cell by cell.

One step changes a cell only through cells within a fixed distance of it (the
reconstruction stencil, the Riemann problems on its faces and the corner EMFs
of its edges, once per stage).  A window of m^3 active cells cut out of the
full periodic grid and stepped by the oracle as a periodic block of its own is
therefore wrong only within that distance of its edges; its inner cells are
the full grid's.  Pure index arithmetic: nothing of the method is computed
here.
"""
import numpy as np


def extract(cons, bface, ng, n, origin, m):
    """Window of m^3 active cells whose first active cell is the full grid's
    active cell `origin` = (o1, o2, o3) (indices wrap periodically), with ng
    ghost layers taken from the wrapped full grid.  Layouts as the library's:
    cons[v][k][j][i], bface[c][k][j][i] padded to (N3+1, N2+1, N1+1)."""
    M = m + 2 * ng
    ci = [ng + (np.arange(M) + o - ng) % nn for o, nn in zip(origin, n)]
    fi = [ng + (np.arange(M + 1) + o - ng) % nn for o, nn in zip(origin, n)]
    c = cons[:, ci[2][:, None, None], ci[1][None, :, None], ci[0][None, None, :]]
    b = bface[:, fi[2][:, None, None], fi[1][None, :, None], fi[0][None, None, :]]
    return np.ascontiguousarray(c), np.ascontiguousarray(b)


def inner(cons, bface, ng, n, origin, m, r):
    """The window's inner (m - 2r)^3 cells and their lower faces, read from
    the full grid (same index map as extract)."""
    c, b = extract(cons, bface, ng, n, origin, m)
    return inner_of_window(c, b, ng, m, r)


def inner_of_window(c, b, ng, m, r):
    """The inner (m - 2r)^3 cells of a window and their lower faces."""
    s = slice(ng + r, ng + m - r)
    return c[:, s, s, s], b[:, s, s, s]


def rel_l1_arrays(ca, ba, cb, bb, mom_speed=0.0):
    """relative L1 of a against b for each of the 5 conserved arrays and the
    3 face arrays.  A face component is measured against at least the mean
    L1 of the three (a component that is zero, like B3 of a field in the
    x1-x2 plane, stays zero only up to rounding); with mom_speed > 0 a
    momentum array is likewise measured against at least sum(rho) * mom_speed
    (gas at rest)."""
    errs = []
    rho = np.abs(cb[0]).sum()
    bmean = np.mean([np.abs(bb[c]).sum() for c in range(bb.shape[0])])
    for x, y, cons in ((ca, cb, True), (ba, bb, False)):
        for v in range(x.shape[0]):
            den = np.abs(y[v]).sum()
            if cons and 1 <= v <= 3:
                den = max(den, rho * mom_speed)
            if not cons:
                den = max(den, bmean)
            errs.append(float(np.abs(x[v] - y[v]).sum() / max(den, 1e-300)))
    return errs


def max_rel_l1(ca, ba, cb, bb, mom_speed=0.0):
    """worst of rel_l1_arrays"""
    return max(rel_l1_arrays(ca, ba, cb, bb, mom_speed))
