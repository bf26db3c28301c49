"""Thin ctypes binding of libathmhd.so (argument marshalling only).

Every step of the method runs in the HIP kernels of the library; this module
only turns torch tensors (device memory, float64, contiguous) into pointers and
the current torch stream into a hipStream_t.  There is no fallback: if the
library is missing or the device is not a HIP GPU, calls raise.
"""
from __future__ import annotations

import ctypes as C
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libathmhd.so")

OK, EINVAL, ENOMEM, EHIP, ENONPHYS, EUNSUP = 0, -1, -2, -3, -4, -5
RECON = {"dc": 0, "plm": 1, "ppm": 2}
RIEMANN = {"hlle": 0, "hlld": 1, "roe": 2}
INTEGRATOR = {"rk1": 0, "vl2": 1, "rk2": 2, "rk3": 3}
EXPORTED = ["athmhd_version", "athmhd_create", "athmhd_create_batch", "athmhd_batch_info",
            "athmhd_batch_set_tile", "athmhd_batch_tune", "athmhd_set_graph", "athmhd_step", "athmhd_newdt",
            "athmhd_prim2cons", "athmhd_fill_ghosts", "athmhd_profile", "athmhd_last_error", "athmhd_destroy",
            "athmhd_step_vjp", "athmhd_prim2cons_vjp", "athmhd_set_floors", "athmhd_floor_count",
            "athmhd_step_stages", "athmhd_create_mesh", "athmhd_restrict", "athmhd_prolong",
            "athmhd_restrict_box", "athmhd_prolong_box", "athmhd_newdt_noalloc", "athmhd_create_levels",
            "athmhd_step_chain", "athmhd_batch_couple"]
BATCH_TILES = [(16, 12), (12, 16), (14, 14), (16, 8)]  # active columns of the batch tile candidates


class AthmhdError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"athmhd error {code}: {msg}")
        self.code = code


class NonPhysicalState(AthmhdError):
    pass


class Config(C.Structure):
    """Mirror of athmhd_config (include/athmhd.h)."""
    _fields_ = [("n1", C.c_int32), ("n2", C.c_int32), ("n3", C.c_int32), ("nghost", C.c_int32),
                ("gamma", C.c_double), ("dx1", C.c_double), ("dx2", C.c_double), ("dx3", C.c_double),
                ("recon", C.c_int32), ("riemann", C.c_int32), ("integrator", C.c_int32),
                ("kernel_path", C.c_int32), ("cfl", C.c_double), ("ct_eps", C.c_double),
                ("nscalars", C.c_int32), ("charac", C.c_int32)]


_lib = None


def lib():
    """Load libathmhd.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2005_06651_amd.build`")
        L = C.CDLL(LIB_PATH)
        vp = C.c_void_p
        L.athmhd_version.restype = C.c_int
        L.athmhd_create.argtypes = [C.POINTER(Config), C.c_int, C.POINTER(vp)]
        L.athmhd_create_mesh.argtypes = [C.POINTER(Config), C.c_int, C.c_int, C.c_int, C.POINTER(vp)]
        L.athmhd_create_levels.argtypes = [C.POINTER(Config), C.POINTER(vp)]
        L.athmhd_create_batch.argtypes = [C.POINTER(Config), C.POINTER(C.c_int32), C.POINTER(C.c_double), C.c_int,
                                          C.POINTER(vp)]
        L.athmhd_batch_info.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
        L.athmhd_batch_set_tile.argtypes = [vp, C.c_int, C.c_int]
        L.athmhd_batch_couple.argtypes = [vp, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]
        L.athmhd_batch_tune.argtypes = [vp, vp, vp, vp, C.POINTER(C.c_int), C.POINTER(C.c_int),
                                        C.POINTER(C.c_double)]
        L.athmhd_set_graph.argtypes = [vp, C.c_int]
        L.athmhd_step.argtypes = [vp, vp, vp, C.c_double, C.c_int, vp]
        L.athmhd_step_chain.argtypes = [vp, vp, vp, C.c_int, vp, vp, vp]
        L.athmhd_newdt.argtypes = [vp, vp, vp, C.c_int, C.POINTER(C.c_double), vp]
        L.athmhd_newdt_noalloc.argtypes = [vp, vp, vp, C.c_int, vp, vp, vp]
        L.athmhd_prim2cons.argtypes = [vp, vp, vp, vp, C.c_int, vp]
        L.athmhd_fill_ghosts.argtypes = [vp, vp, vp, C.c_int, vp]
        L.athmhd_step_vjp.argtypes = [vp, vp, vp, C.c_double, vp, vp, vp, vp, vp, C.c_int, vp]
        L.athmhd_step_stages.argtypes = [vp, vp, vp, C.c_double, vp, C.c_int, vp]
        L.athmhd_set_floors.argtypes = [vp, C.c_double, C.c_double]
        L.athmhd_floor_count.argtypes = [vp, C.POINTER(C.c_longlong), vp]
        L.athmhd_prim2cons_vjp.argtypes = [vp, vp, vp, vp, vp, vp, C.c_int, vp]
        L.athmhd_profile.argtypes = [vp, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_int)]
        L.athmhd_restrict.argtypes = [vp, vp, vp, vp, vp, C.c_int, C.c_int, C.c_int, vp]
        L.athmhd_prolong.argtypes = [vp, vp, vp, vp, vp, C.c_int, C.c_int, C.c_int, C.c_int, vp]
        I3 = C.POINTER(C.c_int)
        L.athmhd_restrict_box.argtypes = [vp, vp, vp, vp, vp, I3, I3, I3, vp]
        L.athmhd_prolong_box.argtypes = [vp, vp, vp, vp, vp, I3, I3, I3, C.c_int, C.c_int, vp]
        L.athmhd_last_error.argtypes = [vp]
        L.athmhd_last_error.restype = C.c_char_p
        L.athmhd_destroy.argtypes = [vp]
        L.athmhd_destroy.restype = None
        _lib = L
    return _lib


KERNEL_PATH = {"fused": 0, "unfused": 1}


def make_config(n, nghost, dx, gamma, recon="plm", riemann="hlld", integrator="vl2", cfl=0.3,
                ct_eps=0.0, kernel_path="fused", nscalars=0, charac=False) -> Config:
    return Config(int(n[0]), int(n[1]), int(n[2]), int(nghost), float(gamma), float(dx[0]), float(dx[1]),
                  float(dx[2]), RECON[recon], RIEMANN[riemann], INTEGRATOR[integrator],
                  KERNEL_PATH[kernel_path], float(cfl), float(ct_eps), int(nscalars), int(bool(charac)))


def _check(rc: int, h) -> None:
    if rc != OK:
        msg = lib().athmhd_last_error(h).decode(errors="replace")
        raise (NonPhysicalState if rc == ENONPHYS else AthmhdError)(rc, msg)


def _scalar_out(t, dtype: str):
    """Device address of a one-element (or longer) contiguous output tensor."""
    import torch
    if not isinstance(t, torch.Tensor) or not t.is_cuda or str(t.dtype) != "torch." + dtype:
        raise TypeError(f"expected a {dtype} tensor in HIP device memory")
    if t.numel() < 1 or not t.is_contiguous():
        raise ValueError("output tensor must be contiguous with at least one element")
    return C.c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


class Solver:
    """One handle of the library: nblocks identical periodic MeshBlocks.

    Tensors: cons (nb, 5 + nscalars, N3, N2, N1) and bface (nb, 3, N3+1, N2+1,
    N1+1), float64, contiguous, on the current HIP device (leading nb axis
    optional when nb == 1).  Passive scalars rho C_i follow the 5 MHD
    variables in cons, and C_i the 5 primitives in prim."""

    def __init__(self, n, nghost, dx, gamma, recon="plm", riemann="hlld", integrator="vl2", cfl=0.3,
                 ct_eps=0.0, nblocks=1, kernel_path="fused", nscalars=0, charac=False):
        self.n = tuple(int(x) for x in n)
        self.ng = int(nghost)
        self.nblocks = int(nblocks)
        self.nv = 5 + int(nscalars)
        self.cfg = make_config(n, nghost, dx, gamma, recon, riemann, integrator, cfl, ct_eps, kernel_path, nscalars,
                               charac)
        h = C.c_void_p()
        rc = lib().athmhd_create(C.byref(self.cfg), self.nblocks, C.byref(h))
        if rc != OK:
            raise AthmhdError(rc, lib().athmhd_last_error(None).decode(errors="replace"))
        self._h = h

    @property
    def cell_shape(self):
        n1, n2, n3 = self.n
        g = self.ng
        return (n3 + 2 * g, n2 + 2 * g, n1 + 2 * g)

    @property
    def face_shape(self):
        return tuple(x + 1 for x in self.cell_shape)

    def _arr(self, t, nvar, shape):
        import torch
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
            raise TypeError("expected a float64 tensor in HIP device memory")
        if not t.is_contiguous():
            raise ValueError("tensor must be contiguous")
        sh = tuple(t.shape)
        if sh == (nvar,) + shape:
            nb = 1
        elif len(sh) == 5 and sh[1:] == (nvar,) + shape:
            nb = sh[0]
        else:
            raise ValueError(f"bad shape {sh}, expected (nb, {nvar}) + {shape}")
        return C.c_void_p(t.data_ptr()), nb

    def _pair(self, cons, bface):
        pc, nb = self._arr(cons, self.nv, self.cell_shape)
        pb, nb2 = self._arr(bface, 3, self.face_shape)
        if nb != nb2:
            raise ValueError("cons and bface hold different block counts")
        return pc, pb, nb

    def step(self, cons, bface, dt: float, stream=None) -> None:
        pc, pb, nb = self._pair(cons, bface)
        _check(lib().athmhd_step(self._h, pc, pb, float(dt), nb, _stream(stream)), self._h)

    def step_chain(self, cons, bface, dt_dev, nbad_out=None, stream=None) -> None:
        """athmhd_step_chain: one step with dt read from dt_dev[0] (float64
        device tensor), which then holds the next step's dt; the non-physical
        count goes to nbad_out[0] (int32 device tensor) when given.
        Asynchronous."""
        pc, pb, nb = self._pair(cons, bface)
        nbp = None if nbad_out is None else _scalar_out(nbad_out, "int32")
        _check(lib().athmhd_step_chain(self._h, pc, pb, nb, _scalar_out(dt_dev, "float64"), nbp, _stream(stream)),
               self._h)

    def newdt(self, cons, bface, stream=None) -> float:
        pc, pb, nb = self._pair(cons, bface)
        out = C.c_double()
        _check(lib().athmhd_newdt(self._h, pc, pb, nb, C.byref(out), _stream(stream)), self._h)
        return out.value

    def newdt_noalloc(self, cons, bface, dt_out, nbad_out, stream=None) -> None:
        """athmhd_newdt_noalloc: dt into dt_out[0] (float64) and the
        non-physical count into nbad_out[0] (int32), both device tensors;
        asynchronous, allocates nothing."""
        pc, pb, nb = self._pair(cons, bface)
        _check(lib().athmhd_newdt_noalloc(self._h, pc, pb, nb, _scalar_out(dt_out, "float64"),
                                          _scalar_out(nbad_out, "int32"), _stream(stream)), self._h)

    def prim2cons(self, prim, bface, out=None, stream=None):
        import torch
        pp, pb, nb = self._pair(prim, bface)
        if out is None:
            out = torch.empty_like(prim)
        po, _ = self._arr(out, self.nv, self.cell_shape)
        _check(lib().athmhd_prim2cons(self._h, pp, pb, po, nb, _stream(stream)), self._h)
        return out

    def fill_ghosts(self, cons, bface, stream=None) -> None:
        pc, pb, nb = self._pair(cons, bface)
        _check(lib().athmhd_fill_ghosts(self._h, pc, pb, nb, _stream(stream)), self._h)

    def _one_block(self, cons, bface):
        pc, pb, nb = self._pair(cons, bface)
        if nb != 1:
            raise ValueError("level operators take one block")
        return pc, pb

    def restrict(self, fine_cons, fine_bface, coarse_cons, coarse_bface, octant, stream=None) -> None:
        """Restrict the fine block onto octant (o1, o2, o3) of the coarse block, in place."""
        fc, fb = self._one_block(fine_cons, fine_bface)
        cc, cb = self._one_block(coarse_cons, coarse_bface)
        o = [int(x) for x in octant]
        _check(lib().athmhd_restrict(self._h, fc, fb, cc, cb, *o, _stream(stream)), self._h)

    def prolong(self, coarse_cons, coarse_bface, fine_cons, fine_bface, octant, primitive=False,
                stream=None) -> None:
        """Prolong octant (o1, o2, o3) of the coarse block onto the fine block's
        active cells and faces (primitive=True: in primitive variables)."""
        cc, cb = self._one_block(coarse_cons, coarse_bface)
        fc, fb = self._one_block(fine_cons, fine_bface)
        o = [int(x) for x in octant]
        _check(lib().athmhd_prolong(self._h, cc, cb, fc, fb, *o, int(bool(primitive)), _stream(stream)), self._h)

    @staticmethod
    def _box(fine_lo, coarse_lo, extent):
        return [(C.c_int * 3)(*[int(x) for x in v]) for v in (fine_lo, coarse_lo, extent)]

    def restrict_box(self, fine_cons, fine_bface, coarse_cons, coarse_bface, fine_lo, coarse_lo, extent,
                     stream=None) -> None:
        """Restrict fine cells [fine_lo, fine_lo + 2 extent) onto coarse cells
        [coarse_lo, coarse_lo + extent) (stored (x1, x2, x3) indices, ghosts included)."""
        fc, fb = self._one_block(fine_cons, fine_bface)
        cc, cb = self._one_block(coarse_cons, coarse_bface)
        _check(lib().athmhd_restrict_box(self._h, fc, fb, cc, cb, *self._box(fine_lo, coarse_lo, extent),
                                         _stream(stream)), self._h)

    def prolong_box(self, coarse_cons, coarse_bface, fine_cons, fine_bface, fine_lo, coarse_lo, extent,
                    primitive=False, keep=0, stream=None) -> None:
        """Prolong coarse cells [coarse_lo, coarse_lo + extent) onto fine cells
        [fine_lo, fine_lo + 2 extent) and their faces; keep bit 2 d + S keeps
        the fine faces already on side S of the box along direction d."""
        cc, cb = self._one_block(coarse_cons, coarse_bface)
        fc, fb = self._one_block(fine_cons, fine_bface)
        _check(lib().athmhd_prolong_box(self._h, cc, cb, fc, fb, *self._box(fine_lo, coarse_lo, extent),
                                        int(bool(primitive)), int(keep), _stream(stream)), self._h)

    @property
    def extra_stages(self) -> int:
        """Stages of the integrator beyond the first (S - 1)."""
        return {0: 0, 1: 1, 2: 1, 3: 2}[self.cfg.integrator]

    def stages_like(self, cons):
        """A buffer for the stage inputs of one step (see step_stages)."""
        import torch
        nb = cons.shape[0] if cons.dim() == 5 else 1
        n1 = self.nv * math.prod(self.cell_shape) + 3 * math.prod(self.face_shape)
        return torch.empty(max(self.extra_stages, 1) * nb * n1, dtype=torch.float64, device=cons.device)

    def step_stages(self, cons, bface, dt: float, stages, stream=None) -> None:
        """One step in place, also recording its stage inputs into `stages`
        (from stages_like) for step_vjp."""
        pc, pb, nb = self._pair(cons, bface)
        ps = self._flat(stages)
        _check(lib().athmhd_step_stages(self._h, pc, pb, float(dt), ps, nb, _stream(stream)), self._h)

    def _flat(self, t):
        import torch
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda or not t.is_contiguous():
            raise TypeError("expected a contiguous float64 tensor in HIP device memory")
        return C.c_void_p(t.data_ptr())

    def step_vjp(self, cons, bface, dt: float, g_cons, g_bface, out_cons=None, out_bface=None, stages=None,
                 stream=None):
        """Cotangents of (cons, bface) at the start of a step of size dt, given
        the cotangents (g_cons, g_bface) of its result; out_* may be g_* (in
        place); stages: the buffer recorded by step_stages for this step, or
        None to recompute.  Returns (out_cons, out_bface)."""
        import torch
        pc, pb, nb = self._pair(cons, bface)
        ps = None if stages is None else self._flat(stages)
        gc, gb, nb2 = self._pair(g_cons, g_bface)
        if out_cons is None:
            out_cons = torch.empty_like(g_cons)
        if out_bface is None:
            out_bface = torch.empty_like(g_bface)
        oc, ob, nb3 = self._pair(out_cons, out_bface)
        if not nb == nb2 == nb3:
            raise ValueError("state and cotangents hold different block counts")
        _check(lib().athmhd_step_vjp(self._h, pc, pb, float(dt), ps, gc, gb, oc, ob, nb, _stream(stream)), self._h)
        return out_cons, out_bface

    def prim2cons_vjp(self, prim, bface, g_cons, g_bface, out_prim=None, stream=None):
        """Cotangent of prim for cons = prim2cons(prim, bface); the face-field
        part is added to g_bface in place.  Returns out_prim."""
        import torch
        pp, pb, nb = self._pair(prim, bface)
        gc, _ = self._arr(g_cons, self.nv, self.cell_shape)
        gbp, _ = self._arr(g_bface, 3, self.face_shape)
        if out_prim is None:
            out_prim = torch.empty_like(prim)
        op, _ = self._arr(out_prim, self.nv, self.cell_shape)
        _check(lib().athmhd_prim2cons_vjp(self._h, pp, pb, gc, op, gbp, nb, _stream(stream)), self._h)
        return out_prim

    def set_floors(self, dfloor: float, pfloor: float) -> None:
        """Optional density / pressure floors on the primitives (0, 0: off)."""
        _check(lib().athmhd_set_floors(self._h, float(dfloor), float(pfloor)), self._h)

    def floor_count(self, stream=None) -> int:
        """Floor activations since the previous call (synchronises)."""
        n = C.c_longlong()
        _check(lib().athmhd_floor_count(self._h, C.byref(n), _stream(stream)), self._h)
        return n.value

    def set_graph(self, enable: bool) -> None:
        """Record the step once into a hipGraph and replay it (needs a
        non-default stream)."""
        _check(lib().athmhd_set_graph(self._h, int(bool(enable))), self._h)

    def profile_start(self) -> None:
        _check(lib().athmhd_profile(self._h, 1, None, None), self._h)

    def profile_stop(self):
        """(summed stage-kernel milliseconds, number of launches) since start"""
        ms = C.c_double()
        n = C.c_int()
        _check(lib().athmhd_profile(self._h, 0, C.byref(ms), C.byref(n)), self._h)
        return ms.value, n.value

    def close(self):
        if getattr(self, "_h", None):
            lib().athmhd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class MeshSolver(Solver):
    """A coupled mesh: mesh = (nbx, nby, nbz) equal blocks of n cells tiling one
    periodic domain; block b = bx + nbx (by + nby bz).  Tensors hold all
    blocks: cons (nb, 5 + nscalars, N3, N2, N1), bface (nb, 3, N3+1, N2+1, N1+1).  Before
    every stage the library exchanges ghost cells and faces between the
    blocks (see athmhd_create_mesh)."""

    def __init__(self, n, mesh, nghost, dx, gamma, recon="plm", riemann="hlld", integrator="vl2", cfl=0.3,
                 ct_eps=0.0, nscalars=0):
        self.n = tuple(int(x) for x in n)
        self.mesh = tuple(int(x) for x in mesh)
        self.ng = int(nghost)
        self.nblocks = self.mesh[0] * self.mesh[1] * self.mesh[2]
        self.nv = 5 + int(nscalars)
        self.cfg = make_config(n, nghost, dx, gamma, recon, riemann, integrator, cfl, ct_eps, "fused", nscalars)
        h = C.c_void_p()
        rc = lib().athmhd_create_mesh(C.byref(self.cfg), self.mesh[0], self.mesh[1], self.mesh[2], C.byref(h))
        if rc != OK:
            raise AthmhdError(rc, lib().athmhd_last_error(None).decode(errors="replace"))
        self._h = h


class TwoLevelSolver(Solver):
    """A two-level composite (see athmhd_create_levels): block 0 coarse with
    widths dx, blocks 1 + a + 2b + 4c fine with widths dx / 2, all of n
    cells.  Tensors hold the nine blocks: cons (9, 5, N3, N2, N1), bface
    (9, 3, N3+1, N2+1, N1+1)."""

    def __init__(self, n, nghost, dx, gamma, recon="plm", riemann="hlld", integrator="vl2", cfl=0.3, ct_eps=0.0,
                 charac=False):
        self.n = tuple(int(x) for x in n)
        self.ng = int(nghost)
        self.nblocks = 9
        self.nv = 5
        self.cfg = make_config(n, nghost, dx, gamma, recon, riemann, integrator, cfl, ct_eps, "unfused", 0, charac)
        h = C.c_void_p()
        rc = lib().athmhd_create_levels(C.byref(self.cfg), C.byref(h))
        if rc != OK:
            raise AthmhdError(rc, lib().athmhd_last_error(None).decode(errors="replace"))
        self._h = h


class BatchSolver:
    """Blocks of uneven sizes advanced together (one persistent launch per
    stage).  cons / bface are flat float64 tensors: the concatenation of every
    block's (5 + nscalars, N3, N2, N1) and (3, N3+1, N2+1, N1+1) arrays."""

    def __init__(self, dims, dxs, nghost, gamma, recon="plm", riemann="hlld", integrator="vl2", cfl=0.3,
                 ct_eps=0.0, nscalars=0):
        import numpy as np
        self.dims = [tuple(int(x) for x in d) for d in dims]
        self.ng = int(nghost)
        self.nblocks = len(self.dims)
        self.nv = 5 + int(nscalars)
        self.cfg = make_config(self.dims[0], nghost, dxs[0], gamma, recon, riemann, integrator, cfl, ct_eps,
                               "fused", nscalars)
        d = np.ascontiguousarray(np.array(self.dims, dtype=np.int32).reshape(-1))
        x = np.ascontiguousarray(np.array(dxs, dtype=np.float64).reshape(-1))
        h = C.c_void_p()
        rc = lib().athmhd_create_batch(C.byref(self.cfg), d.ctypes.data_as(C.POINTER(C.c_int32)),
                                       x.ctypes.data_as(C.POINTER(C.c_double)), self.nblocks, C.byref(h))
        if rc != OK:
            raise AthmhdError(rc, lib().athmhd_last_error(None).decode(errors="replace"))
        self._h = h
        cl, bl = C.c_int64(), C.c_int64()
        offs = (C.c_int64 * (2 * self.nblocks))()
        _check(lib().athmhd_batch_info(self._h, C.byref(cl), C.byref(bl), offs), self._h)
        self.cons_len, self.bface_len = cl.value, bl.value
        self.offsets = [(offs[2 * b], offs[2 * b + 1]) for b in range(self.nblocks)]

    def cell_shape(self, b):
        n1, n2, n3 = self.dims[b]
        g = self.ng
        return (n3 + 2 * g, n2 + 2 * g, n1 + 2 * g)

    def face_shape(self, b):
        return tuple(x + 1 for x in self.cell_shape(b))

    def views(self, flat, kind):
        """Per-block views (5 + nscalars, ...) of a flat cons-like array or
        (3, ...) of a flat bface-like array (numpy or torch)."""
        out = []
        for b in range(self.nblocks):
            if kind == "cons":
                o, sh, nv = self.offsets[b][0], self.cell_shape(b), self.nv
            else:
                o, sh, nv = self.offsets[b][1], self.face_shape(b), 3
            n = nv * sh[0] * sh[1] * sh[2]
            out.append(flat[o:o + n].reshape((nv,) + sh))
        return out

    def _flat(self, t, n):
        import torch
        if not isinstance(t, torch.Tensor) or t.dtype != torch.float64 or not t.is_cuda:
            raise TypeError("expected a float64 tensor in HIP device memory")
        if not t.is_contiguous() or t.numel() != n:
            raise ValueError(f"expected a contiguous tensor of {n} elements")
        return C.c_void_p(t.data_ptr())

    def _pair(self, cons, bface):
        return self._flat(cons, self.cons_len), self._flat(bface, self.bface_len)

    def step(self, cons, bface, dt: float, stream=None) -> None:
        pc, pb = self._pair(cons, bface)
        _check(lib().athmhd_step(self._h, pc, pb, float(dt), self.nblocks, _stream(stream)), self._h)

    def step_chain(self, cons, bface, dt_dev, nbad_out=None, stream=None) -> None:
        pc, pb = self._pair(cons, bface)
        nbp = None if nbad_out is None else _scalar_out(nbad_out, "int32")
        _check(lib().athmhd_step_chain(self._h, pc, pb, self.nblocks, _scalar_out(dt_dev, "float64"), nbp,
                                       _stream(stream)), self._h)

    def newdt(self, cons, bface, stream=None) -> float:
        pc, pb = self._pair(cons, bface)
        out = C.c_double()
        _check(lib().athmhd_newdt(self._h, pc, pb, self.nblocks, C.byref(out), _stream(stream)), self._h)
        return out.value

    def newdt_noalloc(self, cons, bface, dt_out, nbad_out, stream=None) -> None:
        pc, pb = self._pair(cons, bface)
        _check(lib().athmhd_newdt_noalloc(self._h, pc, pb, self.nblocks, _scalar_out(dt_out, "float64"),
                                          _scalar_out(nbad_out, "int32"), _stream(stream)), self._h)

    def prim2cons(self, prim, bface, out=None, stream=None):
        import torch
        pp, pb = self._pair(prim, bface)
        if out is None:
            out = torch.empty_like(prim)
        po = self._flat(out, self.cons_len)
        _check(lib().athmhd_prim2cons(self._h, pp, pb, po, self.nblocks, _stream(stream)), self._h)
        return out

    def fill_ghosts(self, cons, bface, stream=None) -> None:
        pc, pb = self._pair(cons, bface)
        _check(lib().athmhd_fill_ghosts(self._h, pc, pb, self.nblocks, _stream(stream)), self._h)

    def couple(self, origins, domain) -> None:
        """Make the blocks one periodic mesh: origins[b] is block b's first
        active cell in the domain of domain[0] x domain[1] x domain[2] cells
        (x1 first), which the blocks must tile exactly."""
        import numpy as np
        o = np.ascontiguousarray(np.array(origins, dtype=np.int32).reshape(-1))
        d = np.ascontiguousarray(np.array(domain, dtype=np.int32).reshape(3))
        if o.size != 3 * self.nblocks:
            raise ValueError(f"expected {self.nblocks} origins")
        _check(lib().athmhd_batch_couple(self._h, o.ctypes.data_as(C.POINTER(C.c_int32)),
                                         d.ctypes.data_as(C.POINTER(C.c_int32))), self._h)

    def set_tile(self, shape: int, split: int = 0) -> None:
        _check(lib().athmhd_batch_set_tile(self._h, int(shape), int(split)), self._h)

    def tune(self, cons, bface, stream=None):
        """Time every tile candidate on this state, keep the fastest; returns
        (shape, split, ms per stage)."""
        pc, pb = self._pair(cons, bface)
        sh, sp, ms = C.c_int(), C.c_int(), C.c_double()
        _check(lib().athmhd_batch_tune(self._h, pc, pb, _stream(stream), C.byref(sh), C.byref(sp), C.byref(ms)),
               self._h)
        return sh.value, sp.value, ms.value

    def set_floors(self, dfloor: float, pfloor: float) -> None:
        """Optional density / pressure floors on the primitives (0, 0: off)."""
        _check(lib().athmhd_set_floors(self._h, float(dfloor), float(pfloor)), self._h)

    def floor_count(self, stream=None) -> int:
        """Floor activations since the previous call (synchronises)."""
        n = C.c_longlong()
        _check(lib().athmhd_floor_count(self._h, C.byref(n), _stream(stream)), self._h)
        return n.value

    def set_graph(self, enable: bool) -> None:
        _check(lib().athmhd_set_graph(self._h, int(bool(enable))), self._h)

    def profile_start(self) -> None:
        _check(lib().athmhd_profile(self._h, 1, None, None), self._h)

    def profile_stop(self):
        ms = C.c_double()
        n = C.c_int()
        _check(lib().athmhd_profile(self._h, 0, C.byref(ms), C.byref(n)), self._h)
        return ms.value, n.value

    def close(self):
        if getattr(self, "_h", None):
            lib().athmhd_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
