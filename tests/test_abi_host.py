"""Host-side checks of the C ABI that need no GPU: the library loads, exports
every symbol that include/athmhd.h declares, and rejects bad configurations
and calls before touching the HIP runtime."""
import ctypes as C
import os
import re

import pytest

from paper_2005_06651_amd import athmhd

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    out = []
    for name in os.listdir(os.path.join(ROOT, "include")):
        if name.endswith(".h"):
            text = open(os.path.join(ROOT, "include", name)).read()
            out += re.findall(r"ATHMHD_API\s+[\w\s\*]*?\b(athmhd_\w+)\s*\(", text)
    return sorted(set(out))


def test_library_exports_every_declared_symbol():
    L = athmhd.lib()
    syms = declared_symbols()
    assert len(syms) >= 8
    for s in syms:
        assert hasattr(L, s), s
    assert set(athmhd.EXPORTED) <= set(syms)


def test_version():
    assert athmhd.lib().athmhd_version() == 112


def _create(**over):
    kw = dict(n=(8, 8, 8), nghost=2, dx=(0.1, 0.1, 0.1), gamma=5 / 3)
    kw.update({k: v for k, v in over.items() if k in kw})
    cfg = athmhd.make_config(**kw)
    for k, v in over.items():
        if k not in kw:
            setattr(cfg, k, v)
    h = C.c_void_p()
    rc = athmhd.lib().athmhd_create(C.byref(cfg), 1, C.byref(h))
    msg = athmhd.lib().athmhd_last_error(None).decode()
    return rc, msg


@pytest.mark.parametrize("over,needle", [
    (dict(n=(0, 8, 8)), "dims"),
    (dict(nghost=1), "nghost"),
    (dict(recon=2, nghost=2), "nghost"),
    (dict(gamma=1.0), "gamma"),
    (dict(gamma=float("nan")), "gamma"),
    (dict(dx=(0.1, 0.0, 0.1)), "widths"),
    (dict(dx=(0.1, float("inf"), 0.1)), "widths"),
    (dict(recon=7), "reconstruction"),
    (dict(riemann=3), "Riemann"),
    (dict(integrator=9), "integrator"),
    (dict(cfl=0.0), "cfl"),
    (dict(cfl=1.5), "cfl"),
    (dict(ct_eps=-1.0), "ct_eps"),
    (dict(kernel_path=2), "kernel_path"),
    (dict(n=(2000, 2000, 2000)), "too large"),
    (dict(nscalars=-1), "nscalars"),
    (dict(nscalars=65), "nscalars"),
])
def test_create_rejects_bad_config_before_any_hip_call(over, needle):
    rc, msg = _create(**over)
    assert rc == athmhd.EINVAL
    assert needle in msg


def test_scalars_need_the_fused_kernels():
    rc, msg = _create(nscalars=2, kernel_path=1)
    assert rc == athmhd.EUNSUP
    assert "scalars" in msg


@pytest.mark.parametrize("over,code,needle", [
    (dict(charac=2), athmhd.EINVAL, "charac"),
    (dict(charac=1, nscalars=1), athmhd.EUNSUP, "scalars"),
])
def test_characteristic_reconstruction_arguments(over, code, needle):
    rc, msg = _create(**over)
    assert rc == code
    assert needle in msg


def test_calls_reject_null_handle():
    L = athmhd.lib()
    out = C.c_double()
    assert L.athmhd_step(None, None, None, 0.1, 1, None) == athmhd.EINVAL
    assert L.athmhd_newdt(None, None, None, 1, C.byref(out), None) == athmhd.EINVAL
    assert L.athmhd_fill_ghosts(None, None, None, 1, None) == athmhd.EINVAL
    assert L.athmhd_prim2cons(None, None, None, None, 1, None) == athmhd.EINVAL
    assert L.athmhd_step_vjp(None, None, None, 0.1, None, None, None, None, None, 1, None) == athmhd.EINVAL
    assert L.athmhd_step_stages(None, None, None, 0.1, None, 1, None) == athmhd.EINVAL
    assert L.athmhd_prim2cons_vjp(None, None, None, None, None, None, 1, None) == athmhd.EINVAL
    L.athmhd_destroy(None)


def test_create_rejects_null_out():
    cfg = athmhd.make_config((8, 8, 8), 2, (0.1,) * 3, 5 / 3)
    assert athmhd.lib().athmhd_create(C.byref(cfg), 1, None) == athmhd.EINVAL
    assert athmhd.lib().athmhd_create(C.byref(cfg), 0, C.byref(C.c_void_p())) == athmhd.EINVAL


def _create_batch(dims, dxs, **over):
    import numpy as np
    cfg = athmhd.make_config((8, 8, 8), 2, (0.1, 0.1, 0.1), 5 / 3)
    for k, v in over.items():
        setattr(cfg, k, v)
    d = np.ascontiguousarray(np.array(dims, dtype=np.int32).reshape(-1))
    x = np.ascontiguousarray(np.array(dxs, dtype=np.float64).reshape(-1))
    h = C.c_void_p()
    rc = athmhd.lib().athmhd_create_batch(C.byref(cfg), d.ctypes.data_as(C.POINTER(C.c_int32)),
                                          x.ctypes.data_as(C.POINTER(C.c_double)), len(dims), C.byref(h))
    return rc, athmhd.lib().athmhd_last_error(None).decode()


@pytest.mark.parametrize("dims,dxs,over,code,needle", [
    ([(16, 16, 16), (0, 8, 8)], [(0.1,) * 3, (0.1,) * 3], {}, athmhd.EINVAL, "block 1"),
    ([(16, 16, 16)], [(0.1, -1.0, 0.1)], {}, athmhd.EINVAL, "widths"),
    ([(16, 16, 16)], [(0.1,) * 3], {"kernel_path": 1}, athmhd.EUNSUP, "fused"),
    ([(16, 16, 16)], [(0.1,) * 3], {"nghost": 1}, athmhd.EINVAL, "nghost"),
    ([(16, 16, 16)], [(0.1,) * 3], {"nscalars": 65}, athmhd.EINVAL, "nscalars"),
    ([(16, 16, 16)], [(0.1,) * 3], {"charac": 1}, athmhd.EUNSUP, "fused"),
])
def test_create_batch_rejects_bad_blocks(dims, dxs, over, code, needle):
    rc, msg = _create_batch(dims, dxs, **over)
    assert rc == code
    assert needle in msg


@pytest.mark.parametrize("blocks,over,code,needle", [
    ((0, 2, 2), {}, athmhd.EINVAL, "blocks per direction"),
    ((2, 2, 2), {"kernel_path": 1}, athmhd.EUNSUP, "fused"),
    ((2, 2, 2), {"nghost": 1}, athmhd.EINVAL, "nghost"),
    ((2, 2, 2), {"n1": 0}, athmhd.EINVAL, "block dims"),
    ((2, 2, 2), {"nscalars": -1}, athmhd.EINVAL, "nscalars"),
    ((2, 2, 2), {"charac": 1}, athmhd.EUNSUP, "fused"),
])
def test_create_mesh_rejects_bad_arguments_before_any_hip_call(blocks, over, code, needle):
    cfg = athmhd.make_config((8, 8, 8), 2, (0.1, 0.1, 0.1), 5.0 / 3.0)
    for k, v in over.items():
        setattr(cfg, k, v)
    h = C.c_void_p()
    rc = athmhd.lib().athmhd_create_mesh(C.byref(cfg), *blocks, C.byref(h))
    assert rc == code
    assert needle in athmhd.lib().athmhd_last_error(None).decode()
    assert athmhd.lib().athmhd_create_mesh(C.byref(cfg), 1, 1, 1, None) == athmhd.EINVAL


def test_batch_calls_reject_non_batch_use():
    L = athmhd.lib()
    assert L.athmhd_batch_set_tile(None, 0, 0) == athmhd.EINVAL
    assert L.athmhd_batch_info(None, None, None, None) == athmhd.EINVAL
    assert L.athmhd_set_graph(None, 1) == athmhd.EINVAL
    assert L.athmhd_newdt_noalloc(None, None, None, 1, None, None, None) == athmhd.EINVAL
    assert L.athmhd_step_chain(None, None, None, 1, None, None, None) == athmhd.EINVAL
    assert L.athmhd_batch_couple(None, None, None) == athmhd.EINVAL


def test_octree_is_two_to_one_balanced():
    """The batched workload's block levels come from a periodic octree in which
    touching leaves differ by at most one level."""
    from paper_2005_06651_amd import inputs
    leaves = inputs.balanced_octree(300, seed=5)
    assert len(leaves) >= 300
    maxl = max(l[0] for l in leaves)
    n = 1 << maxl
    grid = {}
    for L, i, j, k in leaves:
        s = 1 << (maxl - L)
        for a in range(i * s, (i + 1) * s):
            for b in range(j * s, (j + 1) * s):
                for c in range(k * s, (k + 1) * s):
                    grid[(a, b, c)] = L
    assert len(grid) == n ** 3  # the leaves tile the cube
    for (a, b, c), L in grid.items():
        for d in ((1, 0, 0), (0, 1, 0), (0, 0, 1), (1, 1, 0), (1, 0, 1), (0, 1, 1), (1, 1, 1)):
            M = grid[((a + d[0]) % n, (b + d[1]) % n, (c + d[2]) % n)]
            assert abs(M - L) <= 1
