"""Roe's linearised solver on the GPU (Sec. 3.2.2; reading R-34) against the
oracle: the closed-form eigenvector split of the kernels against the oracle's
explicit Roe matrix and matrix-sign iteration, at the 1e-12 bar with the
element-wise bar beside it, on the fused and unfused pipelines, with
characteristic reconstruction, on the linear wave and on turbulence."""
import numpy as np
import pytest

from paper_2005_06651_amd import inputs
from test_gpu_parity import ELEM_TOL, TOL, elem_rel, rel_l1, rms_l1_rel, to_dev

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a HIP device"
    return torch, torch.device("cuda:0")


@pytest.fixture(scope="module")
def athmhd():
    from paper_2005_06651_amd import athmhd as A
    A.lib()
    return A


def _steps(torch, dev, athmhd, orc, b, nsteps, path="fused", charac=False, **kw):
    s = athmhd.Solver(b.n, b.ng, b.dx, b.gamma, kernel_path=path, charac=charac, **kw)
    cfg = orc.cfg_for(b, charac=charac, **kw)
    cons = orc.prim2cons(cfg, b.prim, b.bface) if b.cons is None else b.cons.copy()
    tc, tb = to_dev(torch, dev, cons), to_dev(torch, dev, b.bface)
    rc, rb = cons.copy(), b.bface.copy()
    for _ in range(nsteps):
        dt, bad = orc.newdt(cfg, rc, rb)
        assert bad == 0
        assert orc.step(cfg, rc, rb, dt) == 0
        s.step(tc, tb, dt)
    gc, gb = tc.cpu().numpy(), tb.cpu().numpy()
    s.fill_ghosts(tc, tb)
    divb = inputs.divb_metric(tb.cpu().numpy(), b.n, b.ng, b.dx)
    s.close()
    return gc, gb, rc, rb, divb


@pytest.mark.parametrize("integ,recon,path,charac", [
    ("vl2", "plm", "fused", False),
    ("rk1", "dc", "fused", False),
    ("rk3", "ppm", "fused", False),
    ("vl2", "plm", "unfused", False),
    ("vl2", "plm", "fused", True),
])
def test_roe_steps_match_oracle(torch_dev, athmhd, orc, integ, recon, path, charac):
    """Three steps of a ragged 37 x 19 x 11 block of smooth random data."""
    torch, dev = torch_dev
    b = inputs.smooth_random(n=(37, 19, 11), seed=101, ng=3 if recon == "ppm" else 2)
    gc, gb, rc, rb, divb = _steps(torch, dev, athmhd, orc, b, 3, path, charac, integrator=integ, recon=recon,
                                  riemann="roe")
    err, el = rel_l1(b, gc, gb, rc, rb), elem_rel(b, gc, gb, rc, rb)
    print(f"Roe {integ}+{recon} {path}{' charac' if charac else ''}: rel L1 {err:.2e}, element-wise {el:.2e}")
    assert err <= TOL and el <= ELEM_TOL
    assert divb <= 1e-13


def test_roe_degenerate_fields_match_oracle(torch_dev, athmhd, orc):
    """No transverse field on the x1-faces and B_n = 0 (the averaged transverse
    field direction and the coinciding wave speeds take their fallbacks)."""
    torch, dev = torch_dev
    for b in (inputs.x1_profile(n=(40, 6, 5), seed=102, base=(1.2, 0.1, 0.0, 0.0, 0.3, 0.0, 0.0),
                                amp=(0.3, 0.2, 0.4, 0.3, 0.2, 0.0, 0.0), b1=2.5),
              inputs.x1_profile(n=(40, 6, 5), seed=103, base=(1.0, 0.1, 0.0, 0.0, 1.0, 0.4, -0.3),
                                amp=(0.5, 0.3, 0.4, 0.3, 0.4, 0.6, 0.5), b1=0.0)):
        gc, gb, rc, rb, divb = _steps(torch, dev, athmhd, orc, b, 4, integrator="vl2", recon="plm", riemann="roe")
        from test_gpu_parity import rel_l1_nonzero
        err, el = rel_l1_nonzero(b, gc, gb, rc, rb), elem_rel(b, gc, gb, rc, rb)
        print(f"Roe degenerate: rel L1 {err:.2e}, element-wise {el:.2e}")
        assert err <= TOL and el <= ELEM_TOL
        assert divb <= 1e-13


def test_roe_linear_wave_one_period(torch_dev, athmhd, orc):
    """16 x 8 x 8 fast linear wave, VL2 + PLM + Roe, one period, dt from each
    side's own newdt; the state-level norm of Eq. (RMS-error), made relative."""
    torch, dev = torch_dev
    b = inputs.linear_wave(8)
    kw = dict(integrator="vl2", recon="plm", riemann="roe", cfl=0.3)
    s = athmhd.Solver(b.n, b.ng, b.dx, b.gamma, **kw)
    cfg = orc.cfg_for(b, **kw)
    rc, rb, t, nsteps = orc.run(cfg, b.cons, b.bface, 0, t_end=0.5)
    tc, tb = to_dev(torch, dev, b.cons), to_dev(torch, dev, b.bface)
    tt, steps = 0.0, 0
    while tt < 0.5 * (1 - 1e-14):
        dt = min(s.newdt(tc, tb), 0.5 - tt)
        s.step(tc, tb, dt)
        tt += dt
        steps += 1
    assert steps == nsteps
    s.fill_ghosts(tc, tb)
    gc, gb = tc.cpu().numpy(), tb.cpu().numpy()
    assert rms_l1_rel(b, gc, gb, rc, rb) <= TOL
    s.close()


def test_roe_turbulence_matches_oracle(torch_dev, athmhd, orc):
    """Turbulence recipe at 20^3, five VL2 + PLM + Roe steps."""
    torch, dev = torch_dev
    b = inputs.turbulence(n=20, seed=7)
    gc, gb, rc, rb, divb = _steps(torch, dev, athmhd, orc, b, 5, integrator="vl2", recon="plm", riemann="roe")
    err, el = rel_l1(b, gc, gb, rc, rb), elem_rel(b, gc, gb, rc, rb)
    print(f"Roe turbulence 20^3 x 5: rel L1 {err:.2e}, element-wise {el:.2e}")
    assert err <= TOL and el <= ELEM_TOL
    assert divb <= 1e-13


def test_roe_unsupported_uses(torch_dev, athmhd, orc):
    torch, dev = torch_dev
    blocks = inputs.amr_batch(3, seed=2)
    with pytest.raises(athmhd.AthmhdError) as e:
        athmhd.BatchSolver([x.n for x in blocks], [x.dx for x in blocks], 2, blocks[0].gamma, riemann="roe")
    assert e.value.code == athmhd.EUNSUP
    b = inputs.smooth_random(n=(8, 8, 8), seed=104)
    s = athmhd.Solver(b.n, b.ng, b.dx, b.gamma, riemann="roe")
    tb = to_dev(torch, dev, b.bface)
    tc = s.prim2cons(to_dev(torch, dev, b.prim), tb)
    with pytest.raises(athmhd.AthmhdError) as e:
        s.step_vjp(tc, tb, 1e-3, tc.clone(), tb.clone())
    assert e.value.code == athmhd.EUNSUP
    s.close()
