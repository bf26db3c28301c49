"""Reverse mode of the step (athmhd_step_vjp), of prim -> cons
(athmhd_prim2cons_vjp) and the checkpointed rollout, checked against the CPU
oracle's exact directional derivatives (forward-mode dual numbers run through
the oracle's own step) and against central finite differences.

Transposition is checked two ways:
  * a full Jacobian assembled column by column from oracle JVPs on a tiny
    block, compared element by element with the GPU's J^T w;
  * the dot-product identity <w, J d> = <J^T w, d> on larger blocks.
"""
import numpy as np
import pytest

from paper_2005_06651_amd import inputs

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


def active_masks(n, ng):
    """Boolean masks of the independent entries: active cells of cons and the
    lower face of every active cell in bface."""
    n1, n2, n3 = n
    N = (n3 + 2 * ng, n2 + 2 * ng, n1 + 2 * ng)
    mc = np.zeros((5,) + N, bool)
    mc[:, ng:ng + n3, ng:ng + n2, ng:ng + n1] = True
    mb = np.zeros((3,) + tuple(x + 1 for x in N), bool)
    mb[:, ng:ng + n3, ng:ng + n2, ng:ng + n1] = True
    return mc, mb


def random_active(rng, mc, mb):
    c = np.zeros(mc.shape)
    b = np.zeros(mb.shape)
    c[mc] = rng.standard_normal(int(mc.sum()))
    b[mb] = rng.standard_normal(int(mb.sum()))
    return c, b


def oracle_jvp(orc, cfg, cons, bface, dc, db, dt):
    c, b, x, y = cons.copy(), bface.copy(), dc.copy(), db.copy()
    assert orc.step_jvp(cfg, c, b, x, y, dt) == 0
    return x, y


def gpu_vjp(torch, dev, s, cons, bface, wc, wb, dt):
    tc = torch.from_numpy(cons).to(dev)
    tb = torch.from_numpy(bface).to(dev)
    gc, gb = s.step_vjp(tc, tb, dt, torch.from_numpy(wc).to(dev), torch.from_numpy(wb).to(dev))
    return gc.cpu().numpy(), gb.cpu().numpy()


SCHEMES = [
    ("vl2", "plm", "hlld", 1e-3),
    ("vl2", "plm", "hlld", 0.0),
    ("rk3", "plm", "hlle", 1e-2),
    ("rk2", "dc", "hlle", 0.0),
    ("rk1", "dc", "hlld", 1e-3),
]


@pytest.mark.parametrize("integ,recon,rs,eps", SCHEMES)
def test_full_jacobian_transpose_tiny_block(torch_dev, athmhd, orc, integ, recon, rs, eps):
    """Every column of J from the oracle; J^T w from the GPU, element by element."""
    torch, dev = torch_dev
    blk = inputs.smooth_random(n=(5, 4, 3), seed=21, ng=2, vmax=0.6)
    kw = dict(integrator=integ, recon=recon, riemann=rs, ct_eps=eps)
    cfg = orc.cfg_for(blk, **kw)
    cons = orc.prim2cons(cfg, blk.prim, blk.bface)
    dt = 0.5 * orc.newdt(cfg, cons, blk.bface)[0]
    mc, mb = active_masks(blk.n, blk.ng)
    idx_c = np.flatnonzero(mc)
    idx_b = np.flatnonzero(mb)
    nin = idx_c.size + idx_b.size
    J = np.zeros((nin, nin))  # J[out, in]
    for col in range(nin):
        dc = np.zeros(mc.shape)
        db = np.zeros(mb.shape)
        if col < idx_c.size:
            dc.flat[idx_c[col]] = 1.0
        else:
            db.flat[idx_b[col - idx_c.size]] = 1.0
        jc, jb = oracle_jvp(orc, cfg, cons, blk.bface, dc, db, dt)
        J[:, col] = np.concatenate([jc.flat[idx_c], jb.flat[idx_b]])
    s = athmhd.Solver(blk.n, blk.ng, blk.dx, blk.gamma, **kw)
    rng = np.random.default_rng(5)
    for _ in range(3):
        wc, wb = random_active(rng, mc, mb)
        gc, gb = gpu_vjp(torch, dev, s, cons, blk.bface, wc, wb, dt)
        ref = J.T @ np.concatenate([wc.flat[idx_c], wb.flat[idx_b]])
        got = np.concatenate([gc.flat[idx_c], gb.flat[idx_b]])
        scale = np.abs(J.T).dot(np.abs(np.concatenate([wc.flat[idx_c], wb.flat[idx_b]])))
        assert np.all(np.abs(got - ref) <= 1e-12 * scale + 1e-300), np.max(np.abs(got - ref) / scale)
        # entries that are not independent pass their cotangent through
        assert np.array_equal(gc[~mc], wc[~mc]) and np.array_equal(gb[~mb], wb[~mb])
    s.close()


@pytest.mark.parametrize("integ,recon,rs,eps", SCHEMES)
def test_dot_product_identity(torch_dev, athmhd, orc, integ, recon, rs, eps):
    """<w, J d> (oracle, forward mode) = <J^T w, d> (GPU, reverse mode) on a
    block spanning several tiles with ragged extents."""
    torch, dev = torch_dev
    blk = inputs.smooth_random(n=(18, 13, 11), seed=22, ng=2)
    kw = dict(integrator=integ, recon=recon, riemann=rs, ct_eps=eps)
    cfg = orc.cfg_for(blk, **kw)
    cons = orc.prim2cons(cfg, blk.prim, blk.bface)
    dt = orc.newdt(cfg, cons, blk.bface)[0]
    mc, mb = active_masks(blk.n, blk.ng)
    s = athmhd.Solver(blk.n, blk.ng, blk.dx, blk.gamma, **kw)
    rng = np.random.default_rng(6)
    wc, wb = random_active(rng, mc, mb)
    gc, gb = gpu_vjp(torch, dev, s, cons, blk.bface, wc, wb, dt)
    for _ in range(4):
        dc, db = random_active(rng, mc, mb)
        jc, jb = oracle_jvp(orc, cfg, cons, blk.bface, dc, db, dt)
        lhs = np.sum(wc[mc] * jc[mc]) + np.sum(wb[mb] * jb[mb])
        rhs = np.sum(gc[mc] * dc[mc]) + np.sum(gb[mb] * db[mb])
        scale = np.sum(np.abs(wc[mc] * jc[mc])) + np.sum(np.abs(wb[mb] * jb[mb]))
        assert abs(lhs - rhs) <= 1e-12 * scale, (lhs, rhs, scale)
    s.close()


def test_multi_block_vjp_equals_single_blocks(torch_dev, athmhd, orc):
    torch, dev = torch_dev
    blocks = [inputs.smooth_random(n=(12, 10, 8), seed=30 + b, ng=2) for b in range(3)]
    b0 = blocks[0]
    kw = dict(integrator="vl2", recon="plm", riemann="hlld", ct_eps=1e-3)
    cfg = orc.cfg_for(b0, **kw)
    cons = np.stack([orc.prim2cons(cfg, b.prim, b.bface) for b in blocks])
    bf = np.stack([b.bface for b in blocks])
    mc, mb = active_masks(b0.n, b0.ng)
    rng = np.random.default_rng(7)
    w = [random_active(rng, mc, mb) for _ in blocks]
    wc = np.stack([x[0] for x in w])
    wb = np.stack([x[1] for x in w])
    dt = 1e-3
    s = athmhd.Solver(b0.n, b0.ng, b0.dx, b0.gamma, nblocks=3, **kw)
    gc, gb = gpu_vjp(torch, dev, s, cons, bf, wc, wb, dt)
    s1 = athmhd.Solver(b0.n, b0.ng, b0.dx, b0.gamma, **kw)
    for b in range(3):
        c1, g1 = gpu_vjp(torch, dev, s1, cons[b], bf[b], wc[b], wb[b], dt)
        assert np.array_equal(c1, gc[b]) and np.array_equal(g1, gb[b])
    s.close()
    s1.close()


@pytest.mark.parametrize("integ", ["vl2", "rk3", "rk1"])
def test_recorded_stages_give_the_same_vjp(torch_dev, athmhd, orc, integ):
    """step_stages records the stage inputs; step_vjp with them equals
    step_vjp recomputing them, bitwise, and step_stages advances the state
    exactly like step."""
    torch, dev = torch_dev
    blk = inputs.smooth_random(n=(20, 14, 9), seed=28, ng=2)
    kw = dict(integrator=integ, recon="plm", riemann="hlld", ct_eps=1e-3)
    cfg = orc.cfg_for(blk, **kw)
    cons = orc.prim2cons(cfg, blk.prim, blk.bface)
    s = athmhd.Solver(blk.n, blk.ng, blk.dx, blk.gamma, **kw)
    tc = torch.from_numpy(cons).to(dev)
    tb = torch.from_numpy(blk.bface).to(dev)
    dt = s.newdt(tc, tb)
    mc, mb = active_masks(blk.n, blk.ng)
    rng = np.random.default_rng(13)
    wc, wb = random_active(rng, mc, mb)
    twc, twb = torch.from_numpy(wc).to(dev), torch.from_numpy(wb).to(dev)
    g0 = s.step_vjp(tc, tb, dt, twc, twb)
    st = s.stages_like(tc)
    c2, b2 = tc.clone(), tb.clone()
    s.step_stages(c2, b2, dt, st)
    c3, b3 = tc.clone(), tb.clone()
    s.step(c3, b3, dt)
    assert torch.equal(c2, c3) and torch.equal(b2, b3)
    g1 = s.step_vjp(tc, tb, dt, twc, twb, stages=st if s.extra_stages else None)
    assert torch.equal(g0[0], g1[0]) and torch.equal(g0[1], g1[1])
    s.close()


def test_prim2cons_vjp_by_differences(torch_dev, athmhd, orc):
    """prim -> cons is a cubic polynomial along any line, so a central
    difference with a small step is exact up to rounding."""
    torch, dev = torch_dev
    blk = inputs.smooth_random(n=(9, 7, 6), seed=23, ng=2)
    cfg = orc.cfg_for(blk)
    s = athmhd.Solver(blk.n, blk.ng, blk.dx, blk.gamma)
    rng = np.random.default_rng(8)
    gcons = rng.standard_normal(blk.prim.shape)
    gbf0 = rng.standard_normal(blk.bface.shape)
    tg_b = torch.from_numpy(gbf0.copy()).to(dev)
    gp = s.prim2cons_vjp(torch.from_numpy(blk.prim).to(dev), torch.from_numpy(blk.bface).to(dev),
                         torch.from_numpy(gcons).to(dev), tg_b).cpu().numpy()
    gb = tg_b.cpu().numpy() - gbf0  # the face part is accumulated
    for _ in range(3):
        dp = rng.standard_normal(blk.prim.shape)
        db = rng.standard_normal(blk.bface.shape)
        h = 1e-5
        up = orc.prim2cons(cfg, blk.prim + h * dp, blk.bface + h * db)
        um = orc.prim2cons(cfg, blk.prim - h * dp, blk.bface - h * db)
        fd = np.sum(gcons * (up - um)) / (2 * h)
        ad = np.sum(gp * dp) + np.sum(gb * db)
        assert abs(fd - ad) <= 1e-8 * np.sum(np.abs(gcons * (up - um)) / (2 * h)), (fd, ad)
    s.close()


def test_vjp_rejects_unsupported_and_aliasing(torch_dev, athmhd):
    torch, dev = torch_dev
    blk = inputs.smooth_random(n=(8, 8, 8), seed=24, ng=3)
    s = athmhd.Solver(blk.n, blk.ng, blk.dx, blk.gamma, recon="ppm", integrator="rk3")
    c = torch.zeros((5,) + s.cell_shape, dtype=torch.float64, device=dev)
    b = torch.zeros((3,) + s.face_shape, dtype=torch.float64, device=dev)
    with pytest.raises(athmhd.AthmhdError) as ei:
        s.step_vjp(c, b, 0.1, c.clone(), b.clone())
    assert ei.value.code == athmhd.EUNSUP
    s.close()
    s = athmhd.Solver(blk.n, blk.ng, blk.dx, blk.gamma)
    with pytest.raises(athmhd.AthmhdError) as ei:
        s.step_vjp(c, b, 0.1, c.clone(), b.clone(), out_cons=c)
    assert ei.value.code == athmhd.EINVAL
    s.close()


def test_rollout_checkpointing_and_finite_differences(torch_dev, athmhd, orc):
    """Gradient of a density mismatch after a rollout with respect to the
    initial velocity (through prim -> cons): checkpointed backward equals the
    plain reverse sweep bitwise, and central differences agree to 1e-6."""
    torch, dev = torch_dev
    from paper_2005_06651_amd.rollout import Prim2Cons, Rollout
    n, nsteps = 16, 8
    blk = inputs.turbulence(n=n, seed=25, mach=0.3)
    s = athmhd.Solver(blk.n, blk.ng, blk.dx, blk.gamma, ct_eps=1e-3)
    prim0 = torch.from_numpy(blk.prim).to(dev)
    bf0 = torch.from_numpy(blk.bface).to(dev)
    cons0 = s.prim2cons(prim0, bf0)
    dt = s.newdt(cons0, bf0)
    g = blk.ng
    rng = np.random.default_rng(9)
    target = torch.from_numpy(1.0 + 0.05 * rng.standard_normal((n, n, n))).to(dev)
    dV = blk.dx[0] * blk.dx[1] * blk.dx[2]

    def loss_of(prim, ncheck):
        c0 = Prim2Cons.apply(prim, bf0, s)
        cN, _ = Rollout.apply(c0, bf0, s, dt, nsteps, ncheck)
        rho = cN[0, g:g + n, g:g + n, g:g + n]
        return ((rho - target) ** 2).sum() * dV

    grads = []
    for ncheck in (3, nsteps):
        p = prim0.clone().requires_grad_(True)
        loss_of(p, ncheck).backward()
        grads.append(p.grad.detach().clone())
    assert torch.equal(grads[0], grads[1])
    grad_v = grads[0][1:4, g:g + n, g:g + n, g:g + n].cpu().numpy()
    for _ in range(3):
        d = rng.standard_normal((3, n, n, n))
        d /= np.linalg.norm(d)
        ad = float(np.sum(grad_v * d))
        best = None
        for h in (1e-3, 1e-4, 1e-5):
            dp = torch.zeros_like(prim0)
            dp[1:4, g:g + n, g:g + n, g:g + n] = torch.from_numpy(h * d).to(dev)
            with torch.no_grad():
                lp = loss_of(prim0 + dp, nsteps).item()
                lm = loss_of(prim0 - dp, nsteps).item()
            fd = (lp - lm) / (2 * h)
            err = abs(fd - ad) / max(abs(ad), 1e-300)
            best = err if best is None else min(best, err)
        assert best <= 1e-6, (best, ad)
    s.close()


def test_rollout_gradient_matches_oracle_directional_derivative(torch_dev, athmhd, orc):
    """<grad_v L, d> from the GPU reverse mode (Prim2Cons + checkpointed
    Rollout) equals the exact directional derivative from the oracle's
    forward-mode dual numbers run through the same rollout on the CPU."""
    torch, dev = torch_dev
    from paper_2005_06651_amd.rollout import Prim2Cons, Rollout
    n, nsteps, eps = 24, 6, 1e-3
    blk = inputs.turbulence(n=n, seed=26, mach=0.3)
    kw = dict(integrator="vl2", recon="plm", riemann="hlld", ct_eps=eps)
    s = athmhd.Solver(blk.n, blk.ng, blk.dx, blk.gamma, **kw)
    cfg = orc.cfg_for(blk, **kw)
    g = blk.ng
    prim0 = torch.from_numpy(blk.prim).to(dev)
    bf0 = torch.from_numpy(blk.bface).to(dev)
    cons_np = orc.prim2cons(cfg, blk.prim, blk.bface)
    dt = orc.newdt(cfg, cons_np, blk.bface)[0]
    rng = np.random.default_rng(11)
    target_np = 1.0 + 0.05 * rng.standard_normal((n, n, n))
    target = torch.from_numpy(target_np).to(dev)
    dV = blk.dx[0] * blk.dx[1] * blk.dx[2]
    p = prim0.clone().requires_grad_(True)
    cN, _ = Rollout.apply(Prim2Cons.apply(p, bf0, s), bf0, s, dt, nsteps, 2)
    loss = ((cN[0, g:g + n, g:g + n, g:g + n] - target) ** 2).sum() * dV
    loss.backward()
    grad_v = p.grad[1:4, g:g + n, g:g + n, g:g + n].cpu().numpy()
    act = (slice(g, g + n),) * 3
    rho0 = blk.prim[0][act]
    v0 = blk.prim[1:4][(slice(None),) + act]
    for _ in range(2):
        d = rng.standard_normal((3, n, n, n))
        # tangent of cons for a velocity change d: dM = rho d, dE = rho v . d
        dc = np.zeros_like(cons_np)
        dc[(slice(1, 4),) + act] = rho0 * d
        dc[(4,) + act] = rho0 * np.sum(v0 * d, axis=0)
        db = np.zeros_like(blk.bface)
        c, b = cons_np.copy(), blk.bface.copy()
        for _ in range(nsteps):
            assert orc.step_jvp(cfg, c, b, dc, db, dt) == 0
        exact = float(np.sum(2.0 * (c[(0,) + act] - target_np) * dc[(0,) + act]) * dV)
        got = float(np.sum(grad_v * d))
        assert abs(got - exact) <= 1e-10 * abs(exact), (got, exact)
    s.close()
