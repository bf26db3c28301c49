#!/usr/bin/env python3
"""Throughput of the FP64 ideal-MHD step (VL2 + PLM + HLLD + upwind CT) on one
MI355X, in zone-cycles per second.

Workload: decaying MHD turbulence on a 256^3 periodic block (nghost 2,
gamma 5/3, rho = 1, p = 1, solenoidal velocity on 1 <= |k| <= 4 at rms Mach 1,
B = 0.5 x + curl A with rms(curl A) = 0.1), CFL 0.3.  One timed step is the
whole hot path (athmhd_step_chain): one full VL2 step (two fused stages of
cons->prim, reconstruction, HLLD fluxes, CT corner EMFs and the conservative
+ face-field update; periodic images are read in place, so no ghost-fill pass
is needed) with dt read on the device, then the CFL reduction of the new
state, which leaves the next step's dt on the device.  Inputs are resident in
HBM before the timed region.

Prints one JSON line.  Only one GPU is supported: --gpus N with N > 1 exits.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E, GB/s
FP64_VECTOR_TFLOPS = 78.6    # MI355X FP64 vector peak: 256 CU x 64 lanes x 2 flops (FMA) x 2.4 GHz
STATE_BYTES_PER_CELL = 64    # 5 conserved + 3 face-field doubles
# Algorithmic FP64 operations (add/sub, mul, div, sqrt) of one VL2+PLM+HLLD
# step per active cell, counted by `python -m oracle.count_flops 256` on this
# workload (per-cell slope form): 2560.0 per zone-cycle, i.e. 1280 per stage.
ALG_FLOPS_PER_ZONE_CYCLE = 2560.0
# HBM bytes per stage launch measured by rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE
# on this workload, scaled by the counters of a plain 1 GiB copy, and the hash
# of the stage-kernel sources they were measured on (traffic is reported only
# while the sources are unchanged).
STAGE_TRAFFIC = {"bytes_per_launch": 2.977e+09, "fetch_bytes_per_launch": 1.858e+09,
                 "write_bytes_per_launch": 1.120e+09, "fetch_scale": 1.9999, "write_scale": 1.0000,
                 "source_hash": "d9dccd87daa965a6"}
# FP64 VALU issue of the same stage launches (rocprofv3 SQ_INSTS_VALU per
# launch over 256 CUs x 2.4 GHz x the launch duration, mean of the DC and PLM
# stages) and the stage time those launches took under the profiler: with the
# traffic above they say which roof binds (the larger measured fraction).
STAGE_ISSUE = {"valu_issue_frac": 0.508, "profiled_ms_per_launch": 1.6894, "source_hash": "d9dccd87daa965a6"}
HBM_FRAC_TARGET = 0.60       # the HBM-roofline fraction the stage kernel is measured against
# The same for the level operators on the 256^3 block (per octant launch).
LEVELS_SOURCES = ("kernels_amr.hip", "common.hpp")
LEVELS_TRAFFIC = {"prolong": {"bytes_per_launch": 1.635e+09, "fetch_bytes_per_launch": 3.96e+08,
                              "write_bytes_per_launch": 1.24e+09},
                  "restrict": {"bytes_per_launch": 1.112e+09, "fetch_bytes_per_launch": 9.696e+08,
                               "write_bytes_per_launch": 1.423e+08},
                  "prolong_primitive": {"bytes_per_launch": 1.799e+09,
                                        "fetch_bytes_per_launch": 5.624e+08,
                                        "write_bytes_per_launch": 1.236e+09},
                  "fetch_scale": 1.9999, "write_scale": 1.0000, "source_hash": "52cd612e9ccca04c"}


def parse():
    p = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=100)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--n", type=int, default=256, help="cells per side of the periodic cube")
    p.add_argument("--seed", type=int, default=1)
    p.add_argument("--no-cpu-baseline", action="store_true", help="skip the CPU oracle timing")
    p.add_argument("--cpu-steps", type=int, default=1, help="oracle steps in the CPU baseline sample")
    p.add_argument("--kernel-path", default="fused", choices=["fused", "unfused"])
    p.add_argument("--workload", default="turbulence",
                   choices=["turbulence", "batch", "adjoint", "blast", "mesh", "levels"],
                   help="turbulence: the 256^3 block (default); batch: 1024 uneven AMR-shaped blocks; "
                        "adjoint: gradient of a 128^3 x 64-step rollout (cost ratio and finite differences); "
                        "blast: 512^3 RK3+PPM MHD blast; mesh: the 256^3 domain as a coupled mesh of equal blocks; "
                        "levels: restriction and prolongation of a 256^3 block")
    p.add_argument("--riemann", default="hlld", choices=["hlld", "hlle"], help="blast: Riemann solver")
    p.add_argument("--blast-n", type=int, default=512, help="blast: cells per side")
    p.add_argument("--blast-steps", type=int, default=200, help="blast: timed steps")
    p.add_argument("--floor", type=float, default=1e-10, help="blast: density and pressure floor")
    p.add_argument("--adj-n", type=int, default=128, help="adjoint: cells per side")
    p.add_argument("--adj-steps", type=int, default=64, help="adjoint: rollout steps")
    p.add_argument("--adj-dirs", type=int, default=16, help="adjoint: finite-difference directions")
    p.add_argument("--adj-eps", type=float, default=1e-3, help="adjoint: continuous CT weight eps")
    p.add_argument("--adj-no-fd", action="store_true", help="adjoint: skip the finite-difference check")
    p.add_argument("--adj-dir-kind", default="smooth", choices=["smooth", "white"],
                   help="adjoint: finite-difference directions: band-limited fields or white noise")
    p.add_argument("--levels-n", type=int, default=256, help="levels: cells per side of the block")
    p.add_argument("--mesh-blocks", type=int, default=8, help="mesh: blocks per direction of the 256^3 domain")
    p.add_argument("--no-tune", action="store_true", help="batch: keep the default tile instead of autotuning")
    p.add_argument("--coupled", action="store_true",
                   help="batch: cubes of 16^3, 24^3 and 32^3 in x3 slabs tiling one 192x192x384 periodic domain at "
                        "one cell width, exchanging their ghost entries (instead of the octree-shaped blocks that "
                        "are each their own periodic neighbour)")
    p.add_argument("--graph", action="store_true", help="replay each step from a hipGraph")
    p.add_argument("--charac", action="store_true",
                   help="turbulence: PLM on characteristic variables (runs the unfused pipeline)")
    p.add_argument("--scalars", type=int, default=0,
                   help="turbulence, batch: passive scalars carried along (a dye, then smooth fields)")
    p.add_argument("--copy-calibration", action="store_true",
                   help="only run a plain device copy of 1 GiB (for scaling PMC byte counters) and exit")
    return p.parse_args()


def stage_source_hash(names=("kernels_fused.hip", "mhd_math.hpp", "common.hpp")) -> str:
    """Hash of the kernels' code (the named sources) with comments and blank
    lines removed, so that a comment edit does not invalidate the stored PMC
    traffic."""
    import hashlib
    import re
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2005_06651_amd", "csrc")
    for name in names:
        with open(os.path.join(csrc, name), encoding="utf-8") as f:
            text = f.read()
        text = re.sub(r"/\*.*?\*/", "", re.sub(r"//[^\n]*", "", text), flags=re.S)
        text = "\n".join(line.rstrip() for line in text.splitlines() if line.strip())
        h.update(text.encode())
    return h.hexdigest()[:16]


def host_cpu() -> dict:
    """Model name and usable cores of the host that runs the oracle."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo", encoding="utf-8") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"model": model, "usable_cores": len(os.sched_getaffinity(0)), "logical_cpus": os.cpu_count()}


def _oracle_step_worker(n, seed, barrier, queue):
    """Worker process: build its own n^3 turbulence state, wait for the other
    workers, then time one oracle step (newdt + VL2+PLM+HLLD)."""
    from oracle import oracle as O
    from paper_2005_06651_amd import inputs
    block = inputs.turbulence(n=n, seed=seed)
    cfg = O.cfg_for(block, integrator="vl2", recon="plm", riemann="hlld", cfl=0.3)
    cons = O.prim2cons(cfg, block.prim, block.bface)
    bf = block.bface.copy()
    barrier.wait()
    t0 = time.perf_counter()
    dt, _ = O.newdt(cfg, cons, bf)
    O.step(cfg, cons, bf, dt)
    queue.put((n ** 3, time.perf_counter() - t0))


def cpu_aggregate(n: int = 96, max_procs: int = 16) -> dict:
    """P independent single-threaded oracle processes on P host cores, started
    together, each stepping its own n^3 turbulence state once: total
    zone-cycles / wall time of the slowest.  Called before anything touches
    the GPU (the workers are forked)."""
    import multiprocessing as mp
    from oracle import oracle as O
    O.build()
    procs = max(1, min(max_procs, len(os.sched_getaffinity(0))))
    ctx = mp.get_context("fork")
    barrier, queue = ctx.Barrier(procs), ctx.Queue()
    workers = [ctx.Process(target=_oracle_step_worker, args=(n, 1 + i, barrier, queue)) for i in range(procs)]
    for w in workers:
        w.start()
    res = [queue.get(timeout=600) for _ in workers]
    for w in workers:
        w.join()
    cells = sum(r[0] for r in res)
    wall = max(r[1] for r in res)
    return {"value": cells / wall, "unit": "zone-cycles/s", "processes": procs, "kind": "oracle, independent processes",
            "sample": f"{procs} processes started together, each one step (newdt + VL2+PLM+HLLD) of its own {n}^3 "
                      f"turbulence state; slowest {wall:.1f} s",
            "per_process_s": sorted(round(r[1], 2) for r in res)}


def cpu_baseline(block, steps: int):
    """The CPU oracle (single thread, as it stands) on a bounded sample of the
    same workload: `steps` VL2+PLM+HLLD steps of the same initial state."""
    from oracle import oracle as O
    cfg = O.cfg_for(block, integrator="vl2", recon="plm", riemann="hlld", cfl=0.3,
                    nscalars=block.prim.shape[0] - 5)
    cons = O.prim2cons(cfg, block.prim, block.bface)
    bf = block.bface.copy()
    zones = block.n[0] * block.n[1] * block.n[2]
    t0 = time.perf_counter()
    for _ in range(steps):
        dt, bad = O.newdt(cfg, cons, bf)
        O.step(cfg, cons, bf, dt)
    el = time.perf_counter() - t0
    return {
        "host": host_cpu(),
        "value": zones * steps / el,
        "unit": "zone-cycles/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{steps} step(s) (newdt + VL2+PLM+HLLD step) of the same {block.n[0]}^3 turbulence "
                  f"initial state on one host core, {el:.1f} s",
    }


def bench_batch(args):
    """1024 MeshBlocks of uneven sizes (40% 16^3, 40% 24^3, 20% 32^3, nghost 2)
    from a seeded 2:1-balanced octree, each with a smooth periodic state, one
    persistent launch per stage, VL2+PLM+HLLD, dt from the CFL reduction of
    every step's new state."""
    import torch

    from paper_2005_06651_amd import athmhd, inputs
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ns = args.scalars
    if args.coupled:
        if ns > 0:
            raise SystemExit("--coupled takes no passive scalars")
        dims, origins, domain = inputs.brick_layout(inputs.brick_slabs(seed=args.seed), 192)
        dom = inputs.smooth_random(n=domain, seed=args.seed, ng=2)
        pcs, fcs = inputs.split_boxes(dom.prim, dom.bface, 2, dims, origins)
        s = athmhd.BatchSolver(dims, [dom.dx] * len(dims), 2, dom.gamma, recon="plm", riemann="hlld",
                               integrator="vl2", cfl=0.3)
        s.couple(origins, domain)
        tb = torch.from_numpy(inputs.pack(fcs)).to(dev)
        tc = s.prim2cons(torch.from_numpy(inputs.pack(pcs)).to(dev), tb)
        s.fill_ghosts(tc, tb)
        del dom, pcs, fcs
        sizes = {n: sum(1 for d in dims if d[0] == n) for n in sorted({d[0] for d in dims})}
        zones = sum(d[0] * d[1] * d[2] for d in dims)
        workload = (f"{len(dims)} cube blocks ({', '.join(f'{c}x{n}^3' for n, c in sizes.items())}, nghost 2) in "
                    f"x3 slabs tiling one {domain[0]}x{domain[1]}x{domain[2]} periodic domain at one cell width, "
                    f"ghost entries exchanged between neighbours before every stage and after the last, one "
                    f"smooth seeded state, VL2+PLM+HLLD+CT, CFL 0.3")
    else:
        blocks = inputs.amr_batch(1024, seed=args.seed)
        if ns > 0:
            blocks = [inputs.with_scalars(b, ns, seed=args.seed + 100 + i) for i, b in enumerate(blocks)]
        s = athmhd.BatchSolver([b.n for b in blocks], [b.dx for b in blocks], 2, blocks[0].gamma, recon="plm",
                               riemann="hlld", integrator="vl2", cfl=0.3, nscalars=ns)
        tb = torch.from_numpy(inputs.pack([b.bface for b in blocks])).to(dev)
        tc = s.prim2cons(torch.from_numpy(inputs.pack([b.prim for b in blocks])).to(dev), tb)
        zones = sum(b.n[0] * b.n[1] * b.n[2] for b in blocks)
        workload = ("1024 AMR-shaped blocks (410x16^3, 410x24^3, 204x32^3, nghost 2) of a seeded 2:1-balanced "
                    "octree, smooth periodic states, VL2+PLM+HLLD+CT, CFL 0.3")
    stream = torch.cuda.Stream() if args.graph else torch.cuda.current_stream()
    tuned = None
    if not args.no_tune:
        tuned = s.tune(tc, tb, stream=stream)
    if args.graph:
        s.set_graph(True)
    with torch.cuda.stream(stream):
        # eager: chained steps (dt stays on the device); graph mode replays
        # athmhd_step with the dt of newdt
        dt_dev = torch.tensor([s.newdt(tc, tb, stream=stream)], dtype=torch.float64, device=dev)

        def one_step():
            if args.graph:
                s.step(tc, tb, s.newdt(tc, tb, stream=stream), stream=stream)
            else:
                s.step_chain(tc, tb, dt_dev, stream=stream)

        for _ in range(args.warmup):
            one_step()
        stream.synchronize()
        if not args.graph:
            s.profile_start()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            one_step()
        stream.synchronize()
        elapsed = time.perf_counter() - t0
        stage_ms, launches = (0.0, 0) if args.graph else s.profile_stop()
        s.newdt(tc, tb, stream=stream)  # raises if any step met a non-physical cell
    out = {
        "metric": "zone-cycles/s, FP64 3D MHD VL2+PLM+HLLD, 1 MI355X, batched uneven blocks"
                  + (", coupled" if args.coupled else "") + (f", with {ns} passive scalar(s)" if ns else ""),
        "value": zones * args.steps / elapsed, "unit": "zone-cycles/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": workload, "cells": zones, "coupled": bool(args.coupled), "tile": None if tuned is None else {"shape": athmhd.BATCH_TILES[tuned[0]],
                                                                        "split": tuned[1]},
                   "graph": bool(args.graph), "nscalars": ns},
        "stage_ms_per_launch": stage_ms / max(launches, 1) if launches else None,
    }
    s.close()
    print(json.dumps(out), flush=True)


def bench_adjoint(args):
    """Gradient of L = sum over active cells of (rho_N - rho_target)^2 dV after
    N steps (VL2+PLM+HLLD, continuous CT weight eps (default 1e-3), dt frozen at its
    value for the initial state) with respect to the initial velocity, through
    prim -> cons, the checkpointed rollout (sqrt(N) checkpoints) and the
    library's reverse mode.  Reports the forward time, the forward + backward
    time and their ratio, and checks the gradient against central differences
    of the loss along seeded unit directions (h swept 1e-2 .. 1e-6)."""
    import numpy as np
    import torch

    from paper_2005_06651_amd import athmhd, inputs
    from paper_2005_06651_amd.rollout import Prim2Cons, Rollout
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n, nsteps = args.adj_n, args.adj_steps
    ncheck = max(1, int(math.isqrt(nsteps)))
    blk = inputs.turbulence(n=n, seed=args.seed, mach=0.3)
    s = athmhd.Solver(blk.n, blk.ng, blk.dx, blk.gamma, recon="plm", riemann="hlld", integrator="vl2", cfl=0.3,
                      ct_eps=args.adj_eps)
    g = blk.ng
    prim0 = torch.from_numpy(blk.prim).to(dev)
    bf0 = torch.from_numpy(blk.bface).to(dev)
    dt = s.newdt(s.prim2cons(prim0, bf0), bf0)
    rng = np.random.default_rng(args.seed + 1000)
    # smooth target density 1 + 0.05 f with f from the same band-limited generator
    tgt = inputs.smooth_random(n=(n, n, n), seed=args.seed + 2000, ng=g, kmax=4.0, rho_range=(0.95, 1.05))
    target = torch.from_numpy(np.ascontiguousarray(tgt.prim[0, g:g + n, g:g + n, g:g + n])).to(dev)
    dV = blk.dx[0] * blk.dx[1] * blk.dx[2]

    def loss_of(prim):
        c0 = Prim2Cons.apply(prim, bf0, s)
        cN, _ = Rollout.apply(c0, bf0, s, dt, nsteps, ncheck)
        return ((cN[0, g:g + n, g:g + n, g:g + n] - target) ** 2).sum() * dV

    # warm-up (also allocates the reverse-mode scratch)
    p = prim0.clone().requires_grad_(True)
    loss_of(p).backward()
    torch.cuda.synchronize()
    # forward only
    t0 = time.perf_counter()
    with torch.no_grad():
        lval = loss_of(prim0).item()
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    # forward + backward
    p = prim0.clone().requires_grad_(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    loss = loss_of(p)
    loss.backward()
    torch.cuda.synchronize()
    t_all = time.perf_counter() - t0
    grad_v = p.grad[1:4, g:g + n, g:g + n, g:g + n].double().cpu().numpy()
    errs = []
    plateau = []
    hs = (1e-2, 1e-3, 1e-4, 1e-5, 1e-6, 1e-7)
    ads = []
    for q in range(0 if args.adj_no_fd else args.adj_dirs):
        if args.adj_dir_kind == "smooth":
            # band-limited random velocity field (|k| <= 4), unit norm
            d = inputs.smooth_random(n=(n, n, n), seed=args.seed + 3000 + q, ng=g, kmax=4.0).prim[
                1:4, g:g + n, g:g + n, g:g + n].copy()
        else:
            d = rng.standard_normal((3, n, n, n))
        d /= np.linalg.norm(d)
        ad = float(np.sum(grad_v * d))
        ads.append(ad)
        row = []
        for h in hs:
            dp = torch.zeros_like(prim0)
            dp[1:4, g:g + n, g:g + n, g:g + n] = torch.from_numpy(h * d).to(dev)
            with torch.no_grad():
                fd = (loss_of(prim0 + dp).item() - loss_of(prim0 - dp).item()) / (2 * h)
            row.append(abs(fd - ad) / max(abs(ad), 1e-300))
        plateau.append(row)
        errs.append(min(row))
    out = {
        "metric": f"adjoint cost: (forward + backward) / forward time of a checkpointed {nsteps}-step rollout "
                  "gradient, FP64 VL2+PLM+HLLD+CT, 1 MI355X",
        "value": t_all / t_fwd, "unit": "ratio", "n_gpus": 1, "steps": nsteps, "warmup": 1,
        "ms_per_step": t_fwd / nsteps * 1e3, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{n}^3 periodic MHD turbulence at rms Mach 0.3 (B = 0.5 x + curl A, rms 0.1), "
                               f"{nsteps} steps of frozen dt, CT weight eps {args.adj_eps:g}, {ncheck} checkpoints; loss = "
                               "sum (rho_N - rho_target)^2 dV, gradient w.r.t. the initial velocity",
                   "cells": n ** 3, "dt": dt, "checkpoints": ncheck},
        "forward_s": t_fwd, "forward_backward_s": t_all, "loss": lval,
        "fd_check": None if not errs else {
            "directions": len(errs), "h": list(hs), "max_rel_err": max(errs),
            "median_rel_err": float(np.median(errs)),
            "rel_err_by_h_max_over_dirs": [max(r[k] for r in plateau) for k in range(len(hs))],
            "direction_kind": args.adj_dir_kind, "abs_directional_derivative_median": float(np.median(np.abs(ads)))},
    }
    s.close()
    print(json.dumps(out), flush=True)


def bench_mesh(args):
    """The 256^3 decaying turbulence as a coupled mesh of m^3 equal blocks
    (default 8^3 blocks of 32^3): ghost cells and faces exchanged between the
    blocks on the device before every stage, VL2+PLM+HLLD, one chained step
    (step, then the CFL reduction for the next dt, on the device) per timed
    step."""
    import torch

    from paper_2005_06651_amd import athmhd, inputs
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    m = args.mesh_blocks
    blk = inputs.turbulence(n=args.n, seed=args.seed)
    if args.n % m:
        sys.exit(f"bench.py: {args.n} cells per side do not split into {m} blocks")
    nb = args.n // m
    single = athmhd.Solver(blk.n, blk.ng, blk.dx, blk.gamma)
    tb = torch.from_numpy(blk.bface).to(dev)
    cons = single.prim2cons(torch.from_numpy(blk.prim).to(dev), tb).cpu().numpy()
    single.close()
    del tb
    mc, mf = inputs.split_mesh(cons, blk.bface, blk.ng, (nb, nb, nb), (m, m, m))
    del cons
    s = athmhd.MeshSolver((nb, nb, nb), (m, m, m), blk.ng, blk.dx, blk.gamma, recon="plm", riemann="hlld",
                          integrator="vl2", cfl=0.3)
    tc, tf = torch.from_numpy(mc).to(dev), torch.from_numpy(mf).to(dev)
    del mc, mf
    zones = args.n ** 3
    dt_dev = torch.tensor([s.newdt(tc, tf)], dtype=torch.float64, device=dev)
    for _ in range(args.warmup):
        s.step_chain(tc, tf, dt_dev)
    torch.cuda.synchronize()
    s.profile_start()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        s.step_chain(tc, tf, dt_dev)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    stage_ms, launches = s.profile_stop()
    s.newdt(tc, tf)  # raises if any step met a non-physical cell
    out = {
        "metric": "zone-cycles/s, FP64 3D MHD VL2+PLM+HLLD, 1 MI355X, coupled mesh of equal blocks",
        "value": zones * args.steps / elapsed, "unit": "zone-cycles/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"decaying MHD turbulence {args.n}^3 periodic as {m}^3 blocks of {nb}^3 (nghost 2), "
                               "ghost exchange between blocks before every stage, VL2+PLM+HLLD+CT, CFL 0.3",
                   "cells": zones, "blocks": m ** 3, "seed": args.seed},
        "stage_ms_per_launch": stage_ms / max(launches, 1),
    }
    print(json.dumps(out))


def bench_levels(args):
    """Level operators of block refinement on one 256^3 block (the largest
    single block; nghost 2, 5 conserved arrays): prolongation of each of the 8
    octants of a coarse block onto a fine block, then restriction of the fine
    block back onto each octant, and prolongation in primitive variables of a
    physical copy of the coarse block, timed with HIP events on the launch
    stream.
    Algorithmic bytes per coarse cell of an octant (nv = 5 cell arrays, 3 face
    components): prolongation reads nv cells and 3 faces and writes 8 nv fine
    cells and 24 fine faces (12 on the coarse faces it owns, 12 inside), i.e.
    (9 nv + 27) x 8 = 576 B; restriction reads 8 nv fine cells and 12 fine
    faces and writes nv cells and 3 faces, (9 nv + 15) x 8 = 480 B."""
    import torch

    from paper_2005_06651_amd import athmhd
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n, ng, nv = args.levels_n, 2, 5
    N = n + 2 * ng
    gen = torch.Generator(device=dev)
    gen.manual_seed(args.seed)
    cc = torch.randn((nv, N, N, N), dtype=torch.float64, device=dev, generator=gen)
    cb = torch.randn((3, N + 1, N + 1, N + 1), dtype=torch.float64, device=dev, generator=gen)
    fc, fb = torch.zeros_like(cc), torch.zeros_like(cb)
    s = athmhd.Solver((n, n, n), ng, (1.0 / n,) * 3, 5.0 / 3.0)
    octs = [(i & 1, (i >> 1) & 1, i >> 2) for i in range(8)]
    stream = torch.cuda.current_stream()

    def run(op, src, dst):
        for o in octs:
            op(*src, *dst, o, stream=stream)

    def prolong_prim(*a, **k):
        s.prolong(*a, primitive=True, **k)

    # primitive prolongation needs a physical coarse state: rho and P positive
    cp = cc.clone()
    cp[0] = 1.0 + 0.1 * cp[0].abs()
    cp[4] = 50.0 + cp[4].abs()
    for _ in range(args.warmup):
        run(s.prolong, (cc, cb), (fc, fb))
        run(s.restrict, (fc, fb), (cc, cb))
        run(prolong_prim, (cp, cb), (fc, fb))
    torch.cuda.synchronize()
    ms = {}
    t0 = time.perf_counter()
    for name, op, src, dst in (("prolong", s.prolong, (cc, cb), (fc, fb)), ("restrict", s.restrict, (fc, fb), (cc, cb)),
                               ("prolong_primitive", prolong_prim, (cp, cb), (fc, fb))):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            run(op, src, dst)
        e1.record(stream)
        torch.cuda.synchronize()
        ms[name] = e0.elapsed_time(e1) / (args.steps * 8)   # per launch (one octant)
    elapsed = time.perf_counter() - t0
    coarse = (n // 2) ** 3                                   # coarse cells per octant
    bytes_p, bytes_r = coarse * (9 * nv + 27) * 8, coarse * (9 * nv + 15) * 8
    gbs_p, gbs_r = bytes_p / (ms["prolong"] * 1e-3) / 1e9, bytes_r / (ms["restrict"] * 1e-3) / 1e9
    measured = LEVELS_TRAFFIC.get("source_hash") == stage_source_hash(LEVELS_SOURCES) and n == 256
    traffic = {k: (LEVELS_TRAFFIC[k]["bytes_per_launch"] if measured else None)
               for k in ("prolong", "restrict", "prolong_primitive")}
    out = {
        "metric": "fine cells prolonged per second, FP64 MHD level operators (Sec. 2.1.5), 1 MI355X",
        "value": 8 * coarse / (ms["prolong"] * 1e-3), "unit": "cells/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"prolongation of the 8 octants of a {n}^3 block (nghost 2, 5 cell arrays, "
                               "face field) onto a fine block, then restriction back, seeded normal values",
                   "octant_coarse_cells": coarse, "seed": args.seed},
        "roofline": {"bound": "hbm", "achieved": gbs_p, "peak": 8000.0, "unit": "GB/s", "frac": gbs_p / 8000.0,
                     "traffic": traffic["prolong"], "kernel": "k_prolong", "ms_per_launch": ms["prolong"],
                     "alg_bytes_per_launch": bytes_p},
        "restrict": {"ms_per_launch": ms["restrict"], "GB/s": gbs_r, "frac": gbs_r / 8000.0,
                     "traffic": traffic["restrict"], "alg_bytes_per_launch": bytes_r,
                     "cells_per_s": coarse / (ms["restrict"] * 1e-3)},
        "prolong_primitive": {"ms_per_launch": ms["prolong_primitive"],
                              "GB/s": bytes_p / (ms["prolong_primitive"] * 1e-3) / 1e9,
                              "frac": bytes_p / (ms["prolong_primitive"] * 1e-3) / 1e9 / 8000.0,
                              "traffic": traffic["prolong_primitive"], "alg_bytes_per_launch": bytes_p},
    }
    print(json.dumps(out))


def bench_blast(args):
    """MHD blast on the 512^3 periodic unit cube (nghost 3, RK3 + PPM + HLLD or
    HLLE + CT, rho = 1, p = 0.1, p = 10 inside r < 0.1 around a seeded centre,
    B = (1/sqrt2, 1/sqrt2, 0), CFL 0.3): one chained RK3 step (step, then the
    CFL reduction for the next dt, on the device) per timed step.
    Density and pressure floors (1e-10 by default) limit the primitives and,
    after each stage, raise the density and total energy of cells below them;
    their activations are counted and reported."""
    import torch

    from paper_2005_06651_amd import athmhd, inputs
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n = args.blast_n
    blk = inputs.blast(n=n, seed=args.seed)
    s = athmhd.Solver(blk.n, blk.ng, blk.dx, blk.gamma, recon="ppm", riemann=args.riemann, integrator="rk3",
                      cfl=0.3)
    # without floors this blast reaches P <= 0 within a few steps (the CPU
    # oracle does too); every floor activation is counted
    s.set_floors(args.floor, args.floor)
    tb = torch.from_numpy(blk.bface).to(dev)
    tc = s.prim2cons(torch.from_numpy(blk.prim).to(dev), tb)
    del blk.prim
    # chained steps: dt read on the device, the CFL reduction of the new state
    # writes the next one there; the simulated time accumulates on the device
    dt_dev = torch.tensor([s.newdt(tc, tb)], dtype=torch.float64, device=dev)
    t_dev = torch.zeros(1, dtype=torch.float64, device=dev)

    def one_step():
        t_dev.add_(dt_dev)
        s.step_chain(tc, tb, dt_dev)

    s.floor_count()
    for _ in range(args.warmup):
        one_step()
    torch.cuda.synchronize()
    s.profile_start()
    t0 = time.perf_counter()
    for _ in range(args.blast_steps):
        one_step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    stage_ms, launches = s.profile_stop()
    nonphys = 0
    try:
        s.newdt(tc, tb)  # reports any non-physical cell met since the warmup
    except athmhd.NonPhysicalState:
        nonphys = 1
    t_sim = t_dev.item()
    floored = s.floor_count()
    s.fill_ghosts(tc, tb)
    torch.cuda.synchronize()
    g = blk.ng
    b1 = tb[0, g:g + n, g:g + n, g:g + n + 1]
    b2 = tb[1, g:g + n, g:g + n + 1, g:g + n]
    b3 = tb[2, g:g + n + 1, g:g + n, g:g + n]
    div = (b1[:, :, 1:] - b1[:, :, :-1]) + (b2[:, 1:, :] - b2[:, :-1, :]) + (b3[1:] - b3[:-1])
    bmax = max(b1.abs().max().item(), b2.abs().max().item(), b3.abs().max().item())
    zones = n ** 3
    out = {
        "metric": f"zone-cycles/s, FP64 3D MHD RK3+PPM+{args.riemann.upper()}, 1 MI355X",
        "value": zones * args.blast_steps / el, "unit": "zone-cycles/s", "n_gpus": 1, "steps": args.blast_steps,
        "warmup": args.warmup, "ms_per_step": el / args.blast_steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"MHD blast {n}^3 periodic unit cube, nghost 3, RK3+PPM+{args.riemann.upper()}+CT, "
                               "rho 1, p 0.1 / 10 inside r < 0.1 (seeded centre), B = (1,1,0)/sqrt2, CFL 0.3, "
                               "dt from the CFL reduction of every step's new state, kept on the device",
                   "cells": zones, "seed": args.seed, "riemann": args.riemann},
        "stage_ms_per_launch": stage_ms / max(launches, 1),
        "t_simulated": t_sim, "nonphysical_reports": nonphys,
        "floors": {"rho": args.floor, "p": args.floor, "activations": floored},
        "divb_after": div.abs().max().item() / bmax,
    }
    if not args.no_cpu_baseline:
        from oracle import oracle as O
        small = inputs.blast(n=64, seed=args.seed)
        cfg = O.cfg_for(small, integrator="rk3", recon="ppm", riemann=args.riemann, cfl=0.3, dfloor=args.floor,
                        pfloor=args.floor)
        cons = O.prim2cons(cfg, small.prim, small.bface)
        bf = small.bface.copy()
        t0 = time.perf_counter()
        dt, _ = O.newdt(cfg, cons, bf)
        O.step(cfg, cons, bf, dt)
        el = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": 64 ** 3 / el, "unit": "zone-cycles/s", "cores": 1, "kind": "oracle",
                               "sample": f"1 step (newdt + RK3+PPM step) of a 64^3 blast on one host core, {el:.1f} s"}
    s.close()
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: the MHD step runs on one GPU (sharding over several GPUs is designed, not built); "
              "--gpus must be 1", file=sys.stderr)
        sys.exit(2)
    # the aggregate CPU baseline forks worker processes: before the GPU is touched
    agg = None
    if args.workload == "turbulence" and not args.no_cpu_baseline and not args.copy_calibration:
        agg = cpu_aggregate()
    import numpy as np
    import torch

    from paper_2005_06651_amd import athmhd, inputs

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.workload == "batch":
        bench_batch(args)
        return
    if args.workload == "adjoint":
        bench_adjoint(args)
        return
    if args.workload == "blast":
        bench_blast(args)
        return
    if args.workload == "mesh":
        bench_mesh(args)
        return
    if args.workload == "levels":
        bench_levels(args)
        return
    if args.copy_calibration:
        a = torch.ones(1 << 27, dtype=torch.float64, device=dev)  # 1 GiB
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": a.numel() * 8, "launches": 3}))
        return
    n = args.n
    ns = args.scalars
    block = inputs.turbulence(n=n, seed=args.seed)
    if ns > 0:
        block = inputs.with_scalars(block, ns, seed=args.seed + 100)
    solver = athmhd.Solver(block.n, block.ng, block.dx, block.gamma, recon="plm", riemann="hlld",
                           integrator="vl2", cfl=0.3, kernel_path=args.kernel_path, nscalars=ns,
                           charac=args.charac)
    tb = torch.from_numpy(block.bface).to(dev)
    tc = solver.prim2cons(torch.from_numpy(block.prim).to(dev), tb)
    torch.cuda.synchronize()

    # each step: the VL2 step with dt read on the device, then the CFL
    # reduction of the new state writing the next step's dt there
    # (athmhd_step_chain); no host round trip between steps
    dt_dev = torch.tensor([solver.newdt(tc, tb)], dtype=torch.float64, device=dev)
    for _ in range(args.warmup):
        solver.step_chain(tc, tb, dt_dev)
    torch.cuda.synchronize()

    solver.profile_start()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        solver.step_chain(tc, tb, dt_dev)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    stage_ms, launches = solver.profile_stop()
    solver.newdt(tc, tb)  # raises if any step met a non-physical cell

    zones = n ** 3
    value = zones * args.steps / elapsed
    # dominant kernel = the fused stage kernel (two launches per step).  It is
    # bound by FP64 VALU issue, not by HBM: report the ALU roofline with the
    # algorithmic flops, and the HBM view with the algorithmic bytes (VL2 stage
    # 0 reads U^n and writes U^(n+1/2): 128 B per cell; stage 1 reads U^(n+1/2)
    # and U^n and writes U^(n+1): 192 B per cell).
    per_launch_s = stage_ms / 1e3 / max(launches, 1)
    alg_flops = ALG_FLOPS_PER_ZONE_CYCLE / 2 * zones
    alg_bytes = (128 + 192) / 2 * zones
    achieved_tf = alg_flops / per_launch_s / 1e12
    achieved_gbs = alg_bytes / per_launch_s / 1e9
    traffic = None
    issue = None
    if STAGE_TRAFFIC and STAGE_TRAFFIC.get("source_hash") == stage_source_hash() and args.kernel_path == "fused" \
            and n == 256 and ns == 0 and not args.charac:
        traffic = STAGE_TRAFFIC["bytes_per_launch"]
        if STAGE_ISSUE.get("source_hash") == STAGE_TRAFFIC["source_hash"]:
            issue = STAGE_ISSUE
    # which roof binds: the larger of the measured FP64 VALU issue fraction
    # and the measured HBM traffic fraction (counters of this kernel source);
    # without current counters, the larger algorithmic fraction
    alu_frac = achieved_tf / FP64_VECTOR_TFLOPS
    hbm_frac = achieved_gbs / HBM_PEAK_GBS
    if issue:
        traffic_frac = traffic / (issue["profiled_ms_per_launch"] * 1e-3) / 1e9 / HBM_PEAK_GBS
        bound = "alu" if issue["valu_issue_frac"] >= traffic_frac else "hbm"
        basis = {"valu_issue_frac": issue["valu_issue_frac"], "hbm_traffic_frac": traffic_frac,
                 "source": "rocprofv3 SQ_INSTS_VALU, FETCH_SIZE, WRITE_SIZE of this kernel source"}
    else:
        bound = "alu" if alu_frac >= hbm_frac else "hbm"
        basis = {"source": "algorithmic fractions (no counters for this kernel source)"}
    # sanity of the final state
    solver.fill_ghosts(tc, tb)
    torch.cuda.synchronize()
    g = block.ng
    b1 = tb[0, g:g + n, g:g + n, g:g + n + 1]
    b2 = tb[1, g:g + n, g:g + n + 1, g:g + n]
    b3 = tb[2, g:g + n + 1, g:g + n, g:g + n]
    div = (b1[:, :, 1:] - b1[:, :, :-1]) + (b2[:, 1:, :] - b2[:, :-1, :]) + (b3[1:] - b3[:-1])
    bmax = max(b1.abs().max().item(), b2.abs().max().item(), b3.abs().max().item())
    divb = div.abs().max().item() / bmax

    out = {
        "metric": "zone-cycles/s, FP64 3D MHD VL2+PLM+HLLD, 1 MI355X"
                  + (f", with {ns} passive scalar(s)" if ns else "") + (", characteristic PLM" if args.charac else ""),
        "value": value,
        "unit": "zone-cycles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": f"decaying MHD turbulence {n}^3 periodic, VL2+PLM+HLLD+CT, gamma 5/3, rms Mach 1, "
                        f"B = 0.5 x + curl A (rms 0.1), CFL 0.3, dt from the CFL reduction of every step's "
                        f"new state, kept on the device",
            "cells": zones, "nghost": g, "integrator": "vl2", "recon": "plm", "riemann": "hlld",
            "seed": args.seed, "kernel_path": "unfused" if args.charac else args.kernel_path, "nscalars": ns,
            "characteristic": bool(args.charac),
        },
        "roofline": {
            "bound": bound,
            "kernel": "k_stage_fused (reconstruct + HLLD + CT + update of one stage), per launch",
            "achieved": achieved_tf if bound == "alu" else achieved_gbs,
            "peak": FP64_VECTOR_TFLOPS if bound == "alu" else HBM_PEAK_GBS,
            "unit": "TFLOP/s" if bound == "alu" else "GB/s",
            "frac": alu_frac if bound == "alu" else hbm_frac,
            "traffic": traffic,
            "alu_frac": alu_frac,
            "hbm_frac": hbm_frac,
            "hbm_frac_target": HBM_FRAC_TARGET,
            "bound_basis": basis,
            "alg_flops_per_launch": alg_flops,
            "stage_ms_per_launch": per_launch_s * 1e3,
            "launches": launches,
            "hbm_view": {"achieved": achieved_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": achieved_gbs / HBM_PEAK_GBS, "alg_bytes_per_launch": alg_bytes},
        },
        "divb_after": divb,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(block, args.cpu_steps)
        if agg:
            out["cpu_baseline"]["aggregate"] = agg
    solver.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
