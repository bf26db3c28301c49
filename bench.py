#!/usr/bin/env python3
"""Throughput of the FP64 ideal-MHD step (VL2 + PLM + HLLD + upwind CT) on one
MI355X, in zone-cycles per second.

Workload: decaying MHD turbulence on a 256^3 periodic block (nghost 2,
gamma 5/3, rho = 1, p = 1, solenoidal velocity on 1 <= |k| <= 4 at rms Mach 1,
B = 0.5 x + curl A with rms(curl A) = 0.1), CFL 0.3.  One timed step is the
whole hot path: the CFL time step (athmhd_newdt) followed by one full VL2 step
(ghost fill, two fused stages of cons->prim, reconstruction, HLLD fluxes, CT
corner EMFs and the conservative + face-field update).  Inputs are resident
in HBM before the timed region.

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
FP64_VECTOR_TFLOPS = 78.6    # MI355X FP64 vector peak (FMA = 2 flops)
STATE_BYTES_PER_CELL = 64    # 5 conserved + 3 face-field doubles


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
    return p.parse_args()


def cpu_baseline(block, steps: int):
    """The CPU oracle (single thread, as it stands) on a bounded sample of the
    same workload: `steps` VL2+PLM+HLLD steps of the same initial state."""
    from oracle import oracle as O
    cfg = O.cfg_for(block, integrator="vl2", recon="plm", riemann="hlld", cfl=0.3)
    cons = O.prim2cons(cfg, block.prim, block.bface)
    bf = block.bface.copy()
    zones = block.n[0] * block.n[1] * block.n[2]
    t0 = time.perf_counter()
    for _ in range(steps):
        dt, bad = O.newdt(cfg, cons, bf)
        O.step(cfg, cons, bf, dt)
    el = time.perf_counter() - t0
    return {
        "value": zones * steps / el,
        "unit": "zone-cycles/s",
        "cores": 1,
        "kind": "oracle",
        "sample": f"{steps} step(s) (newdt + VL2+PLM+HLLD step) of the same {block.n[0]}^3 turbulence "
                  f"initial state on one host core, {el:.1f} s",
    }


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU only; --gpus must be 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch

    from paper_2005_06651_amd import athmhd, inputs

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n = args.n
    block = inputs.turbulence(n=n, seed=args.seed)
    solver = athmhd.Solver(block.n, block.ng, block.dx, block.gamma, recon="plm", riemann="hlld",
                           integrator="vl2", cfl=0.3, kernel_path=args.kernel_path)
    tb = torch.from_numpy(block.bface).to(dev)
    tc = solver.prim2cons(torch.from_numpy(block.prim).to(dev), tb)
    torch.cuda.synchronize()

    for _ in range(args.warmup):
        dt = solver.newdt(tc, tb)
        solver.step(tc, tb, dt)
    torch.cuda.synchronize()

    solver.profile_start()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        dt = solver.newdt(tc, tb)
        solver.step(tc, tb, dt)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    stage_ms, launches = solver.profile_stop()

    zones = n ** 3
    value = zones * args.steps / elapsed
    # stage kernel roofline: VL2 stage 0 reads U^n and writes U^(n+1/2) (128 B
    # per active cell), stage 1 reads U^(n+1/2) and U^n and writes U^(n+1)
    # (192 B); algorithmic bytes per launch averaged over the two stages
    alg_bytes = (128 + 192) / 2 * zones
    per_launch_s = stage_ms / 1e3 / max(launches, 1)
    achieved = alg_bytes / per_launch_s / 1e9
    # sanity of the final state
    g = block.ng
    b1 = tb[0, g:g + n, g:g + n, g:g + n + 1]
    b2 = tb[1, g:g + n, g:g + n + 1, g:g + n]
    b3 = tb[2, g:g + n + 1, g:g + n, g:g + n]
    div = (b1[:, :, 1:] - b1[:, :, :-1]) + (b2[:, 1:, :] - b2[:, :-1, :]) + (b3[1:] - b3[:-1])
    bmax = max(b1.abs().max().item(), b2.abs().max().item(), b3.abs().max().item())
    divb = div.abs().max().item() / bmax

    out = {
        "metric": "zone-cycles/s, FP64 3D MHD VL2+PLM+HLLD, 1 MI355X",
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
                        f"B = 0.5 x + curl A (rms 0.1), CFL 0.3, dt from newdt every step",
            "cells": zones, "nghost": g, "integrator": "vl2", "recon": "plm", "riemann": "hlld",
            "seed": args.seed, "kernel_path": args.kernel_path,
        },
        "roofline": {
            "bound": "hbm",
            "kernel": "stage (reconstruct + HLLD + CT + update), per launch",
            "achieved": achieved,
            "peak": HBM_PEAK_GBS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS,
            "traffic": None,
            "stage_ms_per_launch": per_launch_s * 1e3,
            "launches": launches,
        },
        "divb_after": divb,
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(block, args.cpu_steps)
    solver.close()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
