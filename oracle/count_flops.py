"""Algorithmic floating-point work of one VL2+PLM+HLLD step of the 256^3
turbulence workload, counted by running the oracle with an operation-counting
scalar type (adds/subtracts, multiplies, divides and square roots; no FMA).

The oracle reconstructs every face from its line of cells, so each limited
slope is evaluated twice (once for each face of the cell).  The per-cell form
evaluates it once: the PLM share is taken from the difference to a donor-cell
run and scaled by 10/16 (per variable and direction: one slope of 6 flops plus
two edge values of 2 flops each, instead of two slopes and two edge values).

Usage: python -m oracle.count_flops [n]
"""
import sys

from oracle import oracle as O
from paper_2005_06651_amd import inputs


def main(n: int = 256) -> None:
    b = inputs.turbulence(n=n, seed=1)
    zones = n ** 3
    out = {}
    for recon in ("plm", "dc"):
        cfg = O.cfg_for(b, integrator="vl2", recon=recon, riemann="hlld", cfl=0.3)
        cons = O.prim2cons(cfg, b.prim, b.bface)
        dt, _ = O.newdt(cfg, cons, b.bface)
        ops = O.count_ops(cfg, cons, b.bface, dt)
        out[recon] = sum(ops)
        print(f"VL2+{recon.upper()}+HLLD n={n}: add {ops[0]} mul {ops[1]} div {ops[2]} sqrt {ops[3]}; "
              f"{sum(ops) / zones:.1f} flops per zone-cycle")
    recon_share = out["plm"] - out["dc"]
    alg = out["plm"] - recon_share + recon_share * 10.0 / 16.0
    print(f"per-cell slope form: {alg / zones:.1f} flops per zone-cycle "
          f"(PLM reconstruction share {recon_share / zones:.1f} in the per-face form)")


if __name__ == "__main__":
    main(int(sys.argv[1]) if len(sys.argv) > 1 else 256)
