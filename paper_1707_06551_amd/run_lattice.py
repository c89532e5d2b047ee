"""Operator-apply scaling on the cubic lattices of the paper's scaling experiment
(Section 6, Figs. 8-9): the time of one application of a layer operator (self term,
near series and far field together) as the lattice grows from 2^3 to 17^3 unit spheres,
loosely (q = 1) and densely (q = 4) packed, at p = 4 and 8.

The paper times the double layer D and the single-layer traction K (--op k), whose
near evaluation carries the extra terms of the target normal.  The paper evaluates its
far field with an FMM and reports slopes approaching 1 in
log(time) against log(n_b); the far field here is an all-pairs sum, so the slope tends
to 2 once the far field dominates.  One JSON line per case, then the slopes.

--poly runs the polydisperse lattices (face and cube-centre spheres of radii
2 - sqrt(2) and sqrt(2) - 1 added, Fig. 8 (c), (d); q <= 3, the printed radii overlap
for q = 4).

Usage: python -m paper_1707_06551_amd.run_lattice [--op d] [--precision mixed fp64] [--units 1 2 4 8 16] [--poly]
"""
import argparse
import json
import math

import numpy as np

from . import bie
from .inputs import lattice_centres, lattice_poly

OPS = {"s": bie.OP_S, "d": bie.OP_D, "sd": bie.OP_SD_BIE, "dn": bie.OP_DN_BIE, "k": bie.OP_K}


def time_apply(sph, op, precision, reps):
    import torch
    x = torch.randn(3 * sph.N, dtype=torch.float64, device="cuda")
    u = torch.empty_like(x)
    sph.apply(op, x, u, precision=precision)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        sph.apply(op, x, u, precision=precision)
    e1.record()
    e1.synchronize()
    return e0.elapsed_time(e1) / reps


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--op", choices=sorted(OPS), default="d")
    ap.add_argument("--q", type=int, nargs="+", default=[1, 4])
    ap.add_argument("--p", type=int, nargs="+", default=[4, 8])
    ap.add_argument("--units", type=int, nargs="+", default=[1, 2, 4, 8, 16])
    ap.add_argument("--precision", nargs="+", choices=["mixed", "fp64"], default=["mixed", "fp64"])
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--poly", action="store_true", help="polydisperse lattices (spheres of three radii)")
    args = ap.parse_args()
    op = OPS[args.op]
    for q in args.q:
        for p in args.p:
            for prec in args.precision:
                precision = bie.MIXED if prec == "mixed" else bie.FP64
                rows = []
                for u in args.units:
                    if args.poly:
                        c, rad = lattice_poly(u, q)
                        sph = bie.Spheres(c, p, near_gap=1.0, radii=rad)
                    else:
                        c = lattice_centres(u, q)
                        sph = bie.Spheres(c, p, near_gap=1.0)
                    near = sph.near_pairs().shape[1]
                    pairs = (sph.nb * (sph.nb - 1) - near) * sph.P * sph.P
                    ms = time_apply(sph, op, precision, args.reps if sph.nb > 100 else 20)
                    row = dict(op=args.op, poly=args.poly, q=q, p=p, precision=prec, units=u, n_spheres=sph.nb,
                               nodes=sph.N,
                               near_pairs=near, apply_ms=ms, far_pairs=pairs, far_pairs_per_s=pairs / (ms * 1e-3))
                    rows.append(row)
                    print(json.dumps(row), flush=True)
                    sph.close()
                slopes = [math.log(b["apply_ms"] / a["apply_ms"]) / math.log(b["n_spheres"] / a["n_spheres"])
                          for a, b in zip(rows, rows[1:])]
                print(json.dumps(dict(op=args.op, poly=args.poly, q=q, p=p, precision=prec,
                                      n_spheres=[r["n_spheres"] for r in rows],
                                      slopes=[round(s, 3) for s in slopes])), flush=True)


if __name__ == "__main__":
    main()
