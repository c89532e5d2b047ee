"""Near-pair evaluation: direct series at the target nodes (near_method 0, Section 4.1)
against pole rotation with delayed evaluation (near_method 1, Section 4.2), timed on the
GPU for increasing p on one sphere configuration, with the relative difference of the
two near fields (the band-limited projection error of the rotated method).

The near/far threshold d* is measured per p for the library's default precision (Eq. 4.5),
the same for both methods; --near-gap fixes it instead.

Usage: python -m paper_1707_06551_amd.run_near [--workload spheres1024_p16] [--p 4 8 12 16 20] [--near-gap G]
"""
import argparse
import json

import numpy as np

from . import bie
from .inputs import lattice_centres, make_workload


def main():
    import torch
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="spheres1024_p16", help="a named workload, or lattice_q4 (17^3 lattice)")
    ap.add_argument("--p", type=int, nargs="+", default=[4, 8, 12, 16, 20])
    ap.add_argument("--op", choices=["s", "d"], default="d")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--near-gap", type=float, default=0.0, help="d* (<= 0: measured for the default precision)")
    args = ap.parse_args()
    c = lattice_centres(16, 4) if args.workload == "lattice_q4" else make_workload(args.workload)["centres"]
    op = bie.OP_D if args.op == "d" else bie.OP_S
    for p in args.p:
        res = {}
        fields = {}
        for method in (0, 1):
            sph = bie.Spheres(c, p, near_gap=args.near_gap if args.near_gap > 0 else None, near_method=method)
            x = torch.randn(3 * sph.N, dtype=torch.float64, device="cuda",
                            generator=torch.Generator("cuda").manual_seed(3))
            u = torch.empty_like(x)
            stage = op | bie.STAGE_NEAR
            sph.apply(stage, x, u)
            torch.cuda.synchronize()
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(args.reps):
                sph.apply(stage, x, u)
            e1.record()
            e1.synchronize()
            res[method] = e0.elapsed_time(e1) / args.reps
            fields[method] = u.clone()
            near, dstar = sph.n_near, sph.near_gap
            sph.close()
        diff = float(torch.linalg.norm(fields[1] - fields[0]) / torch.linalg.norm(fields[0]))
        print(json.dumps(dict(workload=args.workload, n_spheres=len(c), p=p, op=args.op, near_gap=dstar, directed_near_pairs=near,
                              direct_ms=res[0], rotation_ms=res[1], rel_difference=diff)), flush=True)


if __name__ == "__main__":
    main()
