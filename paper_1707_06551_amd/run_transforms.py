"""Timing of the batched transforms with the Legendre stages as FMA loops from LDS or
on the matrix cores (bie_opts.legendre_mfma): the self stage of S + D (forward
transform, Theorem 2's eigenvalues, inverse transform, Section 4.1) and the forward
transform alone, per call, float32 and float64, events on the library's stream.

Usage: python -m paper_1707_06551_amd.run_transforms [--workloads spheres512_p12 ...] [--reps 50]
"""
import argparse
import json

import numpy as np

from . import bie
from .inputs import make_workload


def time_calls(fn, reps):
    import torch
    fn()
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    for _ in range(reps):
        fn()
    t1.record()
    t1.synchronize()
    return t0.elapsed_time(t1) * 1e3 / reps


def main():
    import torch
    ap = argparse.ArgumentParser()
    ap.add_argument("--workloads", nargs="+", default=["spheres512_p12", "spheres4096_p8", "spheres1024_p16"])
    ap.add_argument("--reps", type=int, default=50)
    args = ap.parse_args()
    for name in args.workloads:
        w = make_workload(name)
        res = {}
        for mf in (0, 1):
            s = bie.Spheres(w["centres"], w["p"], near_gap=1.0, legendre_mfma=mf)
            mu = torch.from_numpy(np.random.default_rng(0).standard_normal(3 * s.N)).cuda()
            u = torch.empty_like(mu)
            for prec, pname in ((bie.MIXED, "f32"), (bie.FP64, "f64")):
                res[f"self_{pname}_{'mfma' if mf else 'fma'}_us"] = time_calls(
                    lambda: s.apply(bie.OP_SD_BIE | bie.STAGE_SELF, mu, u=u, precision=prec), args.reps)
                res[f"forward_{pname}_{'mfma' if mf else 'fma'}_us"] = time_calls(
                    lambda: s.vsh_forward(mu, precision=prec), args.reps)
            n_spheres, P, p = s.nb, s.P, s.p
            s.close()
        print(json.dumps(dict(workload=name, n_spheres=n_spheres, p=p, nodes_per_sphere=P, **res)), flush=True)


if __name__ == "__main__":
    main()
