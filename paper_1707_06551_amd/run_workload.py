"""Solve a named synthetic workload on one GPU, back to back over seeds.

Each seed places the spheres and draws the right-hand side (``inputs.make_workload``),
builds the context (set-up time reported apart) and solves the workload's problem to
the requested tolerance; one JSON line per seed, then a summary line.

Usage: python -m paper_1707_06551_amd.run_workload spheres2048_p12_slip --seeds 16 --precision mixed --precond m0
       python -m paper_1707_06551_amd.run_workload spheres4096_p8 --precond m0r
       python -m paper_1707_06551_amd.run_workload spheres512_p12 --formulation traction

--formulation traction solves a mobility workload (applied forces and torques, no slip)
in the paper's own form (Eqs. 5.7-5.8) instead of the bordered one; with it the
velocities of the bordered solve are reported beside, as their relative difference.
"""
import argparse
import json
import time

import numpy as np

from . import bie
from .inputs import make_workload, slip_field

PRECONDS = {"none": bie.PC_NONE, "m0": bie.PC_M0, "mlp": bie.PC_MLP, "m0r": bie.PC_M0 | bie.PC_RIGID,
            "mlpr": bie.PC_MLP | bie.PC_RIGID, "mlpl": bie.PC_MLP | bie.PC_LOCAL,
            "mlprl": bie.PC_MLP | bie.PC_RIGID | bie.PC_LOCAL}


def solve_one(w, precision, precond, tol, weights=None, max_iter=3000, formulation="bordered", near_gap=None):
    import torch
    t0 = time.perf_counter()
    s = bie.Spheres(w["centres"], w["p"], near_gap=near_gap)
    if precond & bie.PC_MLP:
        s.load_precond(weights)
    slip = None
    if w["problem"] == "mobility_slip":
        xyz, _ = s.nodes()
        sphere_of = np.arange(s.N) // s.P
        normals = xyz - w["centres"][sphere_of]
        slip = torch.from_numpy(slip_field(w["slip_coef"], normals, sphere_of).reshape(-1)).cuda()
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    t0 = time.perf_counter()
    extra = {}
    if w["problem"] == "resistance":
        out = s.solve_resistance(w["v"], w["omega"], tol=tol, precision=precision, precond=precond, max_iter=max_iter)
    elif formulation == "traction":
        if slip is not None:
            raise SystemExit("the traction formulation takes applied forces and torques only (no slip)")
        out = s.solve_mobility_traction(w["F"], w["T"], tol=tol, precision=precision, precond=precond,
                                        max_iter=max_iter)
    else:
        out = s.solve_mobility(w["F"], w["T"], slip=slip, tol=tol, precision=precision, precond=precond,
                               max_iter=max_iter)
    dt = time.perf_counter() - t0
    info = out[-1]
    if formulation == "traction" and w["problem"] == "mobility":
        ref = s.solve_mobility(w["F"], w["T"], tol=tol, precision=precision, precond=bie.PC_M0, max_iter=max_iter)
        extra = dict(vs_bordered=float(max(np.linalg.norm(out[0] - ref[0]) / np.linalg.norm(ref[0]),
                                           np.linalg.norm(out[1] - ref[1]) / np.linalg.norm(ref[1]))),
                     bordered_iters=ref[-1]["iters"])
    s.close()
    return dict(seed=w["seed"], iters=info["iters"], outer_steps=info["outer_steps"],
                rel_residual=info["rel_residual"], converged=bool(info["converged"]),
                fallback_used=info["fallback_used"], solve_s=dt, setup_s=t_setup, **extra)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("workload")
    ap.add_argument("--seeds", type=int, default=1)
    ap.add_argument("--seed0", type=int, default=0)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="mixed")
    ap.add_argument("--precond", choices=sorted(PRECONDS), default="m0")
    ap.add_argument("--tol", type=float, default=1e-8)
    ap.add_argument("--weights", default=None, help="MLP weights (.npz) for mlp / mlpr")
    ap.add_argument("--formulation", choices=["bordered", "traction"], default="bordered",
                    help="mobility workloads: bordered S + D form or the paper's K + L form (Eq. 5.8)")
    ap.add_argument("--near-gap", type=float, default=0.0,
                    help="d* of Eq. 4.5 (<= 0: measured for the default precision 1e-8)")
    args = ap.parse_args()
    precision = bie.MIXED if args.precision == "mixed" else bie.FP64
    precond = PRECONDS[args.precond]
    weights = None
    if args.precond.startswith("mlp"):
        from .precond_train import DEFAULT_FILES, load_weights
        from .inputs import WORKLOADS
        if args.precond.startswith("mlpr"):
            key = "m0r"
        else:
            key = "m0" if WORKLOADS[args.workload]["problem"] == "resistance" else "mob"
        weights, meta = load_weights(args.weights or DEFAULT_FILES[key])
        if meta.get("composition") == "local":
            precond |= bie.PC_LOCAL
    rows = []
    for k in range(args.seeds):
        w = make_workload(args.workload, seed=args.seed0 + k)
        r = solve_one(w, precision, precond, args.tol, weights, formulation=args.formulation,
                      near_gap=args.near_gap if args.near_gap > 0 else None)
        rows.append(r)
        print(json.dumps(dict(workload=args.workload, precision=args.precision, precond=args.precond,
                              formulation=args.formulation, **r)), flush=True)
    print(json.dumps(dict(workload=args.workload, precision=args.precision, precond=args.precond, seeds=len(rows),
                          total_solve_s=sum(r["solve_s"] for r in rows), total_iters=sum(r["iters"] for r in rows),
                          all_converged=all(r["converged"] for r in rows))), flush=True)


if __name__ == "__main__":
    main()
