"""Writes tests/golden/window64_p8.json from the FP64 oracle only: a full oracle solve
of a 64-sphere case beside the library's.

The case: the 64 spheres nearest to a random interior point of a 1024-sphere placement at
volume fraction 0.30, min gap 0.02 (random sequential addition, seed 8; the windows the
learned correction trains on), p = 8, near/far threshold d* = 1, resistance problem
(completed double layer, Eq. 5.19) with rigid velocities v, omega ~ N(0, 1) (seed 9).
The oracle's unpreconditioned GMRES (restart 300) runs to relative residual 1e-11; its
operator applications are split over target spheres across host processes (the same
oracle code on each chunk).  Stores the centres, v, omega, F, T, the iteration count,
the wall time and the number of processes.

Run from the repository root: python tests/golden/make_golden_window64.py [--procs 7]
"""
import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle.grid import Geometry  # noqa: E402
from oracle.operators import Operators  # noqa: E402
from oracle.solvers import gmres, rigid_rhs  # noqa: E402
from paper_1707_06551_amd.inputs import box_side, place_spheres, window  # noqa: E402

P_ORDER = 8
_ops = None


def _init(centres):
    global _ops
    _ops = Operators(Geometry(centres, P_ORDER, near_gap=1.0))


def _apply_chunk(args):
    z, tg = args
    return _ops.apply("DN_BIE", z, targets=tg)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--procs", type=int, default=7)
    args = ap.parse_args()
    big = place_spheres(1024, box_side(1024, 0.30), 0.02, np.random.default_rng(8))
    centres = window(big, 64, np.random.default_rng(8 + 7919))
    rng = np.random.default_rng(9)
    v, omega = rng.standard_normal((64, 3)), rng.standard_normal((64, 3))
    g = Geometry(centres, P_ORDER, near_gap=1.0)
    b = rigid_rhs(g, v, omega).reshape(-1)
    chunks = np.array_split(np.arange(g.N), 4 * args.procs)
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(args.procs, initializer=_init, initargs=(centres,)) as pool:
        def apply_fn(z):
            zz = z.reshape(g.N, 3)
            parts = pool.map(_apply_chunk, [(zz, tg) for tg in chunks])
            return np.concatenate(parts).reshape(-1)
        psi, info = gmres(apply_fn, b, tol=1e-11, restart=300, max_iter=2000)
    wall = time.perf_counter() - t0
    F, T = Operators(g).moments(psi.reshape(g.N, 3))
    out = dict(
        source="oracle (numpy float64), unpreconditioned GMRES(300) to relative residual 1e-11",
        case="64-sphere window of a 1024-sphere placement, phi 0.30, min gap 0.02; p = 8, d* = 1; resistance",
        p=P_ORDER, near_gap=1.0, centres=centres.tolist(), v=v.tolist(), omega=omega.tolist(),
        F=F[..., 0].tolist(), T=T[..., 0].tolist(), iters=info["iters"], rel_residual=info["rel_residual"],
        oracle_seconds=wall, oracle_processes=args.procs,
    )
    path = os.path.join(ROOT, "tests", "golden", "window64_p8.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path, info["iters"], info["rel_residual"], f"{wall:.1f} s")


if __name__ == "__main__":
    main()
