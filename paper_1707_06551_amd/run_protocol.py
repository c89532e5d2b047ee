"""The boundary-integral validation protocol of Section 6 (Eq. 6.2, Fig. 7) on spheres of
the printed radii (0.903, 0.510, 0.262): a point force inside each sphere at half its
radius from the centre gives boundary data gamma = sum G(x, p_l) F_l, an exterior Stokes
flow; the completed double-layer equation (1/2 I + D + N) psi = gamma is solved, and
D[psi] + N[psi] evaluated at fluid points at distances r_l {1, 10^-0.5, ..., 10^-6} from
each surface must reproduce gamma there.  The relative error per distance class and p
is the accuracy of the whole pipeline (transforms, near series, far quadrature, solve)
up to the boundary.  The centres of the paper's Fig. 6 are not given: the spheres here
are placed with gaps 0.15 and 0.2 between them (the figure is not reproduced).

Usage: python -m paper_1707_06551_amd.run_protocol [--p 4 8 12 16 20]
"""
import argparse
import json
import math

import numpy as np

from . import bie

RADII = np.array([0.903, 0.510, 0.262])
CENTRES = np.array([[0.0, 0.0, 0.0], [0.903 + 0.510 + 0.15, 0.0, 0.0], [0.4, 0.903 + 0.262 + 0.2, 0.3]])


def stokeslet_flow(src, forces, x):
    """sum_l G(x, p_l) F_l with G of Eq. 2.19 (viscosity 1)."""
    u = np.zeros((x.shape[0], 3))
    for p, f in zip(src, forces):
        r = x - p[None, :]
        d = np.linalg.norm(r, axis=1)[:, None]
        u += (f[None, :] / d + r * (r @ f)[:, None] / d ** 3) / (8.0 * math.pi)
    return u


def protocol_points(rng, per_class=8):
    """Targets at distance r_l * 10^(-k/2), k = 0..12, from each sphere's surface, kept
    where they are in the fluid (outside every sphere)."""
    xs, cls = [], []
    for k in range(13):
        h = 10.0 ** (-k / 2.0)
        for c, r in zip(CENTRES, RADII):
            d = rng.standard_normal((per_class, 3))
            d /= np.linalg.norm(d, axis=1)[:, None]
            x = c[None, :] + (r + r * h) * d
            gap = np.linalg.norm(x[:, None, :] - CENTRES[None, :, :], axis=-1) - RADII[None, :]
            keep = gap.min(axis=1) > 0.0
            xs.append(x[keep])
            cls += [k] * int(keep.sum())
    return np.concatenate(xs), np.array(cls)


def run(p, rng_seed=0):
    import torch
    rng = np.random.default_rng(rng_seed)
    dirs = rng.standard_normal((3, 3))
    src = CENTRES + 0.5 * RADII[:, None] * dirs / np.linalg.norm(dirs, axis=1)[:, None]
    forces = rng.standard_normal((3, 3))
    x, cls = protocol_points(rng)
    s = bie.Spheres(CENTRES, p, near_gap=1.0, radii=RADII)
    nodes, _w = s.nodes()
    b = torch.from_numpy(stokeslet_flow(src, forces, nodes).reshape(-1)).cuda()
    psi, info = s.solve(bie.OP_DN_BIE, b, tol=1e-13, precond=bie.PC_M0, max_iter=2000)
    u = s.eval_field(bie.OP_DN_BIE, psi, x).cpu().numpy().reshape(-1, 3)
    exact = stokeslet_flow(src, forces, x)
    err = np.linalg.norm(u - exact, axis=1) / np.abs(exact).max()
    s.close()
    per = {f"1e-{k / 2:g}": float(err[cls == k].max()) for k in range(13) if (cls == k).any()}
    return dict(p=p, iters=info["iters"], converged=info["converged"], max_rel_err_by_distance=per,
                max_rel_err=float(err.max()))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--p", type=int, nargs="+", default=[4, 8, 12, 16, 20])
    args = ap.parse_args()
    for p in args.p:
        print(json.dumps(dict(protocol="Eq. 6.2, radii 0.903 / 0.510 / 0.262", **run(p))), flush=True)


if __name__ == "__main__":
    main()
