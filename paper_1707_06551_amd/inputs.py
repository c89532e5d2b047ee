"""Seeded synthetic workloads (sphere placements and right-hand-side draws).

This module holds no arithmetic of the boundary integral method: it only draws random
numbers and places spheres.  Both the HIP path and the CPU oracle consume its outputs.

Placement: random sequential addition.  Centres are drawn i.i.d. uniform in
[1, L-1]^3 (so each unit sphere lies inside [0, L]^3) and a draw is rejected when its
surface gap to any accepted sphere is below ``min_gap``.  For a target volume fraction
phi, L = (n * 4 pi / 3 / phi)^(1/3).

Right-hand sides are drawn from the same generator after placement.
"""
import math

import numpy as np

# Workloads of the benchmark suite: spheres, SH order, volume fraction or box, gap, problem.
WORKLOADS = {
    "spheres8_p8": dict(n=8, p=8, box=8.0, min_gap=0.5, problem="resistance", tol=1e-10),
    "spheres512_p12": dict(n=512, p=12, phi=0.10, min_gap=0.2, problem="mobility", tol=1e-8),
    "spheres4096_p8": dict(n=4096, p=8, phi=0.15, min_gap=0.1, problem="resistance", tol=1e-8),
    "spheres1024_p16": dict(n=1024, p=16, phi=0.30, min_gap=0.02, problem="resistance", tol=1e-8),
    "spheres2048_p12_slip": dict(n=2048, p=12, phi=0.25, min_gap=0.02, problem="mobility_slip", tol=1e-8),
    "spheres64_p16_train": dict(n=64, p=16, phi=0.25, min_gap=0.02, problem="resistance", tol=1e-10),
    "spheres64_p12_slip_train": dict(n=64, p=12, phi=0.25, min_gap=0.02, problem="mobility_slip", tol=1e-10),
}


def box_side(n, phi):
    return (n * 4.0 * math.pi / 3.0 / phi) ** (1.0 / 3.0)


def place_spheres(n, box, min_gap, rng, max_tries=2_000_000):
    """Random sequential addition of n unit spheres in [0, box]^3 (centres in
    [1, box-1]^3) with pairwise surface gap >= min_gap.  Uses a uniform cell list."""
    lo, hi = 1.0, box - 1.0
    dmin = 2.0 + min_gap
    dmin2 = dmin * dmin
    ncell = max(1, int((hi - lo) / dmin))
    h = (hi - lo) / ncell
    cells = {}
    out = np.empty((n, 3))
    k = 0
    tries = 0
    reach = int(math.ceil(dmin / h))
    while k < n:
        tries += 1
        if tries > max_tries:
            raise RuntimeError(f"placement stalled after {k} of {n} spheres")
        c = lo + (hi - lo) * rng.random(3)
        ci = tuple(np.minimum(((c - lo) / h).astype(int), ncell - 1))
        ok = True
        for dx in range(-reach, reach + 1):
            for dy in range(-reach, reach + 1):
                for dz in range(-reach, reach + 1):
                    lst = cells.get((ci[0] + dx, ci[1] + dy, ci[2] + dz))
                    if not lst:
                        continue
                    d = out[lst] - c
                    if np.any(np.einsum("ij,ij->i", d, d) < dmin2):
                        ok = False
                        break
                if not ok:
                    break
            if not ok:
                break
        if ok:
            out[k] = c
            cells.setdefault(ci, []).append(k)
            k += 1
    return out


def place_spheres_radii(radii, box, min_gap, rng, max_tries=2_000_000):
    """Random sequential addition of spheres of the given radii (largest first) in
    [0, box]^3, each inside the box, with pairwise surface gap >= min_gap.  Returns the
    centres in the order of `radii`."""
    radii = np.asarray(radii, dtype=np.float64)
    order = np.argsort(-radii, kind="stable")
    out = np.empty((len(radii), 3))
    placed = []
    tries = 0
    for idx in order:
        a = radii[idx]
        while True:
            tries += 1
            if tries > max_tries:
                raise RuntimeError(f"placement stalled after {len(placed)} of {len(radii)} spheres")
            cand = a + (box - 2 * a) * rng.random(3)
            if placed:
                pc = out[placed]
                gap = np.linalg.norm(pc - cand[None, :], axis=1) - radii[placed] - a
                if gap.min() < min_gap:
                    continue
            out[idx] = cand
            placed.append(idx)
            break
    return out


def window(centres, n, rng):
    """n spheres cut out of a larger placement: the sphere nearest to a uniformly drawn
    point of the middle half of the placement's bounding box, and its n - 1 nearest
    neighbours (centre distance).  Gives small configurations with the neighbour
    statistics of the bulk of a dense suspension, which random sequential addition of
    n spheres in a small box cannot reach at the same volume fraction."""
    c = np.asarray(centres, dtype=np.float64)
    lo, hi = c.min(axis=0), c.max(axis=0)
    x = lo + (hi - lo) * (0.25 + 0.5 * rng.random(3))
    k0 = int(np.argmin(np.einsum("ij,ij->i", c - x, c - x)))
    d = np.einsum("ij,ij->i", c - c[k0], c - c[k0])
    return c[np.argsort(d, kind="stable")[:n]].copy()


def make_workload(name, seed=0):
    """Centres and right-hand-side data of a named workload.

    resistance:     v, omega ~ N(0, 1) per component
    mobility:       F, T ~ N(0, 1)
    mobility_slip:  F = T = 0 and slip coefficients ~ N(0, 1) (see ``slip_field``)
    """
    cfg = dict(WORKLOADS[name])
    rng = np.random.default_rng(seed)
    box = cfg.get("box") or box_side(cfg["n"], cfg["phi"])
    centres = place_spheres(cfg["n"], box, cfg["min_gap"], rng)
    n = cfg["n"]
    cfg["box"] = box
    out = dict(name=name, seed=seed, centres=centres, **cfg)
    if cfg["problem"] == "resistance":
        out["v"] = rng.standard_normal((n, 3))
        out["omega"] = rng.standard_normal((n, 3))
    elif cfg["problem"] == "mobility":
        out["F"] = rng.standard_normal((n, 3))
        out["T"] = rng.standard_normal((n, 3))
    else:
        out["F"] = np.zeros((n, 3))
        out["T"] = np.zeros((n, 3))
        out["slip_coef"] = rng.standard_normal((n, len(MONOMIALS4), 3))
    return out


MONOMIALS4 = [(a, b, c) for a in range(5) for b in range(5) for c in range(5) if a + b + c <= 4]


def slip_field(slip_coef, normals, sphere_of):
    """Tangential active slip of degree <= 4 (a squirmer-like surface velocity):
    u_s(n) = (I - n n^T) sum_alpha C_alpha n^alpha for each node with unit normal n,
    C drawn per sphere.  normals (N, 3), sphere_of (N,) -> (N, 3)."""
    n = np.asarray(normals, dtype=np.float64)
    C = slip_coef[sphere_of]                                  # (N, 35, 3)
    mono = np.stack([n[:, 0] ** a * n[:, 1] ** b * n[:, 2] ** c for (a, b, c) in MONOMIALS4], axis=1)
    u = np.einsum("nk,nkc->nc", mono, C)
    return u - np.sum(u * n, axis=1)[:, None] * n


def random_density(n_nodes, rng):
    """A random node density (N, 3) ~ N(0, 1) for matvec parity tests."""
    return rng.standard_normal((n_nodes, 3))


def lattice_centres(units, q):
    """Centres of the monodisperse cubic lattice of the scaling experiment (Section 6,
    Fig. 8 (a), (b)) rescaled to unit spheres: (units + 1)^3 spheres on the vertices of
    a cubic grid of spacing 2 / (1 - 2^-q) (radius 1 - 2^-q at spacing 2 in the paper's
    units): spacing 4 (q = 1, loosely packed) or 32/15 (q = 4, densely packed, gap 2/15)."""
    h = 2.0 / (1.0 - 2.0 ** (-q))
    g = np.arange(units + 1, dtype=np.float64) * h
    x, y, z = np.meshgrid(g, g, g, indexing="ij")
    return np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)


def lattice_poly(units, q):
    """The polydisperse lattice units of the scaling experiment (Section 6, Fig. 8 (c),
    (d)) rescaled so that the vertex spheres are unit: vertex spheres of radius 1 on a
    cubic grid of spacing 2 / (1 - 2^-q), one sphere of radius 2 - sqrt(2) at the centre
    of every cube face and one of radius sqrt(2) - 1 at the centre of every cube.
    Returns (centres (n, 3), radii (n,)); (units+1)^3 + 3 (units+1) units^2 + units^3
    spheres (15, 71, 429, 2969, 22065 for 1, 2, 4, 8, 16 units).  With the printed radii a
    face sphere overlaps its vertex spheres once (3 - sqrt(2)) (1 - 2^-q) > sqrt(2),
    i.e. for q >= 4: those lattices are refused."""
    rv = 1.0 - 2.0 ** (-q)
    if (3.0 - math.sqrt(2.0)) * rv >= math.sqrt(2.0):
        raise ValueError(f"q = {q}: face and vertex spheres of the printed radii overlap")
    h = 2.0 / rv
    v = lattice_centres(units, q)
    g = np.arange(units + 1, dtype=np.float64) * h
    m = (np.arange(units, dtype=np.float64) + 0.5) * h
    faces = []
    for axis in range(3):
        a, b, c = np.meshgrid(g, m, m, indexing="ij")
        f = np.stack([a.ravel(), b.ravel(), c.ravel()], axis=1)
        faces.append(np.roll(f, axis, axis=1))
    x, y, z = np.meshgrid(m, m, m, indexing="ij")
    cen = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    centres = np.concatenate([v] + faces + [cen], axis=0)
    radii = np.concatenate([np.ones(len(v)), np.full(sum(len(f) for f in faces), 2.0 - math.sqrt(2.0)),
                            np.full(len(cen), math.sqrt(2.0) - 1.0)])
    return centres, radii
