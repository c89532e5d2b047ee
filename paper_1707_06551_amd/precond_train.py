"""Training driver of the learned close-pair coarse correction (BIE_PC_MLP).

Data: for each training configuration (seeded placements of a 64-sphere training
workload), random low-mode right-hand sides b = P xi (xi ~ N(0, 1), 25 coefficients per
sphere) are solved with the plain float64 method; the target is t = R x - R B b, the
part of the low-mode response that the base preconditioner B misses.  Two forms:
  --form dn   the completed double-layer (resistance) form, A x = b; B is the
              isolated-sphere inverse M0 (--base m0), or M0 followed by the global
              rigid-mode coarse correction (--base m0r, BIE_PC_RIGID);
  --form mob  the bordered mobility form (Eqs. 5.15, 5.17) with b = [P xi; 0], a
              low-mode slip with no applied force or torque; B = M0 and R, P act on
              the density part only.  Training runs on
the GPU in the library's own forward / backward / Adam kernels (bie_mlp_train).
Applied at full strength the additive correction over-corrects, so a relaxation omega
(theta -> omega theta) is chosen on held-out configurations by GMRES iteration count
and folded into the saved output layer.

Composition (--composition): additive, z = B r + P zeta(R r) (BIE_PC_MLP), or local,
z = z0 + P zeta(R (r - A_loc z0)) with z0 = B r and A_loc the self and near-series part
of the operator (BIE_PC_MLP | BIE_PC_LOCAL).  The library forms each sample's input and
target (bie_precond_sample).  --windows K trains on 64-sphere windows cut from
1024-sphere placements (K windows per placement) at the volume fraction of the form's
large workload (0.30 for the resistance form, 0.25 for the mobility form with slip): the
bulk neighbour statistics of the dense suspension.

Usage: python -m paper_1707_06551_amd.precond_train --configs 200 --rhs 4 --p 16 --epochs 400 [--base m0r]
       python -m paper_1707_06551_amd.precond_train --form mob --configs 200 --rhs 4 --p 12 --epochs 400
       python -m paper_1707_06551_amd.precond_train --base m0r --composition local --windows 16 --configs 500 \
           --select 1 --select-workload spheres1024_p16 --omegas 0.075,0.1,0.125,0.15 --procs 6
"""
import argparse
import json
import os
import time

import numpy as np

from . import bie
from .inputs import make_workload, slip_field

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_WEIGHTS = os.path.join(HERE, "weights", "precond_dn.npz")
HIDDEN = 64


def init_weights(seed=0, out_scale=1e-3):
    """Glorot-uniform hidden layers, a small output layer (the correction starts near 0)."""
    rng = np.random.default_rng(seed)
    shapes = [(bie.NFEAT, HIDDEN), (HIDDEN,), (HIDDEN, HIDDEN), (HIDDEN,), (HIDDEN, 278), (278,)]
    parts = []
    for s in shapes:
        if len(s) == 1:
            parts.append(np.zeros(s))
        else:
            lim = np.sqrt(6.0 / (s[0] + s[1])) * (out_scale if s[1] == 278 else 1.0)
            parts.append(rng.uniform(-lim, lim, s))
    w = np.concatenate([p.reshape(-1) for p in parts]).astype(np.float32)
    assert w.size == bie.mlp_n_weights()
    return w


BASES = {"m0": bie.PC_M0, "m0r": bie.PC_M0 | bie.PC_RIGID}
DEFAULT_FILES = {"m0": DEFAULT_WEIGHTS, "m0r": os.path.join(HERE, "weights", "precond_dn_rigid.npz"),
                 "mob": os.path.join(HERE, "weights", "precond_mob.npz")}
# per form: operator, training workload
FORMS = {"dn": (bie.OP_DN_BIE, "spheres64_p16_train"), "mob": (bie.OP_MOBILITY, "spheres64_p12_slip_train")}


def config_samples(sph, n_rhs, rng, tol=1e-8, base=bie.PC_M0, op=bie.OP_DN_BIE, local=False):
    """(xi, target) of one configuration: (nb, n_rhs, 25) each, plus solve statistics.
    The library forms both (bie_precond_sample): target = R x - R B b, xi = R b, or
    R (b - A_loc B b) for the local-residual composition."""
    import torch
    xi = np.empty((sph.nb, n_rhs, bie.NLOW))
    target = np.empty_like(xi)
    iters = []
    for r in range(n_rhs):
        rho = torch.from_numpy(rng.standard_normal(sph.nb * bie.NLOW)).cuda()
        b = sph.lowmodes_synth(rho)
        if op == bie.OP_MOBILITY:
            b = torch.cat([b, torch.zeros(6 * sph.nb, dtype=b.dtype, device=b.device)])
        x, info = sph.solve(op, b, tol=tol, precision=bie.FP64, precond=base)
        if not info["converged"]:
            raise RuntimeError(f"training solve did not converge: {info}")
        iters.append(info["iters"])
        a, t = sph.precond_sample(op, base | (bie.PC_LOCAL if local else 0), b, x)
        torch.cuda.synchronize()
        xi[:, r, :] = a.cpu().numpy().reshape(sph.nb, bie.NLOW)
        target[:, r, :] = t.cpu().numpy().reshape(sph.nb, bie.NLOW)
    return xi, target, iters


def _placement(args):
    """Centres of one large placement (random sequential addition), for windows."""
    n, phi, gap, seed = args
    from .inputs import box_side, place_spheres
    return place_spheres(n, box_side(n, phi), gap, np.random.default_rng(seed))


def window_configs(n_configs, per_placement, seed0, n=64, big=1024, phi=0.30, gap=0.02, procs=16):
    """n-sphere windows of larger placements at volume fraction phi: ceil(n_configs /
    per_placement) placements of `big` spheres (seeds seed0, seed0 + 1, ...; built in
    parallel host processes before the GPU is used), per_placement windows each."""
    import multiprocessing as mp
    from .inputs import window
    n_pl = (n_configs + per_placement - 1) // per_placement
    jobs = [(big, phi, gap, seed0 + k) for k in range(n_pl)]
    if procs <= 1 or n_pl == 1:
        placements = [_placement(j) for j in jobs]
    else:
        with mp.get_context("fork").Pool(min(procs, n_pl)) as pool:
            placements = pool.map(_placement, jobs)
    out = []
    for k, c in enumerate(placements):
        rng = np.random.default_rng(seed0 + 7919 * (k + 1))
        for _ in range(per_placement):
            if len(out) < n_configs:
                out.append(window(c, n, rng))
    return out


def _samples_of(job):
    """Samples of configurations ks (one GPU process): [(pi, pj, feats, frames, xi, target, iters)]."""
    ks, centres_list, n_rhs, p, seed0, base, op, local = job
    out = []
    for k, centres in zip(ks, centres_list):
        sph = bie.Spheres(centres, p)
        pi, pj, feats, frames = sph.pair_geometry()
        xi, target, iters = config_samples(sph, n_rhs, np.random.default_rng(seed0 + k + 7919), base=base, op=op,
                                           local=local)
        sph.close()
        out.append((pi, pj, feats, frames, xi, target, iters))
    return out


def build_set(n_configs, n_rhs, p, seed0=1000, workload="spheres64_p16_train", log=print, base=bie.PC_M0,
              op=bie.OP_DN_BIE, local=False, windows=None, procs=1, chunk=8):
    """Training set of n_configs configurations: seeded placements of the training
    workload, or the given list of window centres.  procs > 1 solves chunks of
    configurations in that many GPU processes at once (small systems leave the GPU mostly
    idle between launches); the set is the same for any procs."""
    ts = bie.TrainingSet(n_rhs)
    t0 = time.time()
    centres = [windows[k] if windows is not None else make_workload(workload, seed=seed0 + k)["centres"]
               for k in range(n_configs)]
    jobs = [(list(range(a, min(a + chunk, n_configs))), centres[a:a + chunk], n_rhs, p, seed0, base, op, local)
            for a in range(0, n_configs, chunk)]
    if procs > 1:
        import multiprocessing as mp
        pool = mp.get_context("spawn").Pool(procs)
        results = pool.imap(_samples_of, jobs)
    else:
        pool, results = None, map(_samples_of, jobs)
    done = 0
    try:
        for res in results:
            for (pi, pj, feats, frames, xi, target, iters) in res:
                ts.add(pi, pj, feats, frames, xi, target)
                done += 1
            if log:
                log(f"configs {done}/{n_configs}: {len(pi)} pairs, solve iters {iters}, {time.time() - t0:.1f} s")
    finally:
        if pool is not None:
            pool.close()
            pool.join()
    return ts


OFF_W3 = bie.NFEAT * HIDDEN + HIDDEN + HIDDEN * HIDDEN + HIDDEN   # output layer (W3, b3) start


def scaled(w, omega):
    """Weights whose output (theta) is omega times that of w (theta is linear in W3, b3)."""
    ws = np.array(w, dtype=np.float32, copy=True)
    ws[OFF_W3:] *= omega
    return ws


def select_relaxation(w, p, seeds, omegas=(0.1, 0.15, 0.2, 0.25, 0.3, 0.4, 0.6, 1.0), workload="spheres64_p16_train",
                      log=print, base=bie.PC_M0, local=False, windows=None, precision=bie.FP64):
    """The correction can over-correct at full strength; choose the relaxation omega
    (theta -> omega theta) that minimises the float64 GMRES iterations of the workload's
    problem (resistance, or mobility with active slip) on held-out configurations: the
    workload's placements for `seeds`, or the given window centres (resistance with the
    rigid motions of the workload seeds)."""
    import torch
    table = {om: [] for om in omegas}
    base_its = []

    def run(sph, wk, slip, pc):
        if wk["problem"] == "resistance":
            info = sph.solve_resistance(wk["v"], wk["omega"], tol=1e-8, precond=pc, precision=precision)[-1]
        else:
            info = sph.solve_mobility(wk["F"], wk["T"], slip=slip, tol=1e-8, precond=pc, precision=precision)[-1]
        if log:
            log(f"  selection: seed {wk['seed']}, precond {pc:#x}: {info['iters']} iterations")
        return info["iters"]

    pc_mlp = bie.PC_MLP | (base & bie.PC_RIGID) | (bie.PC_LOCAL if local else 0)
    for k, sd in enumerate(seeds):
        wk = make_workload(workload, seed=sd)
        if windows is not None:
            wk["centres"] = windows[k]
        sph = bie.Spheres(wk["centres"], p)
        slip = None
        if wk["problem"] == "mobility_slip":
            xyz, _ = sph.nodes()
            sphere_of = np.arange(sph.N) // sph.P
            slip = torch.from_numpy(slip_field(wk["slip_coef"], xyz - wk["centres"][sphere_of], sphere_of)
                                    .reshape(-1)).cuda()
        base_its.append(run(sph, wk, slip, base))
        for om in omegas:
            sph.load_precond(scaled(w, om))
            table[om].append(run(sph, wk, slip, pc_mlp))
        sph.close()
    best = min(omegas, key=lambda om: (sum(table[om]), om))
    if log:
        log(f"base iterations {base_its}; with the learned correction: " +
            ", ".join(f"omega {om}: {table[om]}" for om in omegas) + f"; chosen {best}")
    return best, {str(k): v for k, v in table.items()}, base_its


def save_weights(path, w, meta):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    np.savez(path, weights=np.asarray(w, np.float32), meta=np.array(json.dumps(meta)))


def load_weights(path=DEFAULT_WEIGHTS):
    with np.load(path, allow_pickle=False) as z:
        return z["weights"].astype(np.float32), json.loads(str(z["meta"]))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--configs", type=int, default=200)
    ap.add_argument("--holdout", type=int, default=20)
    ap.add_argument("--rhs", type=int, default=4)
    ap.add_argument("--p", type=int, default=16)
    ap.add_argument("--epochs", type=int, default=300)
    ap.add_argument("--batch", type=int, default=8)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--select", type=int, default=4, help="held-out configurations for choosing the relaxation")
    ap.add_argument("--base", choices=sorted(BASES), default="m0",
                    help="preconditioner the correction is trained on top of (m0r: M0 + BIE_PC_RIGID, dn form only)")
    ap.add_argument("--form", choices=sorted(FORMS), default="dn",
                    help="dn: resistance (completed double-layer) form; mob: bordered mobility form with slip")
    ap.add_argument("--composition", choices=["additive", "local"], default="additive",
                    help="additive: z = B r + P zeta(R r); local: z = z0 + P zeta(R (r - A_loc z0)), z0 = B r "
                         "(BIE_PC_LOCAL)")
    ap.add_argument("--windows", type=int, default=0,
                    help="> 0: train on 64-sphere windows of 1024-sphere placements at volume fraction 0.30 "
                         "(this many windows per placement) instead of the workload's placements")
    ap.add_argument("--select-workload", default=None,
                    help="choose the relaxation on this workload's placements (seeds 1..select, mixed precision) "
                         "instead of held-out training configurations")
    ap.add_argument("--omegas", default="0.1,0.15,0.2,0.25,0.3,0.4,0.6,1.0", help="relaxations scanned")
    ap.add_argument("--procs", type=int, default=1, help="GPU processes forming the training samples")
    ap.add_argument("--out", default=None)
    args = ap.parse_args()
    if args.form == "mob" and args.base != "m0":
        ap.error("the mobility form is trained on M0 only (BIE_PC_RIGID acts on the resistance form)")
    base = BASES[args.base]
    local = args.composition == "local"
    op, workload = FORMS[args.form]
    out = args.out or DEFAULT_FILES["mob" if args.form == "mob" else args.base]
    wtrain = whold = wsel = None
    # windows: 64-sphere windows of 1024-sphere placements at the volume fraction of the
    # form's large workload (resistance 0.30, mobility with slip 0.25)
    wphi = 0.30 if args.form == "dn" else 0.25
    if args.windows:
        # host work first (forked placement processes), then the GPU
        wtrain = window_configs(args.configs, args.windows, seed0=1000, phi=wphi)
        whold = window_configs(args.holdout, args.windows, seed0=900000, phi=wphi)
        if not args.select_workload:
            wsel = window_configs(args.select, args.windows, seed0=600000, phi=wphi)
    omegas = tuple(float(x) for x in args.omegas.split(","))
    if args.select_workload:
        sel = dict(seeds=list(range(1, 1 + args.select)), workload=args.select_workload, windows=None,
                   precision=bie.MIXED)
    else:
        sel = dict(seeds=[600000 + k for k in range(args.select)], workload=workload, windows=wsel,
                   precision=bie.FP64)
    train = build_set(args.configs, args.rhs, args.p, seed0=1000, base=base, op=op, workload=workload, local=local,
                      windows=wtrain, procs=args.procs)
    hold = build_set(args.holdout, args.rhs, args.p, seed0=900000, base=base, op=op, workload=workload, local=local,
                     windows=whold, procs=args.procs)
    w0 = init_weights(0)
    l0, _ = hold.eval(w0)
    t0 = time.time()
    w, hist = train.train(w0, args.epochs, cfg_per_batch=args.batch, lr=args.lr)
    t_train = time.time() - t0
    l1, _ = hold.eval(w)
    ltr, _ = train.eval(w)
    omega, table, base_its = select_relaxation(w, args.p, omegas=omegas, base=base, local=local, **sel)
    meta = dict(version=2, formulation="MOBILITY" if args.form == "mob" else "DN_BIE", base=args.base,
                composition=args.composition, workload=workload,
                windows=(f"64-sphere windows of 1024-sphere placements, phi {wphi:.2f}, {args.windows} per placement"
                         if args.windows else None),
                selection=(f"{args.select_workload} seeds 1-{args.select}, mixed precision" if args.select_workload
                           else f"{args.select} held-out training configurations, float64"),
                rigid_modes=("left to the rigid-mode correction" if base & bie.PC_RIGID else "included"),
                p=args.p, hidden=HIDDEN, nfeat=bie.NFEAT, nout=278,
                configs=args.configs, rhs=args.rhs, epochs=args.epochs, lr=args.lr, batch=args.batch,
                train_loss=float(ltr), holdout_loss_init=float(l0), holdout_loss=float(l1),
                train_seconds=t_train, relaxation=omega, relaxation_scan=table, base_iters=base_its,
                note="output layer scaled by the relaxation")
    save_weights(out, scaled(w, omega), meta)
    print(json.dumps(dict(meta, loss_hist_first=float(hist[0]), loss_hist_last=float(hist[-1]))))


if __name__ == "__main__":
    main()
