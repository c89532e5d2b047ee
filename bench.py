"""Benchmark: P2P pair-interactions/s and time-to-solution of the sphere Stokes BIE.

Workload (default): 2048 unit spheres, p = 12 (638,976 nodes), volume fraction 0.25,
min gap 0.02, active slip of degree <= 4 with zero applied force and torque (the
mobility problem of Section 5, Problem 4, Eqs. 5.14-5.17, in the bordered second-kind
form); 16 seeded configurations.  One step = one solve of one configuration (step i
solves seed i mod 16) to relative residual 1e-8 with float32 transforms and far-field
sums inside float64 GMRES with iterative refinement, and the isolated-sphere block
preconditioner with the learned close-pair correction (--precond m0: without it).  Near pairs use the
separation threshold of Eq. 4.5 measured for the requested precision 1e-8.  Every
context is built and every input is resident on the device before the timed region
(set-up time reported apart).  value = far-field pair interactions evaluated by the
timed solves / wall time of the timed solves.

Reported beside it, on seed 0: plain float64 GMRES (no preconditioner) and float64
GMRES with the same preconditioner (isolating the mixed-precision gain from the
preconditioning gain), the roofline of the dominant kernel (float32 far-field pair sum,
timed live with HIP events on the library's stream), the near-series stage, per-step
device time of each step of the hot path, and the CPU oracle: its far-field direct sum
on a bounded sample of target nodes across the host's cores, and its full solve of the
8-sphere workload beside the library's.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--precond m0|mlp|m0r|mlpr]
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "P2P pair-interactions/s + time-to-solution at 1e-8 vs plain FP64 GMRES"
FLOP_PER_PAIR = {"S": 29, "D": 30, "SD": 38}   # FMA = 2, rsqrt = 1 (straight-line formula count)
PEAK_FP32_VECTOR_TFLOPS = 157.3
PEAK_FP64_VECTOR_TFLOPS = 78.6
N_SEEDS = {"spheres2048_p12_slip": 16}
MLP_WEIGHTS = {"mobility": "precond_mob.npz", "resistance": "precond_dn.npz"}


def code_sha(path):
    """First 16 hex digits of the SHA-256 of a C++ / HIP source with its // comments,
    trailing blanks and empty lines removed: changes to the code change it, comment
    edits do not.  (No string literal in the kernel sources holds //.)"""
    import hashlib
    lines = []
    for line in open(path, encoding="utf-8").read().splitlines():
        code = line.split("//", 1)[0].rstrip()
        if code:
            lines.append(code)
    return hashlib.sha256("\n".join(lines).encode()).hexdigest()[:16]


def profile_fields(name):
    """key: value lines of a committed profile summary, or {}."""
    try:
        return dict(l.split(": ", 1) for l in open(os.path.join(ROOT, "profiles", name)).read().splitlines()
                    if ": " in l and l[:1].isalpha())
    except OSError:
        return {}


def measured_counters(workload):
    """HBM bytes and hardware-counted float32 flop per pair of the far-field kernel from
    the committed PMC summary of this workload, or None for each when the kernel's code
    has changed since the counters were taken."""
    src = os.path.join(ROOT, "paper_1707_06551_amd", "csrc", "p2p.hip")
    f = profile_fields(f"far_kernel_{workload}_pmc.md")
    if not f or f.get("source_sha256_16", "").strip() != code_sha(src):
        return None, None
    def num(k):
        try:
            return float(f[k])
        except (KeyError, ValueError):
            return None
    return num("traffic_bytes_per_launch"), num("counted_flop_per_pair")


def cpu_baseline_worker(args):
    """One host process of the CPU baseline: the oracle's far-field S + D direct sum for
    chunks of random target nodes (all sources) until `seconds` have passed."""
    name, seed, chunk, seconds = args
    from threadpoolctl import threadpool_limits

    from oracle.grid import Geometry
    from oracle.operators import Operators
    from paper_1707_06551_amd.inputs import make_workload
    w = make_workload(name)
    g = Geometry(w["centres"], w["p"], near_gap=1.0)
    ops = Operators(g)
    mu = np.random.default_rng(5).standard_normal((g.N, 3))
    rng = np.random.default_rng(seed)
    allowed_per_t = g.nb - 1 - g.near.sum(axis=1)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        nt = pairs = 0
        while time.perf_counter() - t0 < seconds:
            tg = rng.choice(g.N, chunk, replace=False)
            ops.far_part(mu, 1.0, 1.0, targets=tg)
            nt += tg.size
            pairs += int(allowed_per_t[g.sphere_of[tg]].sum()) * g.P
        dt = time.perf_counter() - t0
    return nt, pairs, dt


def log(msg):
    """Progress line on stderr (the JSON result goes to stdout)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def host_cores():
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    return max(1, min(n, 16))


def cpu_baseline(name, seconds=12.0):
    """The oracle's far-field direct sum on a bounded sample (random target nodes x all
    sources) with one process per host core; rate in pair-interactions/s.  Runs before
    the GPU is touched (the worker processes are forked)."""
    import multiprocessing as mp
    cores = host_cores()
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        res = pool.map(cpu_baseline_worker, [(name, 1000 + i, 16, seconds) for i in range(cores)])
    wall = time.perf_counter() - t0
    nt = sum(r[0] for r in res)
    pairs = sum(r[1] for r in res)
    rate = sum(r[1] / r[2] for r in res)
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    return dict(value=rate, unit="pair-interactions/s", cores=cores, kind="oracle",
                sample=f"far-field S+D direct sum (numpy float64, 1 thread per process) for {nt} random target "
                       f"nodes x all sources of {name}, {pairs:.3e} pairs over {cores} processes in "
                       f"{wall:.1f} s wall",
                host_cpus=os.cpu_count(), cpu_model=model)


def cpu_baseline_small_solve():
    """The oracle's full solve of the 8-sphere workload (p = 8, resistance, GMRES to
    1e-10, d* measured for 1e-10 by the oracle's own shell test)."""
    from oracle.calibration import calibrated_gap
    from oracle.grid import Geometry
    from oracle.solvers import solve_resistance
    from paper_1707_06551_amd.inputs import make_workload
    w = make_workload("spheres8_p8")
    d = calibrated_gap(w["p"], w["tol"])
    t0 = time.perf_counter()
    F, T, _psi, info = solve_resistance(Geometry(w["centres"], w["p"], near_gap=d), w["v"], w["omega"], tol=w["tol"])
    return dict(workload=w["name"], seconds=time.perf_counter() - t0, iters=info["iters"],
                rel_residual=info["rel_residual"], near_gap=d, F=F, T=T)


def time_stage(sph, torch, bie, op, stage, precision, reps=20, warmup=3):
    """Median and mean duration (s) of one pass of one stage of op, each pass bracketed
    by its own events on the stream the library launches on (torch's current stream,
    passed at context creation); `warmup` untimed passes first."""
    x = torch.randn(sph.dof(op), dtype=torch.float64, device="cuda")
    u = torch.empty_like(x)
    for _ in range(warmup):
        sph.apply(op | stage, x, u, precision=precision)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for e0, e1 in ev:
        e0.record()
        sph.apply(op | stage, x, u, precision=precision)
        e1.record()
    torch.cuda.synchronize()
    ms = np.array([e0.elapsed_time(e1) for e0, e1 in ev])
    return float(np.median(ms)) / 1e3, float(ms.mean()) / 1e3


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=4)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="spheres2048_p12_slip")
    ap.add_argument("--precond", choices=["m0", "mlp", "m0r", "mlpr"], default=None,
                    help="default: mlp (M0 + the learned correction) on the 2048-sphere slip workload, m0 elsewhere; "
                         "m0r / mlpr: with the rigid-mode coarse correction (resistance workloads)")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true", help="skip the float64 reference solves")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a 1 GiB device-to-device copy (HBM byte-counter calibration under rocprofv3 --pmc)")
    args = ap.parse_args()
    if args.precond is None:
        args.precond = "mlp" if args.workload == "spheres2048_p12_slip" else "m0"
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (the far field would shard "
              "by target spheres with one all-gather of the source strengths per matvec)",
              file=sys.stderr)
        sys.exit(2)

    cpu = small = None
    if not args.no_cpu and not args.calibrate_copy:
        # host work first, before anything initialises the GPU
        cpu = cpu_baseline(args.workload)
        log(f"CPU baseline: {cpu['value']:.3e} pairs/s on {cpu['cores']} processes")
        small = cpu_baseline_small_solve()
        log(f"oracle solve of {small['workload']}: {small['seconds']:.1f} s, {small['iters']} iterations")

    import torch

    if args.calibrate_copy:
        # a copy of known size: 1 GiB read + 1 GiB written per dispatch
        a = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"calibration_copy_bytes": 2 * a.numel() * 4, "dispatches": 3}))
        return

    from paper_1707_06551_amd import bie
    from paper_1707_06551_amd.inputs import make_workload, slip_field
    from paper_1707_06551_amd.precond_train import load_weights

    n_seeds = N_SEEDS.get(args.workload, 1)
    ws = [make_workload(args.workload, seed=s) for s in range(n_seeds)]
    w0 = ws[0]
    p = w0["p"]
    mobility = w0["problem"].startswith("mobility")
    pc = {"m0": bie.PC_M0, "mlp": bie.PC_MLP, "m0r": bie.PC_M0 | bie.PC_RIGID,
          "mlpr": bie.PC_MLP | bie.PC_RIGID}[args.precond]
    if (pc & bie.PC_RIGID) and mobility:
        ap.error("the rigid-mode correction acts on the resistance form")
    weights = None
    if pc & bie.PC_MLP:
        weights, meta = load_weights(os.path.join(ROOT, "paper_1707_06551_amd", "weights",
                                                  "precond_dn_rigid.npz" if pc & bie.PC_RIGID else
                                                  MLP_WEIGHTS["mobility" if mobility else "resistance"]))
        if meta.get("composition") == "local":
            pc |= bie.PC_LOCAL
    ctx, slips, t_setup = [], [], []
    for w in ws:
        t0 = time.perf_counter()
        s = bie.Spheres(w["centres"], p)
        if weights is not None:
            s.load_precond(weights)
        slip = None
        if w["problem"] == "mobility_slip":
            xyz, _ = s.nodes()
            sphere_of = np.arange(s.N) // s.P
            slip = torch.from_numpy(slip_field(w["slip_coef"], xyz - w["centres"][sphere_of], sphere_of)
                                    .reshape(-1)).cuda()
        torch.cuda.synchronize()
        t_setup.append(time.perf_counter() - t0)
        ctx.append(s)
        slips.append(slip)
        log(f"context seed {w['seed']}: {s.nb} spheres, {s.N} nodes, d* {s.near_gap:.4g}, "
            f"{s.n_near} near pairs, set-up {t_setup[-1]:.2f} s")
    s0 = ctx[0]
    n_near = s0.near_pairs().shape[1]

    def solve(k, precision, precond, max_iter=1000, x0=None):
        s, w = ctx[k], ws[k]
        if mobility:
            v, om, mu, info = s.solve_mobility(w["F"], w["T"], slip=slips[k], tol=w["tol"], precision=precision,
                                               precond=precond, max_iter=max_iter, x0=x0, want_mu=True)
            x = torch.cat([mu, torch.from_numpy(np.concatenate([v.reshape(-1), om.reshape(-1)])).to(mu.device)])
        else:
            _F, _T, x, info = s.solve_resistance(w["v"], w["omega"], tol=w["tol"], precision=precision,
                                                 precond=precond, max_iter=max_iter, x0=x0, want_psi=True)
        return info, x

    def solve_chunked(k, precision, precond, chunk=100, max_iter=3000):
        """A solve in pieces of `chunk` iterations, each resumed from the last iterate
        (the GMRES restart length is 100, so the pieces are the solver's own restart
        cycles), with a progress line per piece; the statistics are summed."""
        tot, x = None, None
        while True:
            info, x = solve(k, precision, precond, max_iter=chunk, x0=x)
            if tot is None:
                tot = dict(info)
            else:
                for key in ("iters", "outer_steps", "matvecs_fp64", "matvecs_mixed", "seconds"):
                    tot[key] += info[key]
                tot["rel_residual"], tot["converged"] = info["rel_residual"], info["converged"]
            log(f"  seed {k} precision {precision} precond {precond}: {tot['iters']} iterations, "
                f"residual {info['rel_residual']:.2e}, {tot['seconds']:.1f} s")
            if info["converged"] or tot["iters"] >= max_iter:
                return tot

    for i in range(args.warmup):
        info, _x = solve(i % n_seeds, bie.MIXED, pc)
        log(f"warm-up solve seed {i % n_seeds}: {info['iters']} iterations, {info['seconds']:.2f} s")
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        infos.append(solve(i % n_seeds, bie.MIXED, pc)[0])
        log(f"step {i}: seed {i % n_seeds}, {infos[-1]['iters']} iterations, {infos[-1]['seconds']:.2f} s")
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    assert all(i["converged"] for i in infos), [i["rel_residual"] for i in infos]
    pairs = sum(i["pairs_evaluated"] for i in infos)
    value = pairs / elapsed
    tts = elapsed / args.steps
    stage_s = {k: sum(i["t_stage_s"][k] for i in infos) / args.steps for k in bie.STAGE_NAMES}

    ref64 = ref64pc = None
    if not args.no_fp64:
        ref64 = solve_chunked(0, bie.FP64, bie.PC_NONE)
        ref64pc = solve_chunked(0, bie.FP64, pc)
    mixed0 = infos[0] if args.steps > 0 else solve(0, bie.MIXED, pc)[0]

    op = bie.OP_MOBILITY if mobility else bie.OP_DN_BIE
    kind = "SD" if mobility else "D"
    t_far32, t_far32_mean = time_stage(s0, torch, bie, op, bie.STAGE_FAR, bie.MIXED)
    t_far64, t_far64_mean = time_stage(s0, torch, bie, op, bie.STAGE_FAR, bie.FP64)
    t_near, t_near_mean = time_stage(s0, torch, bie, op, bie.STAGE_NEAR, bie.FP64)
    log(f"stage timing: far float32 {t_far32 * 1e3:.2f} ms, far float64 {t_far64 * 1e3:.2f} ms, "
        f"near {t_near * 1e3:.2f} ms")
    pairs_mv = s0.far_node_pairs
    ach32 = pairs_mv * FLOP_PER_PAIR[kind] / t_far32 / 1e12
    ach64 = pairs_mv * FLOP_PER_PAIR[kind] / t_far64 / 1e12
    traffic, counted = measured_counters(args.workload)

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "pair-interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": tts * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": w0["name"], "n_spheres": w0["n"], "p": p, "nodes": s0.N, "seeds": n_seeds,
                   "problem": w0["problem"], "tol": w0["tol"],
                   "precision": "mixed (f32 P2P/SHT, f64 near+GMRES)",
                   "precond": {"m0": "M0 (isolated-sphere inverse)", "mlp": "M0 + learned close-pair correction",
                               "m0r": "M0 + rigid-mode coarse correction",
                               "mlpr": "M0 + rigid-mode + learned corrections"}[args.precond],
                   "volume_fraction": w0.get("phi"), "min_gap": w0["min_gap"],
                   "near_gap": s0.near_gap, "near_tol": s0.near_tol, "near_pairs_seed0": n_near},
        "time_to_solution_s": tts,
        "time_to_solution_per_step_s": [i["seconds"] for i in infos],
        "iters_per_step": [i["iters"] for i in infos],
        "outer_steps_per_step": [i["outer_steps"] for i in infos],
        "rel_residual_max": max(i["rel_residual"] for i in infos),
        "matvecs_per_step": [[i["matvecs_fp64"], i["matvecs_mixed"]] for i in infos],
        "stage_seconds_per_step": stage_s,
        "pairs_per_matvec_seed0": pairs_mv,
        "setup_s_per_context": float(np.mean(t_setup)),
        "roofline": {"bound": "alu", "kernel": f"far_kernel<float,{kind}> (float32 far-field pair sum)",
                     "achieved": ach32, "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                     "frac": ach32 / PEAK_FP32_VECTOR_TFLOPS, "traffic": traffic,
                     "traffic_unit": "bytes per launch (HBM, PMC FETCH_SIZE + WRITE_SIZE, calibrated)",
                     "flop_per_pair": FLOP_PER_PAIR[kind],
                     "counted_flop_per_pair": counted,
                     "frac_counted": (None if counted is None else
                                      pairs_mv * counted / t_far32 / 1e12 / PEAK_FP32_VECTOR_TFLOPS),
                     "launch_ms": t_far32 * 1e3, "launch_ms_mean": t_far32_mean * 1e3,
                     "timing": "median of 20 event-timed far-field passes after 3 warm-up passes, seed 0",
                     "pairs_per_launch": pairs_mv},
        "far_fp64": {"achieved_tflops": ach64, "peak": PEAK_FP64_VECTOR_TFLOPS, "frac": ach64 / PEAK_FP64_VECTOR_TFLOPS,
                     "launch_ms": t_far64 * 1e3, "launch_ms_mean": t_far64_mean * 1e3,
                     "pairs_per_s": pairs_mv / t_far64},
        "far_fp32_pairs_per_s": pairs_mv / t_far32,
        "near_stage": {"ms": t_near * 1e3, "ms_mean": t_near_mean * 1e3, "directed_pairs": n_near,
                       "evals_per_s": n_near * s0.P / t_near},
    }
    # time-to-solution against its roofline: the far-field flop of every matvec of a
    # solve at the vector peak of its precision
    flop_mv = pairs_mv * FLOP_PER_PAIR[kind]
    ideal = (mixed0["matvecs_mixed"] * flop_mv / (PEAK_FP32_VECTOR_TFLOPS * 1e12)
             + mixed0["matvecs_fp64"] * flop_mv / (PEAK_FP64_VECTOR_TFLOPS * 1e12))
    out["time_to_solution_roofline"] = {
        "seed": 0, "ideal_s": ideal, "measured_s": mixed0["seconds"], "frac": ideal / mixed0["seconds"],
        "model": f"far-field flop ({FLOP_PER_PAIR[kind]} per pair) of each matvec at the float32 "
                 f"({PEAK_FP32_VECTOR_TFLOPS}) or float64 ({PEAK_FP64_VECTOR_TFLOPS} TFLOP/s) vector peak"}
    if ref64 is not None:
        out["fp64_plain"] = {"seed": 0, "seconds": ref64["seconds"], "iters": ref64["iters"],
                             "converged": ref64["converged"], "rel_residual": ref64["rel_residual"],
                             "roofline_frac": ref64["matvecs_fp64"] * flop_mv / (PEAK_FP64_VECTOR_TFLOPS * 1e12)
                             / ref64["seconds"]}
        out["fp64_precond"] = {"seed": 0, "seconds": ref64pc["seconds"], "iters": ref64pc["iters"],
                               "converged": ref64pc["converged"], "rel_residual": ref64pc["rel_residual"]}
        out["speedup_vs_fp64_plain"] = ref64["seconds"] / mixed0["seconds"]
        out["speedup_mixed_vs_fp64_same_precond"] = ref64pc["seconds"] / mixed0["seconds"]
        out["speedup_precond_vs_none_fp64"] = ref64["seconds"] / ref64pc["seconds"]
    if cpu is not None:
        out["cpu_baseline"] = cpu
        # the 8-sphere workload solved by the oracle and by the library, same d* and tolerance
        w1 = make_workload("spheres8_p8")
        s1 = bie.Spheres(w1["centres"], w1["p"], near_gap=small["near_gap"])
        F1, T1, _p, i1 = s1.solve_resistance(w1["v"], w1["omega"], tol=w1["tol"])
        s1.close()
        out["small_solve"] = {"workload": small["workload"], "oracle_s": small["seconds"],
                              "oracle_iters": small["iters"], "gpu_s": i1["seconds"], "gpu_iters": i1["iters"],
                              "near_gap": small["near_gap"],
                              "max_rel_diff_F_T": float(max(np.abs(F1 - small["F"]).max() / np.abs(small["F"]).max(),
                                                            np.abs(T1 - small["T"]).max() / np.abs(small["T"]).max()))}
    for s in ctx:
        s.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
