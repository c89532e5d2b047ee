"""Benchmark: P2P pair-interactions/s and time-to-solution of the sphere Stokes BIE.

One step = one mobility solve (bordered second-kind S+D equation, Problem 4 with the
applied force/torque rows) on 512 unit spheres, p = 12 (159,744 nodes), volume fraction
0.10, min gap 0.2, to relative residual 1e-8, with float32 transforms and far-field
sums inside float64 GMRES with iterative refinement and the isolated-sphere block
preconditioner.  Inputs (geometry, forces, torques) are resident on the device before
the timed region.  value = far-field pair interactions evaluated / wall time.

Reported beside it: the time-to-solution of plain float64 GMRES (no preconditioner) on
the same GPU, the roofline of the dominant kernel (float32 far-field pair sum, timed
live with HIP events on the library's stream), the time-to-solution as a fraction of its
own roofline (every matvec's far-field flop at the vector peak of its precision), and
the CPU oracle's pair rate on a bounded sample of the same workload.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]
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


def measured_traffic():
    """HBM bytes per launch of the far-field kernel from the committed PMC summary, or
    None when the kernel's code has changed since the counters were taken."""
    src = os.path.join(ROOT, "paper_1707_06551_amd", "csrc", "p2p.hip")
    prof = os.path.join(ROOT, "profiles", "far_kernel_spheres512_p12_pmc.md")
    try:
        sha = code_sha(src)
        fields = dict(l.split(": ", 1) for l in open(prof).read().splitlines() if ": " in l and l[:1].isalpha())
        if fields.get("source_sha256_16", "").strip() == sha:
            return float(fields["traffic_bytes_per_launch"])
    except (OSError, KeyError, ValueError):
        pass
    return None


def far_pairs(sph):
    """Pairs of nodes on distinct, well-separated spheres evaluated by one far-field pass."""
    near = sph.near_pairs().shape[1]
    return (sph.nb * (sph.nb - 1) - near) * sph.P * sph.P


def time_far_stage(sph, torch, bie, precision, reps=20, warmup=3):
    """Median and mean duration (s) of one far-field pass (S+D: the pair-sum kernel and
    the reduction of its split partial sums), each pass bracketed by its own events on
    the stream the library launches on (torch's current stream, passed at context
    creation); `warmup` untimed passes first."""
    x = torch.randn(3 * sph.N, dtype=torch.float64, device="cuda")
    u = torch.empty_like(x)
    op = bie.OP_SD_BIE | bie.STAGE_FAR
    for _ in range(warmup):
        sph.apply(op, x, u, precision=precision)
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
    for e0, e1 in ev:
        e0.record()
        sph.apply(op, x, u, precision=precision)
        e1.record()
    torch.cuda.synchronize()
    ms = np.array([e0.elapsed_time(e1) for e0, e1 in ev])
    return float(np.median(ms)) / 1e3, float(ms.mean()) / 1e3


def cpu_baseline(w, seconds_target=15.0):
    """The oracle's far-field direct sum on a bounded sample of target nodes (all
    sources), timed on the host; rate in pair-interactions/s."""
    from threadpoolctl import threadpool_limits

    from oracle.grid import Geometry
    from oracle.operators import Operators
    g = Geometry(w["centres"], w["p"], near_gap=1.0)
    ops = Operators(g)
    rng = np.random.default_rng(5)
    mu = rng.standard_normal((g.N, 3))
    allowed_per_t = g.nb - 1 - g.near.sum(axis=1)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        nt = 0
        pairs = 0
        while time.perf_counter() - t0 < seconds_target:
            tg = rng.choice(g.N, 32, replace=False)
            ops.far_part(mu, 1.0, 1.0, targets=tg)
            nt += tg.size
            pairs += int(allowed_per_t[g.sphere_of[tg]].sum()) * g.P
        dt = time.perf_counter() - t0
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    return dict(value=pairs / dt, unit="pair-interactions/s", cores=1, kind="oracle",
                sample=f"far-field S+D direct sum for {nt} random target nodes x all sources of "
                       f"{w['name']} ({pairs:.3e} pairs, {dt:.1f} s, numpy float64, 1 thread)",
                host_cpus=os.cpu_count(), cpu_model=model)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="spheres512_p12")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true", help="skip the plain float64 reference solve")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a 1 GiB device-to-device copy (HBM byte-counter calibration under rocprofv3 --pmc)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (the far field would shard "
              "by target spheres with one all-gather of the source strengths per matvec)",
              file=sys.stderr)
        sys.exit(2)

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
    from paper_1707_06551_amd.inputs import make_workload

    w = make_workload(args.workload)
    p = w["p"]
    t_setup = time.perf_counter()
    sph = bie.Spheres(w["centres"], p, near_gap=1.0)
    t_setup = time.perf_counter() - t_setup
    pairs_per_mv = far_pairs(sph)
    mobility = w["problem"].startswith("mobility")

    def solve(precision, precond):
        if mobility:
            return sph.solve_mobility(w["F"], w["T"], tol=w["tol"], precision=precision, precond=precond)
        return sph.solve_resistance(w["v"], w["omega"], tol=w["tol"], precision=precision, precond=precond)

    for _ in range(args.warmup):
        solve(bie.MIXED, bie.PC_M0)
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    for _ in range(args.steps):
        infos.append(solve(bie.MIXED, bie.PC_M0)[-1])
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    n_mv = sum(i["matvecs_fp64"] + i["matvecs_mixed"] for i in infos)
    value = n_mv * pairs_per_mv / elapsed
    tts = elapsed / args.steps

    ref = None
    if not args.no_fp64:
        ref = solve(bie.FP64, bie.PC_NONE)[-1]

    t_far32, t_far32_mean = time_far_stage(sph, torch, bie, bie.MIXED)
    t_far64, t_far64_mean = time_far_stage(sph, torch, bie, bie.FP64)
    kind = "SD" if mobility else "D"
    ach32 = pairs_per_mv * FLOP_PER_PAIR[kind] / t_far32 / 1e12
    ach64 = pairs_per_mv * FLOP_PER_PAIR[kind] / t_far64 / 1e12

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
        "config": {"workload": w["name"], "n_spheres": w["n"], "p": p, "nodes": sph.N,
                   "problem": w["problem"], "tol": w["tol"], "precision": "mixed (f32 P2P/SHT, f64 near+GMRES)",
                   "precond": "M0 (isolated-sphere inverse)", "volume_fraction": w.get("phi"),
                   "min_gap": w["min_gap"], "near_gap": 1.0},
        "time_to_solution_s": tts,
        "iters": infos[-1]["iters"],
        "outer_steps": infos[-1]["outer_steps"],
        "rel_residual": infos[-1]["rel_residual"],
        "matvecs_per_solve": {"fp64": infos[-1]["matvecs_fp64"], "mixed": infos[-1]["matvecs_mixed"]},
        "pairs_per_matvec": pairs_per_mv,
        "setup_s": t_setup,
        "roofline": {"bound": "alu", "kernel": f"far_kernel<float,{kind}> (float32 far-field pair sum)",
                     "achieved": ach32, "peak": PEAK_FP32_VECTOR_TFLOPS, "unit": "TFLOP/s",
                     "frac": ach32 / PEAK_FP32_VECTOR_TFLOPS, "traffic": measured_traffic(),
                     "traffic_unit": "bytes per launch (HBM, PMC FETCH_SIZE + WRITE_SIZE, calibrated)",
                     "flop_per_pair": FLOP_PER_PAIR[kind], "launch_ms": t_far32 * 1e3,
                     "launch_ms_mean": t_far32_mean * 1e3,
                     "timing": "median of 20 event-timed far-field passes after 3 warm-up passes",
                     "pairs_per_launch": pairs_per_mv},
        "far_fp64": {"achieved_tflops": ach64, "peak": PEAK_FP64_VECTOR_TFLOPS, "frac": ach64 / PEAK_FP64_VECTOR_TFLOPS,
                     "launch_ms": t_far64 * 1e3, "launch_ms_mean": t_far64_mean * 1e3,
                     "pairs_per_s": pairs_per_mv / t_far64},
        "far_fp32_pairs_per_s": pairs_per_mv / t_far32,
    }
    # time-to-solution against its roofline: the far-field flop of every matvec of the
    # solve at the vector peak of the precision it runs in
    flop_mv = pairs_per_mv * FLOP_PER_PAIR[kind]
    ideal = (infos[-1]["matvecs_mixed"] * flop_mv / (PEAK_FP32_VECTOR_TFLOPS * 1e12)
             + infos[-1]["matvecs_fp64"] * flop_mv / (PEAK_FP64_VECTOR_TFLOPS * 1e12))
    out["time_to_solution_roofline"] = {
        "ideal_s": ideal, "frac": ideal / tts,
        "model": f"far-field flop ({FLOP_PER_PAIR[kind]} per pair) of each matvec at the float32 "
                 f"({PEAK_FP32_VECTOR_TFLOPS}) or float64 ({PEAK_FP64_VECTOR_TFLOPS} TFLOP/s) vector peak"}
    if ref is not None:
        out["time_to_solution_fp64_plain_s"] = ref["seconds"]
        out["fp64_plain_iters"] = ref["iters"]
        out["speedup_vs_fp64_plain"] = ref["seconds"] / tts
        ideal64 = ref["matvecs_fp64"] * flop_mv / (PEAK_FP64_VECTOR_TFLOPS * 1e12)
        out["time_to_solution_fp64_plain_roofline_frac"] = ideal64 / ref["seconds"]
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(w)
    sph.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
