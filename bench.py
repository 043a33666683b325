#!/usr/bin/env python3
"""BlockBP message-update throughput on one MI355X.

Workload (the paper's infinite-kagome setting at its benchmark size): a
hexagonal block of face length N=3 (57 sites) of the infinite kagome PEPS,
D=3, chi=16, site tensors from 20 second-order simple-update imaginary-time
steps (dtau=0.05, Heisenberg J=1, seed 2), messages from identity.  One step
is one Jacobi sweep: all six message updates of the block (boundary-chain
contraction, QR/truncated SVD, normalisation) plus the convergence distance.

Prints one JSON line: message updates per second over the timed sweeps, the
dominant kernel's roofline figures (timed live with HIP events on the
library's stream), expectation-value latency (p50/p99 of blockbp_expect once
converged to 1e-5), and the FP64 oracle timed on the host cores on a bounded
sample.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAKS = {  # MI355X published peaks
    "hbm_GBs": 8000.0,
    "fp64_tflops": 78.6,
    "fp32_tflops": 157.3,
    "bf16_tflops": 2500.0,
}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--trunc", choices=["T1", "T2"], default="T1")
    ap.add_argument("--precision", choices=["fp64", "fp32", "bf16x3"], default="fp32")
    ap.add_argument("--N", type=int, default=3)
    ap.add_argument("--D", type=int, default=3)
    ap.add_argument("--chi", type=int, default=16)
    ap.add_argument("--q", type=int, default=2)
    ap.add_argument("--p", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--profile-sweeps", type=int, default=3)
    ap.add_argument("--expect-reps", type=int, default=20)
    return ap.parse_args()


def cpu_baseline(ts, args):
    """The FP64 oracle, as it stands, on a bounded sample of the same
    workload: identity start, sweeps until ~10 s of work (at least one)."""
    from oracle import geometry as geo
    from oracle.blockbp import BlockBP
    try:
        from threadpoolctl import threadpool_info
        cores = max([x.get("num_threads", 1) for x in threadpool_info()] or [1])
    except Exception:
        cores = os.cpu_count() or 1
    P = geo.HexProblem(args.N)
    O = BlockBP(P, ts, chi=args.chi, chi_env=args.chi, trunc=args.trunc, q=args.q, p=args.p,
                seed=7)
    n, t0 = 0, time.perf_counter()
    while True:
        O.sweep()
        n += 1
        if time.perf_counter() - t0 > 10.0 or n >= 5:
            break
    dt = time.perf_counter() - t0
    upd = n * len(P.msg_keys)
    return {"value": upd / dt, "unit": "msg_updates/s", "cores": int(cores), "kind": "oracle",
            "sample": f"{n} sweeps ({upd} message updates) of the same workload from identity "
                      f"messages, {args.trunc} truncation, numpy FP64, {dt:.1f} s"}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU; --gpus {args.gpus} is not supported "
              "(the sweep would shard its six message updates over GPUs with one all-gather "
              "per sweep; not built)", file=sys.stderr)
        sys.exit(2)
    import paper_2603_13304_amd as pn
    from paper_2603_13304_amd.binding import make_desc, profile_sweeps
    from synth import inputs as syn

    prec = {"fp64": 0, "fp32": 1, "bf16x3": 2}[args.precision]
    trunc = 1 if args.trunc == "T2" else 0
    ts = syn.simple_update_cell(args.D, seed=2, steps=20, dtau=0.05)
    desc = make_desc(pn.BBP_KAGOME_INF_HEX, D=args.D, chi=args.chi, hex_N=args.N,
                     precision=prec, trunc=trunc, q=args.q, p=args.p, seed=7)
    g = pn.PepsNet(desc, ts)
    g.use_graph(not args.no_graph)
    n_msg = g.num_messages()
    print(f"[bench] created N={args.N} D={args.D} chi={args.chi} {args.trunc} {args.precision}",
          file=sys.stderr, flush=True)

    # warmup sweeps (messages reach full bond dimension, graph gets captured)
    g.blockbp_sweep(args.warmup, 0.0)
    print(f"[bench] warmup {args.warmup} sweeps done", file=sys.stderr, flush=True)
    # timed region: exactly K sweeps
    import ctypes
    lib = g.lib
    g.timing(reset=True)
    t0 = time.perf_counter()
    done, err, _ = g.blockbp_sweep(args.steps, 0.0)
    t1 = time.perf_counter()
    assert done == args.steps
    dev_ms, _ = g.timing(reset=True)
    wall = t1 - t0
    ms_per_step = 1e3 * wall / args.steps
    value = n_msg * args.steps / wall
    print(f"[bench] timed {args.steps} sweeps: {ms_per_step:.3f} ms/sweep, {value:.1f} updates/s",
          file=sys.stderr, flush=True)

    # per-kernel live timing (HIP events on the library's stream)
    prof = profile_sweeps(g, args.profile_sweeps)
    dom = max(prof.items(), key=lambda kv: kv[1][0])
    name, (kms, nl, kfl, kby) = dom
    avg_s = kms / nl / 1e3
    if name.startswith("gemm"):
        bound, unit = "mfma", "TFLOP/s"
        peak = {"gemm_fp64": PEAKS["fp64_tflops"], "gemm_fp32": PEAKS["fp32_tflops"],
                "gemm_bf16x3": PEAKS["bf16_tflops"]}[name]
        achieved = kfl / nl / avg_s / 1e12
    elif name in ("qr", "jacobi"):
        bound, unit, peak = "alu", "TFLOP/s", PEAKS["fp64_tflops"]
        achieved = kfl / nl / avg_s / 1e12
    else:
        bound, unit, peak = "hbm", "GB/s", PEAKS["hbm_GBs"]
        achieved = kby / nl / avg_s / 1e9
    total_ms = sum(v[0] for v in prof.values()) / args.profile_sweeps
    breakdown = {k: {"ms_per_sweep": round(v[0] / args.profile_sweeps, 4),
                     "launches_per_sweep": v[1] // args.profile_sweeps,
                     "avg_us": round(1e3 * v[0] / v[1], 3)} for k, v in sorted(prof.items())}
    cf, gf, nlaunch = g.sweep_stats()

    # expectation latency once converged to 1e-5
    g.blockbp_sweep(60, 1e-5)
    lat = []
    for _ in range(args.expect_reps):
        t = time.perf_counter()
        _, ss, e = g.blockbp_expect()
        lat.append(1e3 * (time.perf_counter() - t))
    lat = np.array(lat)

    out = {
        "metric": "block msg updates/s + % MFMA peak; p50/p99 expect-value latency at 1e-5",
        "value": round(value, 3),
        "unit": "msg_updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "c128", "fp32": "c64+f64", "bf16x3": "bf16x3+f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"infinite kagome BlockBP, hexagonal block N={args.N} "
                               f"({3 * (3 * args.N ** 2 - 3 * args.N + 1)} sites), D={args.D}, "
                               f"chi={args.chi}, simple-update tensors (20 steps, dtau=0.05), "
                               f"{args.trunc} truncation (q={args.q}, p={args.p}), "
                               f"{args.precision} contraction GEMMs, FP64 QR/SVD",
                   "message_updates_per_step": n_msg, "graph": not args.no_graph},
        "roofline": {"bound": bound, "kernel": name, "achieved": round(achieved, 6),
                     "peak": peak, "unit": unit, "frac": achieved / peak, "traffic": None,
                     "avg_launch_us": round(avg_s * 1e6, 3)},
        "expect_latency_ms": {"p50": float(np.percentile(lat, 50)),
                              "p99": float(np.percentile(lat, 99)),
                              "energy_per_site": e, "bonds": len(ss)},
        "sweep": {"device_ms": round(dev_ms, 4), "launches": int(nlaunch),
                  "contraction_gflop": cf / 1e9, "gemm_gflop": gf / 1e9,
                  "profiled_kernel_ms": round(total_ms, 4), "kernels": breakdown},
    }
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(ts, args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
