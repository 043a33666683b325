#!/usr/bin/env python3
"""BlockBP message-update throughput on one MI355X.

Sections after the headline line (on by default unless noted): a batched
sweep of 64 independent blocks of uneven N, D, chi against sweeping them one
handle at a time; a serving run (Poisson stream of expectation requests on
resident states) with continuous batching against one request at a time;
and, with --precision-report, the FP32 / split-BF16 contraction error at
N=4, D=6, chi=64.

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
    ap.add_argument("--expect-reps", type=int, default=10)
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-sweep section")
    ap.add_argument("--batched-blocks", type=int, default=64)
    ap.add_argument("--no-serving", action="store_true", help="skip the serving section")
    ap.add_argument("--serving-states", type=int, default=8)
    ap.add_argument("--serving-requests", type=int, default=16)
    ap.add_argument("--serving-inflight", type=int, default=4)
    ap.add_argument("--precision-report", action="store_true",
                    help="add the FP32 / split-BF16 error report at N=4, D=6, chi=64")
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


def batched_section(args):
    """Independent blocks of uneven N, D, chi: one merged launch sequence (HIP
    graph) per sweep against sweeping every handle on its own."""
    import paper_2603_13304_amd as pn
    from paper_2603_13304_amd.binding import make_desc
    from synth import inputs as syn
    rng = np.random.default_rng(2026)
    cfgs = [(int(rng.integers(2, 6)), int(rng.choice([2, 3, 4])), int(rng.choice([8, 16, 32, 64])))
            for _ in range(args.batched_blocks)]
    nets = []
    for i, (N, D, chi) in enumerate(cfgs):
        ts = [t / np.linalg.norm(t) for t in syn.random_unit_cell(D, seed=100 + i)]
        desc = make_desc(pn.BBP_KAGOME_INF_HEX, D=D, chi=chi, hex_N=N, precision=1, trunc=1,
                         q=2, p=8, seed=7)
        nets.append(pn.PepsNet(desc, ts))
    b = pn.Batch(nets)
    b.use_graph(True)
    gf, nl = b.stats()
    b.sweep(1)                                   # warmup (captures the graph)
    t0 = time.perf_counter()
    _, dev_ms = b.sweep(1)
    wall_b = time.perf_counter() - t0
    print(f"[bench] batched: {len(nets)} blocks, {nl} launches per sweep, {wall_b:.2f} s",
          file=sys.stderr, flush=True)
    for g in nets:
        g.use_graph(True)
        g.blockbp_sweep(1, 0.0)                  # capture each handle's graph
    t0 = time.perf_counter()
    for g in nets:
        g.blockbp_sweep(1, 0.0)
    wall_s = time.perf_counter() - t0
    print(f"[bench] per-block: {wall_s:.2f} s", file=sys.stderr, flush=True)
    upd = 6 * len(nets)
    b.close()
    for g in nets:
        g.close()
    return {"workload": f"{len(nets)} infinite-kagome blocks, N in 2..5, D in 2..4, chi in "
                        "8..64 (seeded), unit-norm random tensors, randomized truncation "
                        "(q=2, p=8), fp32 contraction GEMMs",
            "updates_per_sweep": upd, "launches_per_sweep": int(nl), "gemm_flop_per_sweep": gf,
            "batched_msg_updates_per_s": upd / wall_b, "batched_device_ms": dev_ms,
            "per_block_msg_updates_per_s": upd / wall_s,
            "speedup": wall_s / wall_b}


def serving_section(args):
    """Poisson stream of expectation requests on resident states (each an
    imaginary-time-step perturbation of its state, messages warm-started),
    continuous batching vs one request at a time on the same stream."""
    import paper_2603_13304_amd as pn
    from paper_2603_13304_amd.binding import make_desc
    from synth import inputs as syn
    rng = np.random.default_rng(5)
    states = []
    for i in range(args.serving_states):
        D, chi = int(rng.choice([3, 4, 5])), int(rng.choice([16, 32, 64]))
        ts = [t / np.linalg.norm(t) for t in syn.random_unit_cell(D, seed=300 + i)]
        desc = make_desc(pn.BBP_KAGOME_INF_HEX, D=D, chi=chi, hex_N=3, precision=1, trunc=1,
                         q=2, p=8, seed=7)
        g = pn.PepsNet(desc, ts)
        g.blockbp_sweep(2, 0.0)                  # resident, partly converged messages
        g.release_workspace()
        states.append((g, ts))
    ws = [g.memory()[1] for g, _ in states]
    res_bytes = sum(g.memory()[0] for g, _ in states)
    budget = int(64e9)
    arrivals = np.cumsum(rng.exponential(1.0 / 200.0, size=args.serving_requests))
    reqs = []
    for k in range(args.serving_requests):
        si = int(rng.integers(0, len(states)))
        g, ts = states[si]
        prng = np.random.default_rng(1000 + k)
        new = [t + 1e-3 * (prng.standard_normal(t.shape) + 1j * prng.standard_normal(t.shape))
               for t in ts]
        reqs.append((arrivals[k], g, new))

    def run(inflight):
        srv = pn.Server(budget, inflight)
        t0 = time.perf_counter()
        tickets = []
        for at, g, new in reqs:
            now = time.perf_counter() - t0
            if at > now:
                time.sleep(at - now)
            tickets.append(srv.submit(g, new, tol=1e-5, max_sweeps=3))
        lat = [srv.poll(t)["latency_s"] for t in tickets]
        wall = time.perf_counter() - t0
        st = srv.stats()
        srv.close()
        return np.array(lat), wall, st

    lat_b, wall_b, st_b = run(args.serving_inflight)
    print(f"[bench] serving: {len(reqs)} requests, continuous batching {wall_b:.2f} s",
          file=sys.stderr, flush=True)
    lat_s, wall_s, st_s = run(1)
    print(f"[bench] serving: one at a time {wall_s:.2f} s", file=sys.stderr, flush=True)
    for g, _ in states:
        g.close()
    n = len(reqs)
    return {"workload": f"{len(states)} resident infinite-kagome states (N=3, D in 3..5, chi in "
                        "16..64, fp32 contraction GEMMs, randomized truncation), Poisson arrivals "
                        f"at 200 req/s, {n} requests, each an ITE-step perturbation + warm-started "
                        "sweeps to 1e-5 (at most 3) + expectation",
            "hbm_budget_bytes": budget, "resident_bytes": int(res_bytes),
            "max_workspace_bytes": int(max(ws)), "peak_workspace_bytes": int(st_b["peak_bytes"]),
            "max_inflight": args.serving_inflight, "peak_inflight": int(st_b["peak_inflight"]),
            "throughput_req_per_s": n / wall_b,
            "latency_p50_s": float(np.percentile(lat_b, 50)),
            "latency_p99_s": float(np.percentile(lat_b, 99)),
            "one_at_a_time": {"throughput_req_per_s": n / wall_s,
                              "latency_p50_s": float(np.percentile(lat_s, 50)),
                              "latency_p99_s": float(np.percentile(lat_s, 99))}}


def precision_section():
    """FP32 and split-BF16 contraction against the FP64 path at N=4, D=6,
    chi=64 (randomized truncation): the same input messages (FP64 after two
    sweeps) go through one sweep and the expectation in each precision."""
    import paper_2603_13304_amd as pn
    from paper_2603_13304_amd.binding import make_desc
    from synth import inputs as syn
    ts = syn.simple_update_cell(6, seed=2, steps=20, dtau=0.05)
    nets = {}
    for prec in (0, 1, 2):
        desc = make_desc(pn.BBP_KAGOME_INF_HEX, D=6, chi=64, hex_N=4, precision=prec, trunc=1,
                         q=2, p=8, seed=7)
        nets[prec] = pn.PepsNet(desc, ts)
    nets[0].blockbp_sweep(2, 0.0)
    start = nets[0].get_messages()
    out = {}
    for prec in (0, 1, 2):
        g = nets[prec]
        if prec:
            g.set_messages(start)
        t0 = time.perf_counter()
        _, err, _ = g.blockbp_sweep(1, 0.0)
        dt = time.perf_counter() - t0
        _, ss, e = g.blockbp_expect()
        out[prec] = (g.get_messages(), np.array(ss), e, err, dt)
        print(f"[bench] precision {prec}: sweep {dt:.2f} s, E {e:.12f}", file=sys.stderr, flush=True)
    rep = {"workload": "infinite kagome, hexagonal block N=4 (111 sites), D=6, chi=64, "
                       "simple-update tensors, randomized truncation (q=2, p=8); one sweep and "
                       "the expectation from the same FP64 messages"}
    for prec, name in ((1, "fp32"), (2, "bf16x3")):
        m0, ss0, e0, err0, _ = out[0]
        m1, ss1, e1, err1, dt = out[prec]
        rep[name] = {"abs_dE_per_site": abs(e1 - e0), "max_abs_d_bond_ss": float(np.abs(ss1 - ss0).max()),
 "abs_d_convergence_distance": abs(err1 - err0),
                     "sweep_s": dt}
    rep["fp64_sweep_s"] = out[0][4]
    for g in nets.values():
        g.close()
    return rep


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
    elif name in ("qr", "qr_tall", "jacobi", "svd_bidiag", "svd_top"):
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
    g.close()
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(ts, args)
    if not args.no_batched:
        out["batched"] = batched_section(args)
    if not args.no_serving:
        out["serving"] = serving_section(args)
    if args.precision_report:
        out["precision_report"] = precision_section()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
