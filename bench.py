#!/usr/bin/env python3
"""BlockBP message-update throughput on one MI355X.

Headline workload (the largest single-GPU configuration): the infinite
kagome lattice, hexagonal block of face length N=4 (111 sites), D=6, chi=64,
site tensors from 20 second-order simple-update imaginary-time steps
(dtau=0.05, Heisenberg J=1, seed 2), randomized truncation (Halko,
Martinsson & Tropp 2011, Alg. 4.4; q=2, p=8), contraction GEMMs in FP64
(complex128, the oracle's arithmetic), QR / SVD / normalisation FP64.
Messages start from identity; the warmup sweeps bring them to full bond
dimension.  One step is one Jacobi sweep: all six message updates of the
block plus the convergence distance.

Printed as one JSON line: message updates per second over the timed sweeps;
the dominant kernel's roofline figures (timed live with HIP events on the
library's stream) and the contraction GEMMs' fraction of the FP64 MFMA
peak; expectation-value latency (p50/p99 of blockbp_expect once the sweep
has converged or stalled, with the distance reached); the same workload with
FP32 and split-BF16 contraction GEMMs (throughput and |dE/site| against
FP64); the FP64 oracle timed on the host cores on one message update; and
the sections after it (N=3, D=3, chi=16 with exact truncation; a batched
sweep of 64 independent blocks; the serving loop).
"""
import argparse
import hashlib
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
PREC = {"fp64": 0, "fp32": 1, "bf16x3": 2}
DTYPE = {"fp64": "c128", "fp32": "c64+f64", "bf16x3": "bf16x3+f64"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--trunc", choices=["T1", "T2"], default="T2")
    ap.add_argument("--precision", choices=list(PREC), default="fp64")
    ap.add_argument("--N", type=int, default=4)
    ap.add_argument("--D", type=int, default=6)
    ap.add_argument("--chi", type=int, default=64)
    ap.add_argument("--q", type=int, default=2)
    ap.add_argument("--p", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true")
    ap.add_argument("--profile-sweeps", type=int, default=2)
    ap.add_argument("--expect-reps", type=int, default=5)
    ap.add_argument("--converge-sweeps", type=int, default=20,
                    help="sweeps toward 1e-5 before the expectation latency")
    ap.add_argument("--no-precisions", action="store_true",
                    help="skip the FP32 / split-BF16 runs of the headline workload")
    ap.add_argument("--no-small", action="store_true", help="skip the N=3, D=3, chi=16 section")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-sweep section")
    ap.add_argument("--batched-blocks", type=int, default=64)
    ap.add_argument("--no-serving", action="store_true", help="skip the serving section")
    ap.add_argument("--serving-states", type=int, default=32)
    ap.add_argument("--serving-requests", type=int, default=64)
    ap.add_argument("--serving-inflight", type=int, default=8)
    return ap.parse_args()


def workload_name(args, precision):
    nt = 3 * (3 * args.N ** 2 - 3 * args.N + 1)
    return (f"infinite kagome BlockBP, hexagonal block N={args.N} ({nt} sites), D={args.D}, "
            f"chi={args.chi}, simple-update tensors (20 steps, dtau=0.05, seed 2), "
            f"{args.trunc} truncation (q={args.q}, p={args.p}), {precision} contraction GEMMs, "
            "FP64 QR/SVD/normalisation, messages from identity")


def make_net(args, precision, ts):
    import paper_2603_13304_amd as pn
    from paper_2603_13304_amd.binding import make_desc
    desc = make_desc(pn.BBP_KAGOME_INF_HEX, D=args.D, chi=args.chi, hex_N=args.N,
                     precision=PREC[precision], trunc=1 if args.trunc == "T2" else 0,
                     q=args.q, p=args.p, seed=7)
    g = pn.PepsNet(desc, ts)
    g.use_graph(not args.no_graph)
    return g


def timed_sweeps(g, warmup, steps):
    g.blockbp_sweep(warmup, 0.0)
    g.timing(reset=True)
    t0 = time.perf_counter()
    done, err, _ = g.blockbp_sweep(steps, 0.0)
    wall = time.perf_counter() - t0
    assert done == steps
    dev_ms, _ = g.timing(reset=True)
    return wall, dev_ms, err


def traffic_record(kernel):
    """HBM bytes per launch of ``kernel`` from the committed rocprofv3 counter
    summary, or None when there is none or kernels.hip changed since."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    src = os.path.join(ROOT, "paper_2603_13304_amd", "csrc", "kernels.hip")
    with open(src, "rb") as f:
        if hashlib.sha256(f.read()).hexdigest() != rec.get("kernels_hip_sha256"):
            return None
    return rec.get("kernels", {}).get(kernel)


KERNEL_NAMES = {"gemm_fp64": "k_gemm", "gemm_fp32": "k_gemm", "gemm_bf16x3": "k_gemm",
                "chol": "k_chol", "jacobi": "k_jacobi", "qr": "k_qr", "qr_tall": "k_qr_tall",
                "svd_bidiag": "k_svt_bidiag", "svd_top": "k_svd_top", "norm": "k_norm_apply",
                "ksum": "k_sum_parts", "transpose": "k_permute", "pad": "k_pad",
                "split_gauge": "k_colphase", "sketch": "k_omega", "msg_phase": "k_phase"}


def roofline(prof, n_sweeps):
    """Dominant kernel of the profiled sweeps against its bound, and the
    contraction GEMMs' FP64/FP32/BF16 MFMA fractions."""
    name, (kms, nl, kfl, kby) = max(prof.items(), key=lambda kv: kv[1][0])
    avg_s = kms / nl / 1e3
    if name.startswith("gemm"):
        bound, unit = "mfma", "TFLOP/s"
        peak = {"gemm_fp64": PEAKS["fp64_tflops"], "gemm_fp32": PEAKS["fp32_tflops"],
                "gemm_bf16x3": PEAKS["bf16_tflops"]}[name]
        achieved = kfl / nl / avg_s / 1e12
    elif name in ("qr", "qr_tall", "jacobi", "svd_bidiag", "svd_top", "chol"):
        bound, unit, peak = "alu", "TFLOP/s", PEAKS["fp64_tflops"]
        achieved = kfl / nl / avg_s / 1e12
    else:
        bound, unit, peak = "hbm", "GB/s", PEAKS["hbm_GBs"]
        achieved = kby / nl / avg_s / 1e9
    tr = traffic_record(KERNEL_NAMES.get(name, name))
    out = {"bound": bound, "kernel": name, "achieved": round(achieved, 6), "peak": peak,
           "unit": unit, "frac": achieved / peak,
           "traffic": None if tr is None else tr["bytes_per_launch"],
           "avg_launch_us": round(avg_s * 1e6, 3), "ms_per_sweep": round(kms / n_sweeps, 3)}
    mfma = {}
    for k, pk in (("gemm_fp64", "fp64_tflops"), ("gemm_fp32", "fp32_tflops"),
                  ("gemm_bf16x3", "bf16_tflops")):
        if k in prof:
            ms, n, fl, _ = prof[k]
            tf = fl / (ms / 1e3) / 1e12
            mfma[k] = {"tflops": round(tf, 3), "frac_of_peak": tf / PEAKS[pk],
                       "ms_per_sweep": round(ms / n_sweeps, 3), "launches_per_sweep": n // n_sweeps}
    return out, mfma


def cpu_baseline(ts, args):
    """The FP64 oracle, as it stands, on one message update of the same
    workload (the first of a sweep's six) from seeded messages in the
    converged regime's shapes (every bond at its full dimension)."""
    from oracle import geometry as geo
    from oracle.blockbp import BlockBP
    from synth import inputs as syn
    try:
        from threadpoolctl import threadpool_info
        cores = max([x.get("num_threads", 1) for x in threadpool_info()] or [1])
    except Exception:
        cores = os.cpu_count() or 1
    P = geo.HexProblem(args.N)
    O = BlockBP(P, ts, chi=args.chi, chi_env=args.chi, trunc=args.trunc, q=args.q, p=args.p,
                seed=7)
    keys = list(range(6))
    shapes = [[x.shape for x in O.msgs[k]] for k in keys]
    for k, A in zip(keys, syn.random_messages(shapes, 41)):
        O.msgs[k] = A
    t0 = time.perf_counter()
    O.update(P.msg_keys[0])
    dt = time.perf_counter() - t0
    return {"value": 1.0 / dt, "unit": "msg_updates/s", "cores": int(cores), "kind": "oracle",
            "sample": f"1 message update (one of the 6 in a sweep) of the same workload from "
                      f"seeded full-rank messages, {args.trunc} truncation, numpy FP64, {dt:.1f} s"}


def precision_runs(args, ts, fp64_msgs, e_fp64, err_fp64):
    """The headline workload with FP32 and split-BF16 contraction GEMMs:
    throughput over timed sweeps, and the error of one sweep plus the
    expectation from the same FP64 messages against FP64."""
    out = {}
    for prec in ("fp32", "bf16x3"):
        g = make_net(args, prec, ts)
        wall, _, _ = timed_sweeps(g, 1, 3)
        g.set_messages(fp64_msgs)
        _, err, _ = g.blockbp_sweep(1, 0.0)
        _, ss, e = g.blockbp_expect()
        g.close()
        out[prec] = {"msg_updates_per_s": 6 * 3 / wall, "ms_per_sweep": 1e3 * wall / 3,
                     "abs_dE_per_site_vs_fp64": abs(e - e_fp64),
                     "abs_d_convergence_distance_vs_fp64": abs(err - err_fp64)}
        print(f"[bench] {prec}: {6 * 3 / wall:.2f} updates/s, |dE| {abs(e - e_fp64):.2e}",
              file=sys.stderr, flush=True)
    return out


def small_section(args):
    """N=3, D=3, chi=16 with exact truncated SVDs (T1), FP32 contraction: the
    round-trip-latency-bound end of the method."""
    from synth import inputs as syn
    a = argparse.Namespace(**vars(args))
    a.N, a.D, a.chi, a.trunc = 3, 3, 16, "T1"
    ts = syn.simple_update_cell(3, seed=2, steps=20, dtau=0.05)
    g = make_net(a, "fp32", ts)
    wall, dev_ms, _ = timed_sweeps(g, 5, 20)
    g.blockbp_sweep(40, 1e-5)
    lat = []
    for _ in range(5):
        t = time.perf_counter()
        g.blockbp_expect()
        lat.append(1e3 * (time.perf_counter() - t))
    g.close()
    return {"workload": workload_name(a, "fp32"), "msg_updates_per_s": 6 * 20 / wall,
            "ms_per_sweep": 1e3 * wall / 20, "expect_latency_ms_p50": float(np.median(lat))}


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


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py: this build measures one GPU; --gpus {args.gpus} is not supported "
              "(the sweep would shard its six message updates over GPUs with one all-gather "
              "per sweep; not built)", file=sys.stderr)
        sys.exit(2)
    from paper_2603_13304_amd.binding import profile_sweeps
    from synth import inputs as syn

    ts = syn.simple_update_cell(args.D, seed=2, steps=20, dtau=0.05)
    g = make_net(args, args.precision, ts)
    n_msg = g.num_messages()
    print(f"[bench] created N={args.N} D={args.D} chi={args.chi} {args.trunc} {args.precision}",
          file=sys.stderr, flush=True)
    # warmup sweeps (messages reach full bond dimension, graph captured),
    # then exactly K timed sweeps
    wall, dev_ms, err_timed = timed_sweeps(g, args.warmup, args.steps)
    ms_per_step = 1e3 * wall / args.steps
    value = n_msg * args.steps / wall
    print(f"[bench] timed {args.steps} sweeps: {ms_per_step:.2f} ms/sweep, {value:.3f} updates/s",
          file=sys.stderr, flush=True)
    # per-kernel live timing (HIP events on the library's stream)
    prof = profile_sweeps(g, args.profile_sweeps)
    roof, mfma = roofline(prof, args.profile_sweeps)
    breakdown = {k: {"ms_per_sweep": round(v[0] / args.profile_sweeps, 3),
                     "launches_per_sweep": v[1] // args.profile_sweeps,
                     "avg_us": round(1e3 * v[0] / v[1], 2)} for k, v in sorted(prof.items())}
    cf, gf, nlaunch = g.sweep_stats()
    # expectation latency once converged to 1e-5 (or after converge_sweeps)
    sw, err_c, _ = g.blockbp_sweep(args.converge_sweeps, 1e-5)
    msgs = g.get_messages()
    lat = []
    for _ in range(args.expect_reps):
        t = time.perf_counter()
        _, ss, e = g.blockbp_expect()
        lat.append(1e3 * (time.perf_counter() - t))
    _, err_next, _ = g.blockbp_sweep(1, 0.0)
    g.set_messages(msgs)
    g.close()
    out = {
        "metric": "block msg updates/s + % MFMA peak; p50/p99 expect-value latency at 1e-5",
        "value": round(value, 4),
        "unit": "msg_updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[args.precision],
        "data": "synthetic",
        "config": {"workload": workload_name(args, args.precision),
                   "message_updates_per_step": n_msg, "graph": not args.no_graph},
        "roofline": roof,
        "mfma": mfma,
        "expect_latency_ms": {"p50": float(np.percentile(lat, 50)),
                              "p99": float(np.percentile(lat, 99)),
                              "sweeps_before": sw, "distance_reached": err_c,
                              "tolerance_reached": bool(err_c <= 1e-5),
                              "energy_per_site": e, "bonds": len(ss)},
        "sweep": {"device_ms": round(dev_ms, 3), "launches": int(nlaunch),
                  "contraction_gflop": cf / 1e9, "gemm_gflop": gf / 1e9, "kernels": breakdown},
    }
    if not args.no_precisions and args.precision == "fp64":
        out["precisions"] = precision_runs(args, ts, msgs, e, err_next)
    if not args.no_cpu_baseline:
        print("[bench] timing the CPU oracle", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(ts, args)
        print(f"[bench] oracle: {out['cpu_baseline']['sample']}", file=sys.stderr, flush=True)
    if not args.no_small:
        out["small_block"] = small_section(args)
        print("[bench] small block done", file=sys.stderr, flush=True)
    if not args.no_batched:
        out["batched"] = batched_section(args)
    if not args.no_serving:
        out["serving"] = serving_section(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
