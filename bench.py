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
    ap.add_argument("--streams", type=int, default=4,
                    help="streams for the independent message updates of a sweep (1-4)")
    ap.add_argument("--no-autotune", action="store_true", help="keep the fixed GEMM tile rule")
    ap.add_argument("--tile-cache", default=None,
                    help="GEMM tile cache file (shapes found there are not timed again)")
    ap.add_argument("--profile-sweeps", type=int, default=2)
    ap.add_argument("--expect-reps", type=int, default=5)
    ap.add_argument("--converge-sweeps", type=int, default=8,
                    help="sweeps toward 1e-5 before the expectation latency (the randomized "
                         "split stops at a distance floor of about 3e-2 here)")
    ap.add_argument("--no-precisions", action="store_true",
                    help="skip the FP32 / split-BF16 runs of the headline workload")
    ap.add_argument("--no-small", action="store_true", help="skip the N=3, D=3, chi=16 section")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched-sweep section")
    ap.add_argument("--batched-blocks", type=int, default=64)
    ap.add_argument("--no-serving", action="store_true", help="skip the serving section")
    ap.add_argument("--serving-states", type=int, default=32)
    ap.add_argument("--serving-requests", type=int, default=48)
    ap.add_argument("--serving-inflight", type=int, default=8)
    ap.add_argument("--serving-max-sweeps", type=int, default=3)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (for the HBM counter scale)")
    ap.add_argument("--traffic-from", nargs=4, metavar=("FETCH", "WRITE", "COPY_FETCH", "COPY_WRITE"),
                    help="only summarise four rocprofv3 --pmc counter CSVs into "
                         "profiles/hbm_traffic.json and exit")
    ap.add_argument("--traffic-command", default="", help="commands recorded with --traffic-from")
    ap.add_argument("--copy-mib", type=int, default=256, help="size of the calibration copy")
    ap.add_argument("--traffic-out", default=os.path.join(ROOT, "profiles", "hbm_traffic.json"))
    ap.add_argument("--stats-summary", metavar="KERNEL_STATS_CSV",
                    help="only print a per-kernel table of a rocprofv3 --stats CSV and exit")
    ap.add_argument("--timeline-summary", nargs=4,
                    metavar=("KERNEL_TRACE_CSV", "LAUNCHES_PER_SWEEP", "TIMED", "TRAILING"),
                    help="only print how the kernels of the timed sweeps of a traced run overlap "
                         "(the trace ends with TIMED sweeps, then TRAILING others) and exit")
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
    g.use_streams(args.streams)
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
        if not args.no_autotune:
            g.autotune(args.tile_cache)
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
    round-trip-latency-bound end of the method, and the workload on which the
    sweeps reach 1e-5 (the expectation latency at that tolerance)."""
    from synth import inputs as syn
    a = argparse.Namespace(**vars(args))
    a.N, a.D, a.chi, a.trunc = 3, 3, 16, "T1"
    ts = syn.simple_update_cell(3, seed=2, steps=20, dtau=0.05)
    g = make_net(a, "fp32", ts)
    wall, dev_ms, _ = timed_sweeps(g, 5, 20)
    g.set_sites(ts, reset_messages=True)       # identity messages again
    sw, err, _ = g.blockbp_sweep(60, 1e-5)
    lat = []
    for _ in range(args.expect_reps * 4):
        t = time.perf_counter()
        _, ss, e = g.blockbp_expect()
        lat.append(1e3 * (time.perf_counter() - t))
    g.close()
    return {"workload": workload_name(a, "fp32"), "msg_updates_per_s": 6 * 20 / wall,
            "ms_per_sweep": 1e3 * wall / 20,
            "expect_latency_ms": {"p50": float(np.percentile(lat, 50)),
                                  "p99": float(np.percentile(lat, 99)), "reps": len(lat),
                                  "sweeps_from_identity": sw, "distance_reached": err,
                                  "tolerance_reached": bool(err <= 1e-5),
                                  "energy_per_site": e}}


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
    # tile shapes per GEMM shape, timed once per shape across the blocks
    import tempfile
    t0 = time.perf_counter()
    n_timed = 0
    with tempfile.TemporaryDirectory() as tmp:
        cache = os.path.join(tmp, "tiles.txt")
        for g in nets:
            n_timed += g.autotune(cache)[0]
    tune_s = time.perf_counter() - t0
    print(f"[bench] batched: autotuned {n_timed} GEMM shapes in {tune_s:.1f} s", file=sys.stderr,
          flush=True)
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
                        "(q=2, p=8), fp32 contraction GEMMs, autotuned GEMM tiles",
            "autotuned_gemm_shapes": n_timed, "autotune_seconds": tune_s,
            "updates_per_sweep": upd, "launches_per_sweep": int(nl), "gemm_flop_per_sweep": gf,
            "batched_msg_updates_per_s": upd / wall_b, "batched_device_ms": dev_ms,
            "per_block_msg_updates_per_s": upd / wall_s,
            "speedup": wall_s / wall_b}


def serving_section(args):
    """Poisson stream of expectation requests on resident states (each an
    imaginary-time-step perturbation of its state, messages warm-started),
    continuous batching against one request at a time.  Half the states are
    N=3, D=3, chi=16 with exact truncation (T1), on which sweeps converge to
    1e-5; the others draw D in 3..5, chi in 16..64 with the randomized split
    (q=2, p=8), whose sweeps stop at a distance floor of 1e-3..3e-2 (the
    sketch's truncation error) and therefore run max_sweeps.  Reported: how
    many requests reached the tolerance, latency over all requests and over
    those that reached it."""
    import paper_2603_13304_amd as pn
    from paper_2603_13304_amd.binding import make_desc
    from synth import inputs as syn
    rng = np.random.default_rng(5)
    others = [(3, 32), (3, 64), (4, 16), (4, 32), (4, 64), (5, 16), (5, 32), (5, 64)]
    tol, max_sweeps = 1e-5, args.serving_max_sweeps
    states = []
    for i in range(args.serving_states):
        if i % 2 == 0:
            D, chi, trunc = 3, 16, 0
        else:
            D, chi = others[int(rng.integers(0, len(others)))]
            trunc = 1
        ts = syn.simple_update_cell(D, seed=300 + i, steps=20, dtau=0.05)
        desc = make_desc(pn.BBP_KAGOME_INF_HEX, D=D, chi=chi, hex_N=3, precision=1, trunc=trunc,
                         q=2, p=8, seed=7)
        g = pn.PepsNet(desc, ts)
        # resident, warm messages: converged (T1) or at the sketch's floor (T2)
        g.blockbp_sweep(30 if trunc == 0 else 3, tol)
        g.release_workspace()
        states.append((g, ts, f"D{D}chi{chi}{'T1' if trunc == 0 else 'T2'}", trunc))
    print(f"[bench] serving: {len(states)} states resident", file=sys.stderr, flush=True)
    ws = [g.memory()[1] for g, _, _, _ in states]
    res_bytes = sum(g.memory()[0] for g, _, _, _ in states)
    budget = int(64e9)
    arrivals = np.cumsum(rng.exponential(1.0 / 200.0, size=args.serving_requests))
    reqs = []
    for k in range(args.serving_requests):
        si = int(rng.integers(0, len(states)))
        g, ts, cls, trunc = states[si]
        prng = np.random.default_rng(1000 + k)
        new = [t + 1e-3 * (prng.standard_normal(t.shape) + 1j * prng.standard_normal(t.shape))
               for t in ts]
        # exact-truncation states converge: enough sweeps to reach tol from
        # the warm start; randomized ones stop at their floor within a few
        reqs.append((arrivals[k], g, new, cls, 4 * max_sweeps if trunc == 0 else max_sweeps))

    def run(inflight):
        srv = pn.Server(budget, inflight)
        t0 = time.perf_counter()
        tickets = []
        for at, g, new, _, ms in reqs:
            now = time.perf_counter() - t0
            if at > now:
                time.sleep(at - now)
            tickets.append(srv.submit(g, new, tol=tol, max_sweeps=ms))
        res = [srv.poll(t) for t in tickets]
        wall = time.perf_counter() - t0
        st = srv.stats()
        srv.close()
        return res, wall, st

    def summary(res, wall):
        lat = np.array([r["latency_s"] for r in res])
        ok = np.array([r["err"] <= tol for r in res])
        out = {"throughput_req_per_s": len(res) / wall,
               "latency_p50_s": float(np.percentile(lat, 50)),
               "latency_p99_s": float(np.percentile(lat, 99)),
               "reached_tol": int(ok.sum())}
        if ok.any():
            out["reached_latency_p50_s"] = float(np.percentile(lat[ok], 50))
            out["reached_latency_p99_s"] = float(np.percentile(lat[ok], 99))
        return out

    res_b, wall_b, st_b = run(args.serving_inflight)
    print(f"[bench] serving: {len(reqs)} requests, continuous batching {wall_b:.2f} s",
          file=sys.stderr, flush=True)
    res_s, wall_s, _ = run(1)
    print(f"[bench] serving: one at a time {wall_s:.2f} s", file=sys.stderr, flush=True)
    for g, _, _, _ in states:
        g.close()
    n = len(reqs)
    by_cls = {}
    for (_, _, _, cls, _), r in zip(reqs, res_b):
        c = by_cls.setdefault(cls, {"requests": 0, "reached_tol": 0, "max_final_distance": 0.0})
        c["requests"] += 1
        c["reached_tol"] += int(r["err"] <= tol)
        c["max_final_distance"] = max(c["max_final_distance"], float(r["err"]))
    out = {"workload": f"{len(states)} resident infinite-kagome states N=3 (half D=3, chi=16 "
                       "exact truncation; half D in 3..5, chi in 16..64 randomized truncation), "
                       "simple-update tensors, fp32 contraction GEMMs; Poisson arrivals at 200 "
                       f"req/s, {n} requests, each an ITE-step perturbation + warm-started "
                       f"sweeps to {tol:g} (at most {4 * max_sweeps} exact, {max_sweeps} "
                       "randomized) + expectation",
           "tolerance": tol, "max_sweeps": max_sweeps,
           "hbm_budget_bytes": budget, "resident_bytes": int(res_bytes),
           "max_workspace_bytes": int(max(ws)), "peak_workspace_bytes": int(st_b["peak_bytes"]),
           "slot_allocations": int(st_b["slot_allocations"]),
           "max_inflight": args.serving_inflight, "peak_inflight": int(st_b["peak_inflight"]),
           "by_state_class": by_cls,
           "one_at_a_time": summary(res_s, wall_s)}
    out.update(summary(res_b, wall_b))
    return out


def copy_calibration(mib):
    """A plain device-to-device copy of a known size, for scaling the HBM
    counters (FETCH_SIZE, WRITE_SIZE) of the kernels."""
    import torch
    n = mib << 20
    src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n, "launches": 3}), flush=True)


def _counter_means(path, counter):
    """Mean value of ``counter`` per dispatch, per kernel name, from a
    rocprofv3 counter-collection CSV."""
    import csv
    acc = {}
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            if row.get("Counter_Name") != counter:
                continue
            name = row["Kernel_Name"]
            base = name.split("(")[0].split("<")[0].replace("void ", "").strip()
            base = base.split("::")[-1]
            a = acc.setdefault(base, [0.0, 0])
            a[0] += float(row["Counter_Value"])
            a[1] += 1
    return {k: (v[0] / v[1], v[1]) for k, v in acc.items()}


def traffic_from(fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, command, copy_mib, out):
    """HBM bytes per launch for each kernel: FETCH_SIZE and WRITE_SIZE (KiB
    per dispatch) scaled by what the same counters read for a plain copy of
    known size (bench.py --copy-calibration)."""
    fetch, write = _counter_means(fetch_csv, "FETCH_SIZE"), _counter_means(write_csv, "WRITE_SIZE")
    cf, cw = _counter_means(copy_fetch_csv, "FETCH_SIZE"), _counter_means(copy_write_csv, "WRITE_SIZE")
    # the copy kernel: the kernel of the calibration run with the largest
    # mean counter value (the copy of copy_mib MiB)
    kf = max(cf.items(), key=lambda kv: kv[1][0])
    kw = max(cw.items(), key=lambda kv: kv[1][0])
    copy_bytes = float(copy_mib << 20)
    scale_f = kf[1][0] * 1024.0 / copy_bytes
    scale_w = kw[1][0] * 1024.0 / copy_bytes
    kernels = {}
    for k in sorted(set(fetch) & set(write)):
        fb = fetch[k][0] * 1024.0 / scale_f
        wb = write[k][0] * 1024.0 / scale_w
        kernels[k] = {"bytes_per_launch": fb + wb, "fetch_bytes_per_launch": fb,
                      "write_bytes_per_launch": wb, "dispatches": fetch[k][1]}
    src = os.path.join(ROOT, "paper_2603_13304_amd", "csrc", "kernels.hip")
    with open(src, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()
    rec = {"command": command, "copy_kernel": kf[0], "copy_bytes": copy_bytes,
           "fetch_scale": scale_f, "write_scale": scale_w, "kernels_hip_sha256": sha,
           "kernels": kernels}
    with open(out, "w") as f:
        json.dump(rec, f, indent=1, sort_keys=True)
    print(out)


def stats_summary(path):
    """Per-kernel table (template instances of k_gemm grouped by precision)
    of a rocprofv3 kernel_stats.csv: calls, total and average duration."""
    import csv
    agg = {}
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            name = row["Name"].replace("void ", "")
            base = name.split("(")[0]
            key = base.split("<")[0].split("::")[-1]
            if key == "k_gemm":   # k_gemm<precision, tile shape>
                key += "<" + base.split("<")[1].split(",")[0] + ">"
            a = agg.setdefault(key, [0, 0.0])
            a[0] += int(row["Calls"])
            a[1] += float(row["TotalDurationNs"])
    tot = sum(v[1] for v in agg.values())
    print("| kernel | calls | total ms | avg us | share |")
    print("|---|---|---|---|---|")
    for k, (n, ns) in sorted(agg.items(), key=lambda kv: -kv[1][1]):
        print(f"| {k} | {n} | {ns / 1e6:.2f} | {ns / n / 1e3:.2f} | {100 * ns / tot:.1f} % |")


def timeline_summary(path, per, timed, trailing):
    """Overlap of the kernels of the timed sweeps in a rocprofv3 kernel trace:
    the share of the window with at least one and with two or more kernels
    running, and per kernel the summed duration and the time it ran alone."""
    import csv
    rows = []
    with open(path, newline="") as f:
        for r in csv.DictReader(f):
            name = r["Kernel_Name"].replace("void ", "").split("(")[0].split("<")[0].split("::")[-1]
            rows.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), name))
    rows.sort()
    sel = rows[len(rows) - per * (timed + trailing):][:per * timed]
    t0, t1 = sel[0][0], max(e for _, e, _ in sel)
    ev = sorted([(s, 1, k) for s, _, k in sel] + [(e, -1, k) for _, e, k in sel],
                key=lambda x: (x[0], x[1]))
    busy = two = 0
    cur, last = 0, t0
    active, alone, total = {}, {}, {}
    for t, d, k in ev:
        dt = t - last
        if cur >= 1:
            busy += dt
        if cur >= 2:
            two += dt
        if cur == 1:
            only = next(iter(active))
            alone[only] = alone.get(only, 0) + dt
        cur += d
        active[k] = active.get(k, 0) + d
        if active[k] == 0:
            del active[k]
        last = t
    for s_, e_, k in sel:
        total[k] = total.get(k, 0) + e_ - s_
    w = t1 - t0
    print(f"{len(sel)} launches in {timed} timed sweeps, window {w / 1e6:.1f} ms "
          f"({w / 1e6 / timed:.1f} ms per sweep)\n")
    print(f"- at least one kernel running: {100 * busy / w:.1f} % of the window")
    print(f"- two or more kernels running: {100 * two / w:.1f} %\n")
    print("| kernel | summed duration, ms per sweep | running alone, ms per sweep |")
    print("|---|---|---|")
    for k, v in sorted(total.items(), key=lambda kv: -kv[1])[:10]:
        print(f"| {k} | {v / 1e6 / timed:.1f} | {alone.get(k, 0) / 1e6 / timed:.1f} |")


def main():
    args = parse()
    if args.timeline_summary:
        path, per, timed, trailing = args.timeline_summary
        timeline_summary(path, int(per), int(timed), int(trailing))
        return
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.traffic_from:
        traffic_from(*args.traffic_from, args.traffic_command, args.copy_mib, args.traffic_out)
        return
    if args.stats_summary:
        stats_summary(args.stats_summary)
        return
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
    t0 = time.perf_counter()
    n_tuned = 0 if args.no_autotune else g.autotune(args.tile_cache)[1]
    tune_s = time.perf_counter() - t0
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
    lat, ss, e = [], [], float("nan")
    for _ in range(args.expect_reps):
        t = time.perf_counter()
        _, ss, e = g.blockbp_expect()
        lat.append(1e3 * (time.perf_counter() - t))
    # the FP64 reference of the precision runs: one more sweep from the same
    # messages, then the expectation
    err_next, e_next = float("nan"), float("nan")
    if not args.no_precisions and args.precision == "fp64":
        _, err_next, _ = g.blockbp_sweep(1, 0.0)
        _, _, e_next = g.blockbp_expect()
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
                   "message_updates_per_step": n_msg, "graph": not args.no_graph, "streams": args.streams,
                   "autotuned_gemm_shapes": n_tuned, "autotune_seconds": round(tune_s, 2)},
        "roofline": roof,
        "mfma": mfma,
        "expect_latency_ms": {"p50": float(np.percentile(lat, 50)) if lat else None,
                              "p99": float(np.percentile(lat, 99)) if lat else None,
                              "sweeps_before": sw, "distance_reached": err_c,
                              "tolerance_reached": bool(err_c <= 1e-5),
                              "energy_per_site": e, "bonds": len(ss)},
        "sweep": {"device_ms": round(dev_ms, 3), "launches": int(nlaunch),
                  "contraction_gflop": cf / 1e9, "gemm_gflop": gf / 1e9, "kernels": breakdown},
    }
    if not args.no_precisions and args.precision == "fp64":
        out["precisions"] = precision_runs(args, ts, msgs, e_next, err_next)
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
