"""Benchmark: local-max matching phase loop on one MI355X.

Workload (one step = one whole lm_match solve, every phase of the path):
2-D random geometric graph, n = 2^24 points uniform in the unit square,
radius for average degree 10, weight 1 - distance (fp32), seed 1; inputs are
resident in HBM as torch tensors before the timed region starts.

Prints ONE JSON line with edges/s (input undirected edges / solve time),
the roofline of the dominant kernel (algorithmic bytes / HIP-event time on
the solve stream), p50/p99 solve latency, and the CPU oracle timed on the
host (one core) on the same graph.

  python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--no-cpu] [--batch]
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published


KERNEL_SOURCES = ["paper_1302_4587_amd/csrc/lm_kernels.hip", "paper_1302_4587_amd/csrc/lm_device.h",
                  "paper_1302_4587_amd/csrc/lm_key.h", "paper_1302_4587_amd/csrc/lm_internal.h"]
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "rgg24_hbm_traffic.md")


def _measured_traffic():
    """HBM bytes per compaction launch from the committed counter summary,
    or None once the kernel sources differ from the ones it was taken on."""
    import hashlib
    try:
        text = open(TRAFFIC_FILE).read()
    except OSError:
        return None
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    sha = tag = None
    for line in text.splitlines():
        if line.startswith("kernel_source_sha256:"):
            sha = line.split(":", 1)[1].strip()
        elif line.startswith("compact_traffic_bytes_per_launch:"):
            tag = float(line.split(":", 1)[1])
    return tag if sha == h.hexdigest() else None


def _percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = (len(xs) - 1) * q / 100.0
    f, c = math.floor(k), math.ceil(k)
    return xs[f] if f == c else xs[f] + (xs[c] - xs[f]) * (k - f)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=["rgg", "rmat"], default="rgg",
                    help="rgg: 2-D random geometric graph (the headline); rmat: R-MAT edge factor 16, unit weights")
    ap.add_argument("--log2n", type=int, default=24)
    ap.add_argument("--avg-degree", type=float, default=10.0)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle leg")
    ap.add_argument("--no-profile", action="store_true", help="time steps without per-kernel events")
    ap.add_argument("--batch", action="store_true", help="also time the 4096-graph batch (extra minutes)")
    ap.add_argument("--hip-graph", action="store_true",
                    help="enqueue set-up and first phases as one captured HIP graph (LM_GRAPH)")
    ap.add_argument("--serve", action="store_true",
                    help="also run the serving trace: continuous-batching server vs FIFO (extra minutes)")
    ap.add_argument("--serve-rates", type=str, default="50,150,300",
                    help="Poisson arrival rates (requests/s) for --serve")
    ap.add_argument("--serve-requests", type=int, default=160)
    ap.add_argument("--weight-array", action="store_true",
                    help="rmat: pass the all-ones weight array instead of no array (unweighted solve)")
    ap.add_argument("--copy-calib-mib", type=int, default=0,
                    help="first run a plain device copy of this many MiB (reference for HBM byte counters)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path (run with --gpus 1)",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import lmgen
    import paper_1302_4587_amd as lm

    dev = torch.device("cuda:0")
    n = 1 << args.log2n
    t0 = time.time()
    if args.workload == "rgg":
        g = lmgen.rgg(n, args.avg_degree, args.seed)
        workload = f"rgg2d n=2^{args.log2n} avg_degree={args.avg_degree:g} w=1-dist seed={args.seed}"
    else:
        g = lmgen.rmat(args.log2n, 16, seed=args.seed)
        rep = "as an all-ones weight array" if args.weight_array else "as an unweighted graph (no weight array)"
        workload = (f"rmat scale={args.log2n} edge_factor=16 (a,b,c,d)=(.57,.19,.19,.05) unit weights "
                    f"{rep} seed={args.seed}")
    gen_s = time.time() - t0
    print(f"bench: generated {args.workload} n={g.n} m={g.m} nnz={g.nnz} in {gen_s:.1f}s", file=sys.stderr, flush=True)
    rp = torch.from_numpy(g.row_ptr).to(dev)
    col = torch.from_numpy(g.col).to(dev)
    # unit weights carry no information: by default they are passed as no
    # weight array (w=None), the library's unweighted mode, which reads none
    w = None if (args.workload == "rmat" and not args.weight_array) else torch.from_numpy(g.w).to(dev)
    mate = torch.empty(g.n, dtype=torch.int32, device=dev)
    torch.cuda.synchronize()

    if args.copy_calib_mib > 0:
        # a plain elementwise copy of known size: reads and writes exactly
        # copy_calib_mib MiB, so HBM counters of the same run can be scaled
        src = torch.ones((args.copy_calib_mib << 20) // 4, dtype=torch.int32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(2):
            torch.add(src, 0, out=dst)
        torch.cuda.synchronize()
        del src, dst

    ctx = lm.Context(0)
    profile = not args.no_profile
    for i in range(args.warmup):
        ctx.match(rp, col, w, seed=args.seed, mate=mate, hip_graph=args.hip_graph)
    # one untimed solve with events on every kernel kind names the dominant
    # kernel; the timed steps put events only around that kernel's launches
    # (each timed launch costs two events on the stream)
    breakdown, dom = None, None
    if profile:
        _, st0 = ctx.match(rp, col, w, seed=args.seed, mate=mate, profile=True)
        breakdown = {k: round(v, 4) for k, v in st0.kernel_ms.items()}
        dom = max(st0.kernel_ms, key=lambda k: st0.kernel_ms[k])
    torch.cuda.synchronize()
    # timed region: exactly K steps
    lat = []
    kms = {k: 0.0 for k in lm._lib.KERNEL_KINDS}
    kbytes = {k: 0.0 for k in lm._lib.KERNEL_KINDS}
    klaunch = {k: 0 for k in lm._lib.KERNEL_KINDS}
    phases = None
    bytes_alg = 0.0
    dev_ms = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        ts = time.perf_counter()
        _, st = ctx.match(rp, col, w, seed=args.seed, mate=mate, profile=profile, hip_graph=args.hip_graph,
                          profile_kinds=[dom] if profile else None)
        lat.append((time.perf_counter() - ts) * 1e3)
        dev_ms.append(st.device_ms)
        phases = st.phases
        bytes_alg = st.bytes_alg
        for k in kms:
            kms[k] += st.kernel_ms[k]
            kbytes[k] += st.kernel_bytes[k]
            klaunch[k] += st.kernel_launches[k]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_per_step = elapsed * 1e3 / args.steps
    edges_per_s = g.m / (ms_per_step / 1e3)

    # correctness of what was timed (cheap property check at full size)
    got = mate.cpu().numpy()
    import oracle  # test infrastructure: certificate and CPU baseline only

    cert = oracle.greedy_certificate(g.n, g.row_ptr, g.col, g.w, args.seed, got)

    roof = None
    if profile:
        achieved = kbytes[dom] / (kms[dom] / 1e3) / 1e9 if kms[dom] > 0 else 0.0
        traffic = _measured_traffic() if dom == "compact" else None
        roof = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": round(traffic, 1) if traffic is not None else None,
                "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "bytes_per_launch": kbytes[dom] / max(klaunch[dom], 1),
                "avg_launch_us": kms[dom] * 1e3 / max(klaunch[dom], 1),
                "kernel_launches_per_step": klaunch[dom] / args.steps,
                "kernel_ms_untimed_solve": breakdown}

    cpu = None
    if not args.no_cpu:
        # the oracle is single-threaded C: one host core, median of 3 solves
        times = []
        for _ in range(3):
            t1 = time.perf_counter()
            ref_mate, ref_log = oracle.local_max_graph(g, args.seed)
            times.append(time.perf_counter() - t1)
        cpu_s = float(np.median(times))
        if not np.array_equal(ref_mate, got):
            print("bench: WARNING gpu mate differs from the oracle", file=sys.stderr, flush=True)
        cpu = {"value": round(g.m / cpu_s, 1), "unit": "edges/s", "cores": 1, "kind": "oracle",
               "sample": f"whole graph (n=2^{args.log2n}, m={g.m}), median of 3 solves, {cpu_s:.2f}s each",
               "host_cpus": os.cpu_count(), "phases": int(len(ref_log)),
               "matches_gpu": bool(np.array_equal(ref_mate, got))}

    batch = None
    if args.batch:
        batch = bench_batch(ctx, dev)
    serve = None
    if args.serve:
        serve = bench_serve(ctx, [float(x) for x in args.serve_rates.split(",") if x],
                            args.serve_requests)

    out = {
        "metric": "input edges matched/sec + achieved HBM GB/s (1 GPU); batched p50/p99 latency",
        "value": round(edges_per_s, 1),
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "fp32",
        "data": "synthetic",
        "config": {"workload": workload,
                   "n": g.n, "m": g.m, "nnz": g.nnz, "phases": phases, "parallelism": "single GPU"},
        "gbps_alg_whole_solve": round(bytes_alg / (np.median(dev_ms) / 1e3) / 1e9, 1),
        "device_ms_median": round(float(np.median(dev_ms)), 4),
        "latency_ms": {"p50": round(_percentile(lat, 50), 4), "p99": round(_percentile(lat, 99), 4)},
        "certificate_violations": cert,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    if batch is not None:
        out["batch"] = batch
    if serve is not None:
        out["serve"] = serve
    print(json.dumps(out), flush=True)


def bench_batch(ctx, dev):
    """4096 random graphs, n log-uniform in [2^8, 2^16], avg degree U[4,32]:
    one batched solve vs a loop of single solves (same GPU)."""
    import torch

    import lmgen

    b = lmgen.er_batch(4096, 1)
    vo = b.vtx_off
    rp = torch.from_numpy(b.row_ptr).to(dev)
    col = torch.from_numpy(b.col).to(dev)
    w = torch.from_numpy(b.w).to(dev)
    mate = torch.empty(b.n_total, dtype=torch.int32, device=dev)
    ctx.match_batch(vo, rp, col, w, mate=mate)
    torch.cuda.synchronize()
    lat = []
    for _ in range(10):
        t = time.perf_counter()
        ctx.match_batch(vo, rp, col, w, mate=mate, want_graph_phases=False)
        lat.append((time.perf_counter() - t) * 1e3)
    # one graph per launch over the same graphs
    t = time.perf_counter()
    for k in range(b.graphs):
        a, e = int(vo[k]), int(vo[k + 1])
        e0, e1 = int(b.row_ptr[a]), int(b.row_ptr[e])
        ctx.match(rp[a:e + 1] - e0, col[e0:e1], w[e0:e1], seed=1, mate=mate[a:e])
    torch.cuda.synchronize()
    single_ms = (time.perf_counter() - t) * 1e3
    return {"graphs": b.graphs, "n_total": b.n_total, "m_total": b.nnz // 2,
            "batched_ms": {"p50": round(_percentile(lat, 50), 3), "p99": round(_percentile(lat, 99), 3)},
            "batched_edges_per_s": round((b.nnz // 2) / (_percentile(lat, 50) / 1e3), 1),
            "one_graph_per_launch_ms": round(single_ms, 3)}


def bench_serve(ctx, rates, requests, pool=48, seed=1):
    """Serving trace: Poisson arrivals of host graphs (50/50 RGG avg degree 10
    and R-MAT edge factor 16, uniform weights, n log-uniform in [2^10, 2^22];
    a pool of `pool` pre-generated graphs is cycled, generation is not timed),
    64 GB admission budget. The continuous-batching server and the FIFO
    server (one lm_match per request) see the same trace; latency is submit
    to result on the host, throughput is input edges over the makespan."""
    import threading

    import lmgen
    import paper_1302_4587_amd as lm

    t0 = time.time()
    shapes = lmgen.serving_trace(pool, 1.0, seed)
    graphs = [lmgen.serving_graph(k, n, seed) for _, k, n in shapes]
    print(f"bench: serving pool of {pool} graphs in {time.time() - t0:.1f}s", file=sys.stderr, flush=True)
    refs = {}
    out = {"pool_graphs": pool, "requests_per_point": requests, "budget_gb": 64,
           "pool_mean_edges": round(float(np.mean([g.nnz // 2 for g in graphs])), 1), "points": []}
    for rate in rates:
        arr = [a for a, _, _ in lmgen.serving_trace(requests, rate, seed + 1)]
        point = {"rate_per_s": rate}
        for name, mode in (("batched", lm.LM_SERVE_BATCHED), ("fifo", lm.LM_SERVE_FIFO)):
            tickets = [None] * requests
            with lm.Server(ctx, hbm_budget_bytes=64 << 30, max_resident=256, mode=mode) as srv:
                sub_s = []

                def submitter(part, parts):
                    for i in range(part, requests, parts):
                        dt = arr[i] - (time.perf_counter() - t_start)
                        if dt > 0:
                            time.sleep(dt)
                        g = graphs[i % pool]
                        t_sub = time.perf_counter()
                        tickets[i] = srv.submit(g.row_ptr, g.col, g.w, seed=1)
                        sub_s.append(time.perf_counter() - t_sub)

                t_start = time.perf_counter()
                ths = [threading.Thread(target=submitter, args=(p, 4)) for p in range(4)]
                for th in ths:
                    th.start()
                lat, qms, edges, bad = [], [], 0, 0
                for i in range(requests):
                    while tickets[i] is None:
                        time.sleep(0.0002)
                    mate, info = srv.wait(tickets[i], -1)
                    lat.append(info["latency_ms"])
                    qms.append(info["queue_ms"])
                    g = graphs[i % pool]
                    edges += g.nnz // 2
                    k = i % pool
                    if k not in refs:
                        refs[k] = mate.copy()
                    elif not np.array_equal(refs[k], mate):
                        bad += 1
                makespan = time.perf_counter() - t_start
                for th in ths:
                    th.join()
            point[name] = {"p50_ms": round(_percentile(lat, 50), 3), "p99_ms": round(_percentile(lat, 99), 3),
                           "queue_p50_ms": round(_percentile(qms, 50), 3), "queue_p99_ms": round(_percentile(qms, 99), 3),
                           "submit_ms_mean": round(1e3 * sum(sub_s) / max(len(sub_s), 1), 3),
                           "edges_per_s": round(edges / makespan, 1), "requests_per_s": round(requests / makespan, 2),
                           "mismatches": bad}
            print(f"bench: serve rate={rate} {name}: {point[name]}", file=sys.stderr, flush=True)
        out["points"].append(point)
    return out


if __name__ == "__main__":
    main()
