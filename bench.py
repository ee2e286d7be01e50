"""Benchmark: local-max matching phase loop on one MI355X.

One step = one whole lm_match solve (every phase of the path) of the
headline workload, R-MAT scale 24 (edge factor 16, (a,b,c,d) =
(.57,.19,.19,.05), unit weights solved as an unweighted graph, seed 1), the
largest single-GPU configuration; inputs are resident in HBM as torch
tensors before the timed region starts.

Prints ONE JSON line: edges/s of the headline (input undirected edges / wall
time per solve), the roofline of its dominant kernel (algorithmic bytes per
launch from the survey's per-phase byte model over the phase log, divided by
the launch's HIP-event time on the solve stream; the library's own byte
model beside it), p50/p99 solve latency, and the CPU oracle timed on the
host (one core) on the same graph. The same line carries the 2-D random
geometric graph (n = 2^24, average degree 10, w = 1 - distance) measured the
same way, and the 4096-graph batch (p50/p99 over the replays, every graph
compared with the oracle, the oracle timed on one core and on all cores).

  python bench.py [--gpus 1] [--steps 20] [--warmup 3] [--workload all|rmat|rgg] [--no-cpu]
                  [--no-batch] [--batch-replays 50] [--serve]
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
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
                  "paper_1302_4587_amd/csrc/lm_key.h", "paper_1302_4587_amd/csrc/lm_internal.h",
                  "paper_1302_4587_amd/csrc/lm_tail.hip", "paper_1302_4587_amd/csrc/lm_first.hip"]
CONTRACT_SOURCES = ["paper_1302_4587_amd/csrc/lm_contract.hip"]


def _kernel_sha():
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def _measured_traffic(workload, kind):
    """HBM bytes per launch of kernel kind `kind` from the committed counter
    summary profiles/<workload>_hbm_traffic.md, or None once the kernel
    sources differ from the ones it was taken on."""
    try:
        text = open(os.path.join(ROOT, "profiles", f"{workload}_hbm_traffic.md")).read()
    except OSError:
        return None
    sha = tag = None
    for line in text.splitlines():
        if line.startswith("kernel_source_sha256:"):
            sha = line.split(":", 1)[1].strip()
        elif line.startswith(f"{kind}_traffic_bytes_per_launch:"):
            tag = float(line.split(":", 1)[1])
    return tag if sha == _kernel_sha() else None


def _percentile(xs, q):
    xs = sorted(xs)
    if not xs:
        return float("nan")
    k = (len(xs) - 1) * q / 100.0
    f, c = math.floor(k), math.ceil(k)
    return xs[f] if f == c else xs[f] + (xs[c] - xs[f]) * (k - f)


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def survey_bytes(log, n, eb):
    """Algorithmic bytes from the per-phase model: per phase t, (eb + 1) L_t
    (each live entry once plus its neighbour's state byte), eb L_{t+1} (the
    survivors written), 12 V_t (row offset, candidate write, partner-candidate
    read); plus 8 n (input offsets and mate). eb = 8 for (col, w) entries, 4
    for an unweighted graph (col only). Returns (whole solve, per phase list)."""
    L = [int(r[0]) for r in log] + [0]
    V = [int(r[1]) for r in log]
    per = [(eb + 1) * L[t] + eb * L[t + 1] + 12 * V[t] for t in range(len(V))]
    return float(sum(per) + 8 * n), per


def run_single(ctx, g, w_t, rp, col, args, name, unweighted):
    """Times args.steps solves of one graph; returns the measurement dict and
    the mate array of the last timed solve."""
    import torch

    import paper_1302_4587_amd as lm

    dev = rp.device
    mate = torch.empty(g.n, dtype=torch.int32, device=dev)
    for _ in range(args.warmup):
        ctx.match(rp, col, w_t, seed=args.seed, mate=mate, hip_graph=args.hip_graph)
    # one untimed solve with events on every kernel kind names the dominant
    # kernel; the timed steps put events only around that kernel's launches
    # (each timed launch costs two events on the stream)
    profile = not args.no_profile
    breakdown, dom = None, None
    if profile:
        _, st0 = ctx.match(rp, col, w_t, seed=args.seed, mate=mate, profile=True)
        breakdown = {k: round(v, 4) for k, v in st0.kernel_ms.items()}
        dom = max(st0.kernel_ms, key=lambda k: st0.kernel_ms[k])
    kms = {k: 0.0 for k in lm._lib.KERNEL_KINDS}
    kbytes = {k: 0.0 for k in lm._lib.KERNEL_KINDS}
    klaunch = {k: 0 for k in lm._lib.KERNEL_KINDS}
    lat, dev_ms = [], []
    st = None
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        _, st = ctx.match(rp, col, w_t, seed=args.seed, mate=mate, profile=profile, hip_graph=args.hip_graph,
                          profile_kinds=[dom] if profile else None)
        lat.append((time.perf_counter() - ts) * 1e3)
        dev_ms.append(st.device_ms)
        for k in kms:
            kms[k] += st.kernel_ms[k]
            kbytes[k] += st.kernel_bytes[k]
            klaunch[k] += st.kernel_launches[k]
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_per_step = elapsed * 1e3 / args.steps
    got = mate.cpu().numpy()
    eb = 4 if unweighted else 8
    b_solve, b_phase = survey_bytes(st.log, g.n, eb)
    roof = None
    if profile and klaunch[dom] > 0:
        launches = klaunch[dom] / args.steps
        avg_s = kms[dom] / 1e3 / klaunch[dom]
        # survey bytes of the dominant kind, per launch
        nc = st.kernel_launches["compact"]
        if dom == "compact":
            b_kind = sum(b_phase[:nc])
        elif dom == "tail":
            b_kind = sum(b_phase[nc:])
        elif dom == "argmax":
            L1 = int(st.log[0][0]) if len(st.log) else 0
            V1 = int(st.log[0][1]) if len(st.log) else 0
            b_kind = eb * L1 + 12 * V1
        else:
            b_kind = float("nan")
        per_launch = b_kind / max(launches, 1e-9)
        achieved = per_launch / avg_s / 1e9
        lib_per_launch = kbytes[dom] / klaunch[dom]
        traffic = _measured_traffic(name, dom)
        roof = {"bound": "hbm", "kernel": dom, "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": round(traffic, 1) if traffic is not None else None,
                "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                "bytes_per_launch": round(per_launch, 1),
                "bytes_model": f"per phase (eb+1)L_t + eb L_(t+1) + 12 V_t, eb = {eb}",
                "avg_launch_us": round(avg_s * 1e6, 2),
                "kernel_launches_per_step": launches,
                "library_model_bytes_per_launch": round(lib_per_launch, 1),
                "library_model_frac": round(lib_per_launch / avg_s / 1e9 / HBM_PEAK_GBS, 4),
                "kernel_ms_untimed_solve": breakdown}
    renew = None
    if not args.no_renew:
        # the same graph with keys renewed every phase (LM_RENEW_KEYS): the
        # phase count against the fixed keys' (the paper's open question of
        # its Section 4); a few solves, outside the timed steps
        rl = []
        sr = None
        for _ in range(4):
            torch.cuda.synchronize()
            ts = time.perf_counter()
            _, sr = ctx.match(rp, col, w_t, seed=args.seed, mate=mate, renew_keys=True)
            rl.append((time.perf_counter() - ts) * 1e3)
        got_r = mate.cpu().numpy()
        chk_f = _matching_check(g, got)
        chk_r = _matching_check(g, got_r)
        renew = {"phases_fixed": st.phases, "phases_renewed": sr.phases,
                 "ms_per_solve_renewed": round(float(np.median(rl[1:])), 4),
                 "live_entries_per_phase_renewed": [int(r[0]) for r in sr.log],
                 "matched_edges_fixed": chk_f["edges"], "matched_edges_renewed": chk_r["edges"],
                 "matched_weight_fixed": chk_f["weight"], "matched_weight_renewed": chk_r["weight"],
                 "renewed_valid_maximal": chk_r["valid_maximal"]}
    contract = None
    if not args.no_contract:
        contract = run_contract(ctx, g, w_t, rp, col, got, args, unweighted)
    import oracle  # test infrastructure: certificate and CPU baseline only

    cert = oracle.greedy_certificate(g.n, g.row_ptr, g.col, g.w, args.seed, got)
    out = {"workload": None, "n": g.n, "m": g.m, "nnz": g.nnz, "phases": st.phases,
           "ms_per_step": round(ms_per_step, 4), "edges_per_s": round(g.m / (ms_per_step / 1e3), 1),
           "device_ms_median": round(float(np.median(dev_ms)), 4),
           "latency_ms": {"p50": round(_percentile(lat, 50), 4), "p99": round(_percentile(lat, 99), 4)},
           "gbps_alg_whole_solve": round(b_solve / (np.median(dev_ms) / 1e3) / 1e9, 1),
           "gbps_alg_whole_solve_library_model": round(st.bytes_alg / (np.median(dev_ms) / 1e3) / 1e9, 1),
           "live_entries_per_phase": [int(r[0]) for r in st.log],
           "certificate_violations": cert, "roofline": roof}
    if renew is not None:
        out["renewed_keys"] = renew
    if contract is not None:
        out["contract"] = contract
    return out, got


def run_contract(ctx, g, w_t, rp, col, got, args, unweighted):
    """Contracts the graph by its matching (lm_contract, the coarsening step):
    args.steps timed calls after two untimed ones, then the oracle on the
    same input for equality and the CPU time."""
    import torch

    dev = rp.device
    mate_t = torch.from_numpy(got).to(dev)
    for _ in range(2):
        ctx.contract(rp, col, w_t, mate_t)
    torch.cuda.synchronize()
    lat, dms = [], []
    out = None
    for _ in range(args.steps):
        ts = time.perf_counter()
        out = ctx.contract(rp, col, w_t, mate_t)
        lat.append((time.perf_counter() - ts) * 1e3)
        dms.append(out[5].device_ms)
    torch.cuda.synchronize()
    st = out[5]
    dev_ms = float(np.median(dms))
    achieved = st.bytes_alg / (dev_ms / 1e3) / 1e9
    res = {"ms_per_call": round(float(np.median(lat)), 4), "device_ms_median": round(dev_ms, 4),
           "fine_edges_per_s": round(g.m / (dev_ms / 1e3), 1), "coarse_n": int(out[1].shape[0]) - 1,
           "coarse_nnz": int(out[2].shape[0]), "long_rows": st.long_rows, "long_entries": st.long_entries,
           "roofline": {"bound": "hbm", "kernel": "whole contraction", "achieved": round(achieved, 1),
                        "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                        "bytes_per_call": st.bytes_alg,
                        "bytes_model": "8(n+1) + 8n + (eb+4) nnz + 8(nc+1) + 8 nnz_c, eb = 4 unweighted, 8 weighted"}}
    if not args.no_cpu:
        import oracle  # test infrastructure: equality check and CPU baseline only

        t1 = time.perf_counter()
        want = oracle.contract(g.n, g.row_ptr, g.col, None if unweighted else g.w, got)
        cpu_s = time.perf_counter() - t1
        gotc = [x.cpu().numpy() for x in out[:4]]
        same = all(np.array_equal(a.view(np.uint32) if a.dtype == np.float32 else a,
                                  np.asarray(b).view(np.uint32) if a.dtype == np.float32 else b)
                   for a, b in zip(gotc, want[:4]))
        res["matches_oracle"] = bool(same)
        res["cpu_baseline"] = {"value": round(g.m / cpu_s, 1), "unit": "fine edges/s", "cores": 1, "kind": "oracle",
                               "sample": f"whole graph, one call, {cpu_s:.2f}s"}
    return res


def _matching_check(g, mate):
    """Vectorised check that mate is a valid maximal matching of g (mutual, on
    edges, no edge with both ends free); returns its size and weight."""
    n = g.n
    deg = np.diff(g.row_ptr)
    rows = np.repeat(np.arange(n, dtype=np.int32), deg)
    m = mate.astype(np.int64)
    matched = m >= 0
    mutual = bool(np.all(m[m[matched]] == np.flatnonzero(matched)))
    on_edge = g.col == mate[rows]
    hits = np.bincount(rows[on_edge], minlength=n)
    edges_ok = bool(np.all(hits[matched] == 1))
    maximal = not bool(np.any((mate[rows] < 0) & (mate[g.col] < 0)))
    del rows
    return {"edges": int(matched.sum()) // 2, "weight": round(float(g.w[on_edge].astype(np.float64).sum()) / 2, 3),
            "valid_maximal": mutual and edges_ok and maximal}


def cpu_oracle(g, seed, got, reps):
    """The oracle (single-threaded C) on the whole graph: median of reps solves."""
    import oracle  # test infrastructure: CPU baseline only

    times = []
    ref_mate = ref_log = None
    for _ in range(reps):
        t1 = time.perf_counter()
        ref_mate, ref_log = oracle.local_max_graph(g, seed)
        times.append(time.perf_counter() - t1)
    cpu_s = float(np.median(times))
    same = bool(np.array_equal(ref_mate, got))
    if not same:
        print("bench: WARNING gpu mate differs from the oracle", file=sys.stderr, flush=True)
    return {"value": round(g.m / cpu_s, 1), "unit": "edges/s", "cores": 1, "kind": "oracle",
            "sample": f"whole graph (n={g.n}, m={g.m}), median of {reps} solve(s), {cpu_s:.2f}s each",
            "host_cpus": os.cpu_count(), "cpu_model": _cpu_model(), "phases": int(len(ref_log)),
            "matches_gpu": same}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", choices=["all", "rmat", "rgg"], default="all",
                    help="all: R-MAT scale 24 (headline), RGG 2^24 and the 4096-graph batch; rmat or rgg: one graph")
    ap.add_argument("--log2n", type=int, default=24)
    ap.add_argument("--avg-degree", type=float, default=10.0)
    ap.add_argument("--seed", type=int, default=1)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle legs")
    ap.add_argument("--no-profile", action="store_true", help="time steps without per-kernel events")
    ap.add_argument("--no-batch", action="store_true", help="skip the 4096-graph batch")
    ap.add_argument("--no-renew", action="store_true", help="skip the renewed-keys solves")
    ap.add_argument("--no-contract", action="store_true", help="skip the contraction by the matching")
    ap.add_argument("--batch-replays", type=int, default=50)
    ap.add_argument("--hip-graph", action="store_true",
                    help="run each solve as one captured HIP graph (LM_GRAPH)")
    ap.add_argument("--serve", action="store_true",
                    help="also run the serving trace: continuous-batching server vs FIFO (extra minutes)")
    ap.add_argument("--serve-fractions", type=str, default="0.1,0.3,0.6,0.9,1.2",
                    help="Poisson arrival rates for --serve, as fractions of the measured saturation rate")
    ap.add_argument("--serve-requests", type=int, default=1000)
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
    results = {}
    mates = {}
    graphs = {}
    for name in (["rmat", "rgg"] if args.workload == "all" else [args.workload]):
        t0 = time.time()
        if name == "rgg":
            g = lmgen.rgg(n, args.avg_degree, args.seed)
            workload = f"rgg2d n=2^{args.log2n} avg_degree={args.avg_degree:g} w=1-dist seed={args.seed}"
            unw = False
        else:
            g = lmgen.rmat(args.log2n, 16, seed=args.seed)
            unw = not args.weight_array
            rep = "an unweighted graph (no weight array)" if unw else "an all-ones weight array"
            workload = (f"rmat scale={args.log2n} edge_factor=16 (a,b,c,d)=(.57,.19,.19,.05) unit weights "
                        f"as {rep} seed={args.seed}")
        print(f"bench: generated {name} n={g.n} m={g.m} nnz={g.nnz} in {time.time() - t0:.1f}s",
              file=sys.stderr, flush=True)
        rp = torch.from_numpy(g.row_ptr).to(dev)
        col = torch.from_numpy(g.col).to(dev)
        # unit weights carry no information: by default they are passed as no
        # weight array (w=None), the library's unweighted mode, which reads none
        w_t = None if unw else torch.from_numpy(g.w).to(dev)
        torch.cuda.synchronize()
        res, got = run_single(ctx, g, w_t, rp, col, args, f"{name}{args.log2n}", unw)
        res["workload"] = workload
        results[name] = res
        mates[name] = got
        graphs[name] = g
        del rp, col, w_t
        print(f"bench: {name}: {res['ms_per_step']} ms/solve, {res['edges_per_s']:.3e} edges/s", file=sys.stderr,
              flush=True)

    batch = None
    if args.workload == "all" and not args.no_batch:
        batch = bench_batch(ctx, dev, args.batch_replays, not args.no_cpu)
    cpu = {}
    if not args.no_cpu:
        for name in results:
            cpu[name] = cpu_oracle(graphs[name], args.seed, mates[name], 1 if name == "rmat" else 3)
    serve = None
    if args.serve:
        serve = bench_serve(ctx, args.serve_requests, [float(x) for x in args.serve_fractions.split(",") if x])

    head = "rmat" if "rmat" in results else "rgg"
    h = results[head]
    out = {
        "metric": "input edges matched/sec + achieved HBM GB/s (1 GPU); batched p50/p99 latency",
        "value": h["edges_per_s"],
        "unit": "edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": h["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        # weighted graphs compare fp32 weights; an unweighted graph compares the
        # 64-bit tie-break keys alone
        "dtype": "fp32" if head == "rgg" or args.weight_array else "u64",
        "data": "synthetic",
        "config": {"workload": h["workload"], "n": h["n"], "m": h["m"], "nnz": h["nnz"], "phases": h["phases"],
                   "parallelism": "single GPU"},
        "gbps_alg_whole_solve": h["gbps_alg_whole_solve"],
        "gbps_alg_whole_solve_library_model": h["gbps_alg_whole_solve_library_model"],
        "device_ms_median": h["device_ms_median"],
        "latency_ms": h["latency_ms"],
        "live_entries_per_phase": h["live_entries_per_phase"],
        "certificate_violations": h["certificate_violations"],
        "roofline": h["roofline"],
        "renewed_keys": h.get("renewed_keys"),
        "contract": h.get("contract"),
        "cpu_baseline": cpu.get(head),
    }
    for name, res in results.items():
        if name != head:
            res = dict(res)
            res["cpu_baseline"] = cpu.get(name)
            out["rgg24" if name == "rgg" else name] = res
    if batch is not None:
        out["batch"] = batch
    if serve is not None:
        out["serve"] = serve
    print(json.dumps(out), flush=True)


def bench_batch(ctx, dev, replays, with_cpu):
    """4096 random graphs, n log-uniform in [2^8, 2^16], avg degree U[4,32],
    uniform weights: one batched solve (one captured HIP graph) timed over
    `replays` replays, against a loop of single solves over the same graphs
    on the same GPU. Every graph's mate is compared with the oracle (which is
    timed on one core, summed over the graphs, and on all host cores)."""
    import torch

    import lmgen

    t0 = time.time()
    b = lmgen.er_batch(4096, 1)
    print(f"bench: generated batch of {b.graphs} graphs, nnz={b.nnz} in {time.time() - t0:.1f}s", file=sys.stderr,
          flush=True)
    vo = b.vtx_off
    rp = torch.from_numpy(b.row_ptr).to(dev)
    col = torch.from_numpy(b.col).to(dev)
    w = torch.from_numpy(b.w).to(dev)
    mate = torch.empty(b.n_total, dtype=torch.int32, device=dev)
    _, st, gph = ctx.match_batch(vo, rp, col, w, mate=mate)
    torch.cuda.synchronize()

    def replay():
        ls = []
        for _ in range(replays):
            t = time.perf_counter()
            ctx.match_batch(vo, rp, col, w, mate=mate, want_graph_phases=False)
            ls.append((time.perf_counter() - t) * 1e3)
        return ls

    lat_default = replay()
    # the autotuner (range size, grid, queued phases, the kernels' long-piece
    # threshold, the tail hand-over) picks the tuning the timed replays use
    base = ctx.tuning()
    t = time.perf_counter()
    tuned = ctx.autotune_batch(vo, rp, col, w)
    tune_s = time.perf_counter() - t
    ctx.match_batch(vo, rp, col, w, mate=mate, want_graph_phases=False)
    lat = replay()
    got = mate.cpu().numpy()
    ctx.set_tuning(**base)
    # one graph per launch over the same graphs: the row offsets of every graph
    # rebased to 0 once, outside the timed loop
    rps = []
    for k in range(b.graphs):
        a, e = int(vo[k]), int(vo[k + 1])
        rps.append(rp[a:e + 1] - rp[a])
    torch.cuda.synchronize()
    t = time.perf_counter()
    for k in range(b.graphs):
        a, e = int(vo[k]), int(vo[k + 1])
        e0, e1 = int(b.row_ptr[a]), int(b.row_ptr[e])
        ctx.match(rps[k], col[e0:e1], w[e0:e1], seed=1, mate=mate[a:e])
    torch.cuda.synchronize()
    single_ms = (time.perf_counter() - t) * 1e3
    out = {"workload": f"{b.graphs} ER graphs, n log-uniform in [2^8, 2^16], avg degree U[4,32], uniform weights",
           "graphs": b.graphs, "n_total": b.n_total, "m_total": b.nnz // 2, "phases": st.phases,
           "replays": replays,
           "batched_ms": {"p50": round(_percentile(lat, 50), 3), "p99": round(_percentile(lat, 99), 3)},
           "tuning": tuned, "autotune_s": round(tune_s, 2),
           "batched_ms_default_tuning": {"p50": round(_percentile(lat_default, 50), 3),
                                         "p99": round(_percentile(lat_default, 99), 3), "tuning": base},
           "batched_edges_per_s": round((b.nnz // 2) / (_percentile(lat, 50) / 1e3), 1),
           "one_graph_per_launch_ms": round(single_ms, 3),
           "one_graph_per_launch_edges_per_s": round((b.nnz // 2) / (single_ms / 1e3), 1)}
    if with_cpu:
        import oracle  # test infrastructure: CPU baseline and parity only

        def one(k):
            a, e = int(vo[k]), int(vo[k + 1])
            e0, e1 = int(b.row_ptr[a]), int(b.row_ptr[e])
            t1 = time.perf_counter()
            m, _ = oracle.local_max(e - a, b.row_ptr[a:e + 1] - e0, b.col[e0:e1], b.w[e0:e1], 1)
            return k, time.perf_counter() - t1, m

        cores = min(os.cpu_count() or 1, 16)
        t1 = time.perf_counter()
        bad = 0
        summed = 0.0
        with cf.ThreadPoolExecutor(cores) as ex:
            for k, dt, m in ex.map(one, range(b.graphs)):
                summed += dt
                a, e = int(vo[k]), int(vo[k + 1])
                bad += int(not np.array_equal(m, got[a:e]))
        wall = time.perf_counter() - t1
        out["graphs_differing_from_oracle"] = bad
        out["cpu_baseline"] = {"value": round((b.nnz // 2) / wall, 1), "unit": "edges/s", "cores": cores,
                               "kind": "oracle", "sample": f"all {b.graphs} graphs, one per task on {cores} threads",
                               "all_core_wall_s": round(wall, 3), "single_core_summed_s": round(summed, 3),
                               "cpu_model": _cpu_model()}
    del rp, col, w, rps
    return out


def bench_serve(ctx, requests, fractions, pool=48, seed=1):
    """Serving trace: Poisson arrivals of host graphs (50/50 RGG avg degree 10
    and R-MAT edge factor 16, uniform weights, n log-uniform in [2^10, 2^22];
    a pool of `pool` pre-generated graphs is cycled, generation is not timed),
    64 GB admission budget. The saturation rate is the batched server's
    throughput with every request submitted at once; the rates swept are the
    given fractions of it. The continuous-batching server and the FIFO server
    (one lm_match per request) see the same trace at each rate; latency is
    submit to result on the host, split into the submit call (pinned copy),
    queue (until admitted), device and copy back; throughput is input edges
    over the makespan. Every result is compared with the oracle."""
    import threading
    from concurrent.futures import ThreadPoolExecutor

    import lmgen
    import oracle  # test infrastructure: results of the pool graphs, checked outside the timed loop
    import paper_1302_4587_amd as lm

    t0 = time.time()
    shapes = lmgen.serving_trace(pool, 1.0, seed)
    graphs = [lmgen.serving_graph(k, n, seed) for _, k, n in shapes]
    with ThreadPoolExecutor(max_workers=16) as ex:
        refs = list(ex.map(lambda g: oracle.local_max_graph(g, 1)[0], graphs))
    print(f"bench: serving pool of {pool} graphs and their oracle results in {time.time() - t0:.1f}s",
          file=sys.stderr, flush=True)

    def run_point(mode, arr):
        count = len(arr)
        tickets = [None] * count
        sub_s = [0.0] * count
        with lm.Server(ctx, hbm_budget_bytes=64 << 30, max_resident=256, mode=mode) as srv:
            def submitter(part, parts):
                for i in range(part, count, parts):
                    dt = arr[i] - (time.perf_counter() - t_start)
                    if dt > 0:
                        time.sleep(dt)
                    g = graphs[i % pool]
                    t_sub = time.perf_counter()
                    tickets[i] = srv.submit(g.row_ptr, g.col, g.w, seed=1)
                    sub_s[i] = time.perf_counter() - t_sub

            t_start = time.perf_counter()
            ths = [threading.Thread(target=submitter, args=(p, 4)) for p in range(4)]
            for th in ths:
                th.start()
            lat, qms, dms, cms, edges, bad = [], [], [], [], 0, 0
            for i in range(count):
                while tickets[i] is None:
                    time.sleep(0.0002)
                mate, info = srv.wait(tickets[i], -1)
                lat.append(info["latency_ms"])
                qms.append(info["queue_ms"])
                dms.append(info["device_ms"])
                cms.append(info["copy_back_ms"])
                edges += graphs[i % pool].nnz // 2
                if not np.array_equal(refs[i % pool], mate):
                    bad += 1
            makespan = time.perf_counter() - t_start
            for th in ths:
                th.join()
        sub_ms = [1e3 * x for x in sub_s]
        q = lambda xs, p: round(_percentile(xs, p), 3)
        return {"p50_ms": q(lat, 50), "p99_ms": q(lat, 99),
                "split_p50_ms": {"submit": q(sub_ms, 50), "queue": q(qms, 50), "device": q(dms, 50),
                                 "copy_back": q(cms, 50)},
                "split_p99_ms": {"submit": q(sub_ms, 99), "queue": q(qms, 99), "device": q(dms, 99),
                                 "copy_back": q(cms, 99)},
                "edges_per_s": round(edges / makespan, 1), "requests_per_s": round(count / makespan, 2),
                "mismatches_vs_oracle": bad}

    nsat = min(requests, 400)
    sat = {}
    for name, mode in (("batched", lm.LM_SERVE_BATCHED), ("fifo", lm.LM_SERVE_FIFO)):
        sat[name] = run_point(mode, [0.0] * nsat)
        print(f"bench: serve saturation {name}: {sat[name]}", file=sys.stderr, flush=True)
    sat_rate = sat["batched"]["requests_per_s"]
    out = {"pool_graphs": pool, "requests_per_point": requests, "budget_gb": 64,
           "pool_mean_edges": round(float(np.mean([g.nnz // 2 for g in graphs])), 1),
           "saturation": {"requests": nsat, **sat}, "points": []}
    for f in fractions:
        rate = f * sat_rate
        arr = [a for a, _, _ in lmgen.serving_trace(requests, rate, seed + 1)]
        point = {"fraction_of_saturation": f, "rate_per_s": round(rate, 2)}
        for name, mode in (("batched", lm.LM_SERVE_BATCHED), ("fifo", lm.LM_SERVE_FIFO)):
            point[name] = run_point(mode, arr)
            print(f"bench: serve rate={rate:.1f} {name}: {point[name]}", file=sys.stderr, flush=True)
        out["points"].append(point)
    return out


if __name__ == "__main__":
    main()
