#!/usr/bin/env python3
"""Benchmark of the weighted-betweenness hot path on one MI355X.

Default workload: betweenness over k = 1024 seeded sampled sources of the
directed R-MAT scale-22 graph (4,194,304 vertices, 2^26 draws with
a, b, c, d = .57, .19, .19, .05, self-loops and duplicates dropped: 65,241,057
arcs), integer weights uniform in [1, 255] (seeded, synthetic), the largest
workload that fits one GPU.  One step is one bc_compute over the whole source
list in the batched form (one persistent launch, one workgroup and one state
slab per source in flight), inputs resident in HBM.  The plain form (one
source at a time on the whole GPU) is timed on a source subset for
comparison, and the CPU oracle on a bounded sample on every host core.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config rmat22]

Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

WORKLOADS = {
    "ba100k": "Barabasi-Albert n=100000 m=5 (499975 edges), w uniform [1,1000], all 100000 sources",
    "er1000": "Erdos-Renyi G(n=1000, M=4000), w uniform [1,100], all 1000 sources",
    "grid1000": "1000x1000 4-neighbour grid minus 2% edges (1958040 edges), w uniform [1,255], "
                "k=1024 sampled sources",
    "rmat22": "directed R-MAT scale 22 (a,b,c=.57,.19,.19; self-loops/duplicates dropped), "
              "w uniform [1,255], k=1024 sampled sources",
    "ablation": "thread-mapping variants on ER and Kronecker graphs n=2^14..2^18 (avg deg 32) "
                "and n=2^17 (avg deg 4), degree sweeps on ER n=20000 and Kronecker 2^15 (avg deg 4..64), "
                "w uniform [1,10], 256 sampled sources per graph",
    "dynamic": "Barabasi-Albert n=100000 m=5, w uniform [1,1000]: a sequence of 8 seeded arc "
               "changes (2 each of insert, delete, weight increase, weight decrease), each "
               "applied to all-source BC with bc_update_arc_device",
    "serving": "8 resident graphs (ER n=10k/500k deg 8 w[1,100]; BA n=50k/1M m=5 w[1,1000]; "
               "grid 100x100/1414x1414 -2% w[1,255]; R-MAT scale 14/21 w[1,255]); Poisson "
               "arrivals; each request k-sampled BC, k log-uniform in [64,4096]",
}


ABLATION_VARIANTS = [
    # (name, options) -- the paper's four thread mappings (Sec. 3.3-3.4, Figs. 3-5)
    # recast for 64-lane waves, plus the adaptive default of this library
    ("node-parallel, thread per vertex", dict(node_parallel=1, virtual_warp=1)),
    ("node-parallel, warp 32", dict(node_parallel=1, virtual_warp=32)),
    ("work-efficient, thread per vertex", dict(virtual_warp=1)),
    ("work-efficient, warp 4", dict(virtual_warp=4)),
    ("work-efficient, warp 8", dict(virtual_warp=8)),
    ("work-efficient, warp 16", dict(virtual_warp=16)),
    ("work-efficient, warp 32", dict(virtual_warp=32)),
    ("work-efficient, wave 64", dict(virtual_warp=64)),
    ("work-efficient, adaptive lane/wave", dict()),
]


def run_ablation(args):
    """Thread-mapping ablation on the paper's synthetic families (Sec. 4.2):
    ER and Kronecker graphs, n = 2^14..2^18 at average degree 32, n = 2^17 at
    average degree 4, and degree sweeps on ER n = 20000 and Kronecker 2^15;
    weights uniform in [1, 10] (Sec. 4.1).  Every variant
    runs the same sources with the same other settings."""
    import torch
    from paper_1701_05975_amd import bc, graphgen as gg

    # (family, n, edge factor = half the average degree); sizes first, then the
    # degree sweeps (Figs. 4-5)
    specs = []
    for sc in range(14, 19):
        specs += [("er", 1 << sc, 16), ("kron", 1 << sc, 16)]
    specs += [("er", 1 << 17, 2), ("kron", 1 << 17, 2)]
    for ef in (2, 4, 8, 32):
        specs += [("er", 20_000, ef), ("kron", 1 << 15, ef)]
    rows = []
    stream = torch.cuda.current_stream()
    for gi, (fam, n, ef) in enumerate(specs):
        sc = n.bit_length() - 1
        g = (gg.er_graph(n, ef * n, 1, 10, seed=300 + gi) if fam == "er"
             else gg.kronecker_graph(sc, ef, 1, 10, seed=400 + gi))
        srcs = gg.sample_sources(g, args.ablation_sources, seed=500 + gi)
        G = bc.Graph(g)
        s_dev = torch.from_numpy(srcs).to("cuda")
        out = torch.empty(g.n, dtype=torch.float64, device="cuda")
        ref = None
        for name, extra in ABLATION_VARIANTS:
            if args.variants and not any(x in name for x in args.variants.split(",")):
                continue
            o = bc.make_options(wg_threads=1024, stream=stream.cuda_stream, **extra)
            bc.bc_compute_device(G.handle, s_dev.data_ptr(), len(srcs), out.data_ptr(), o)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            st = bc.bc_compute_device(G.handle, s_dev.data_ptr(), len(srcs), out.data_ptr(), o)
            torch.cuda.synchronize()
            t = time.perf_counter() - t0
            res = out.cpu().numpy()
            if ref is None:
                ref = res
            nz = ref != 0
            dev = float(np.max(np.abs(res[nz] - ref[nz]) / np.abs(ref[nz]))) if nz.any() else 0.0
            assert dev <= 1e-9 and np.all(res[~nz] == 0), (name, dev)
            row = {"graph": f"{fam} n={n} avg deg {2 * ef}", "m": g.m, "variant": name,
                   "gteps": round(len(srcs) * g.m / t / 1e9, 4), "ms": round(t * 1e3, 2),
                   "iterations_per_source": round(st.iterations / len(srcs), 1)}
            rows.append(row)
            print(json.dumps(row), file=sys.stderr, flush=True)
        G.close()
    print(json.dumps({"metric": "thread-mapping ablation, weighted-BC GTEPS (batched form)",
                      "sources_per_graph": args.ablation_sources, "rows": rows}), flush=True)


def run_dynamic(args):
    """Dynamic updates on the BA workload: all-source BC is computed once, then
    each arc change of a seeded sequence is applied with bc_update_arc_device
    (only the affected sources run again, on the old and the new graph).  The
    final centralities are checked against a full recompute of the final graph."""
    import torch
    from paper_1701_05975_amd import bc, graphgen as gg
    from paper_1701_05975_amd.launch import LAUNCH

    g = gg.config_graph("ba100k")
    opts = bc.make_options(**LAUNCH["ba100k"])
    n = g.n
    G = bc.Graph(g)
    src = torch.arange(n, dtype=torch.int32, device="cuda")
    cur = torch.empty(n, dtype=torch.float64, device="cuda")
    bc.bc_compute_device(G.handle, src.data_ptr(), n, cur.data_ptr(), opts)  # warm-up
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bc.bc_compute_device(G.handle, src.data_ptr(), n, cur.data_ptr(), opts)
    torch.cuda.synchronize()
    full_ms = (time.perf_counter() - t0) * 1e3
    print(f"# full all-source BC {full_ms:.1f} ms", file=sys.stderr, flush=True)
    initial = cur.cpu().numpy()
    rows = []
    rng = np.random.default_rng(7)
    for i, kind in enumerate(["insert", "delete", "increase", "decrease"] * 2):
        change = gg.random_arc_change(g, kind, 1, 1000, seed=int(rng.integers(1 << 30)))
        t0 = time.perf_counter()
        g_new = gg.change_arc(g, *change)
        Gn = bc.Graph(g_new)
        t_build = time.perf_counter() - t0
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        k = bc.bc_update_arc_device(G.handle, Gn.handle, None, *change, cur.data_ptr(), 0, opts)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3
        row = {"change": kind, "arc": list(change), "affected_sources": k,
               "update_ms": round(ms, 1), "graph_build_ms": round(t_build * 1e3, 1)}
        rows.append(row)
        print(json.dumps(row), file=sys.stderr, flush=True)
        G.close()
        g, G = g_new, Gn
    full = torch.empty(n, dtype=torch.float64, device="cuda")
    bc.bc_compute_device(G.handle, src.data_ptr(), n, full.data_ptr(), opts)
    got, want = cur.cpu().numpy(), full.cpu().numpy()
    # each update's rounding is relative to the centralities it started from
    err = float(np.max(np.abs(got - want) /
                       np.maximum(np.maximum(np.abs(want), np.abs(initial)), 1.0)))
    mean_ms = float(np.mean([r["update_ms"] for r in rows]))
    print(json.dumps({
        "metric": "dynamic BC: ms per arc change (all-source BC kept current)",
        "value": round(mean_ms, 1), "unit": "ms", "higher_is_better": False,
        "median_ms": round(float(np.median([r["update_ms"] for r in rows])), 1),
        "full_recompute_ms": round(full_ms, 1), "speedup_vs_full": round(full_ms / mean_ms, 2),
        "mean_affected_fraction": round(float(np.mean([r["affected_sources"] for r in rows])) / n,
                                        4),
        "final_max_rel_dev_vs_full": err, "config": {"workload": WORKLOADS["dynamic"]},
        "rows": rows}), flush=True)
    assert err <= 1e-9, err


def run_serving(args):
    """Open-loop serving run: Poisson arrivals at the fixed rate stored with
    the launch settings (or calibrated with --calibrate), latency from arrival
    to completion measured inside the server; the first requests of the stream
    are warm-up and left out of the percentiles."""
    # sweeps of different graphs run on their own streams; give them hardware
    # queues of their own (HIP reads this before the runtime starts)
    os.environ.setdefault("GPU_MAX_HW_QUEUES", "8")
    import torch  # noqa: F401  (one HIP runtime for the process)
    from paper_1701_05975_amd import bc, graphgen as gg
    from paper_1701_05975_amd.launch import SERVING

    # least work first across graphs, a request overdue after starve_after_s
    # seconds first, and sweeps of 1024-thread workgroups (the batched form's
    # setting on the large graphs)
    serve_opts = dict(order=args.order, graph_order=1, starve_after_s=SERVING["starve_after_s"],
                      wg_threads=args.wg or 1024)
    nreq = args.requests or SERVING["requests"]
    warm = args.serve_warmup if args.serve_warmup >= 0 else SERVING["warmup"]
    if not 0 <= warm < nreq:
        raise SystemExit("serving: need 0 <= warm-up < requests")
    t0 = time.perf_counter()
    graphs = gg.serving_graphs()
    print(f"# generated 8 graphs in {time.perf_counter() - t0:.1f}s: " +
          ", ".join(f"{g.name}(n={g.n},m={g.m})" for g in graphs), file=sys.stderr, flush=True)
    G = [bc.Graph(g) for g in graphs]
    print("# graphs resident on the device", file=sys.stderr, flush=True)
    reqs = gg.serving_requests(graphs, nreq)
    work = np.array([len(s) * graphs[gi].m for gi, s in reqs], dtype=np.float64)
    if args.calibrate:
        # capacity: a prefix of the stream submitted at once and served closed loop
        ncal = min(nreq, 64)
        sv = bc.Server(**serve_opts)
        tw = time.perf_counter()
        ts = [sv.submit(G[gi], s) for gi, s in reqs[:ncal]]
        for (gi, s), t in zip(reqs[:ncal], ts):
            sv.wait(t, graphs[gi].n)
        cap = work[:ncal].sum() / (time.perf_counter() - tw)  # sources x edges per second
        sv.close()
        lam = args.load * cap / work.mean()
        print(json.dumps({"calibration": {"capacity_gteps": round(cap / 1e9, 4),
                                          "load": args.load, "mean_work": float(work.mean()),
                                          "rate_req_per_s": round(lam, 4),
                                          "requests": ncal}}), flush=True)
        return
    lam = args.rate if args.rate > 0 else SERVING["rate"]
    if lam <= 0:
        raise SystemExit("serving: no arrival rate stored; run with --calibrate first")
    print(f"# arrival rate {lam:.4f} req/s, {nreq} requests ({warm} warm-up)",
          file=sys.stderr, flush=True)
    # results kept for the mix-vs-alone check: requests spread over the measured part
    keep = set(np.linspace(warm, nreq - 1, min(args.serve_checks, nreq - warm))
               .round().astype(int).tolist())
    sv = bc.Server(**serve_opts)
    gaps = np.random.default_rng(201).exponential(1.0 / lam, size=nreq)
    # completions are collected (in submission order) by a second thread while
    # arrivals continue, so that finished results are released as they come
    import queue
    import threading
    pending = queue.Queue()
    lat = [0.0] * nreq
    results = {}
    failure = []

    def collect():
        try:
            for _ in range(nreq):
                i, gi, s, t = pending.get()
                out, ms = sv.wait(t, graphs[gi].n)
                lat[i] = ms
                print(f"# request {i}: graph {graphs[gi].name} k={len(s)} latency {ms:.1f} ms",
                      file=sys.stderr, flush=True)
                if i in keep:
                    results[i] = out
        except BaseException as e:  # reported by the main thread
            failure.append(e)

    waiter = threading.Thread(target=collect, daemon=True)
    waiter.start()
    start = time.perf_counter()
    arrivals = start + np.cumsum(gaps)
    for i, ((gi, s), ta) in enumerate(zip(reqs, arrivals)):
        dt = ta - time.perf_counter()
        if dt > 0:
            time.sleep(dt)
        pending.put((i, gi, s, sv.submit(G[gi], s)))
        if failure:
            break
    waiter.join()
    if failure:
        raise failure[0]
    wall = time.perf_counter() - start
    st = sv.stats()
    sv.close()
    # each kept result must equal the same request computed alone
    worst = 0.0
    for i, out in sorted(results.items()):
        gi, s = reqs[i]
        alone, _ = G[gi].bc(s)
        nz = alone != 0
        assert np.all(out[~nz] == 0), i
        if nz.any():
            worst = max(worst, float(np.max(np.abs(out[nz] - alone[nz]) / np.abs(alone[nz]))))
    assert worst <= 1e-9, worst
    print(f"# mix vs alone on {len(results)} requests: max rel err {worst:.2e}",
          file=sys.stderr, flush=True)
    meas = np.array(lat[warm:])
    rec = {
        "metric": "served BC request latency p50/p99 at a fixed Poisson rate; aggregate GTEPS",
        "value": round(float(np.percentile(meas, 50)), 2),
        "unit": "ms (p50)",
        "p50_ms": round(float(np.percentile(meas, 50)), 2),
        "p99_ms": round(float(np.percentile(meas, 99)), 2),
        "mean_ms": round(float(meas.mean()), 2),
        "max_ms": round(float(meas.max()), 2),
        "gteps": round(st["gteps"], 4),
        "offered_gteps": round(float(lam * work.mean() / 1e9), 4),
        "n_gpus": 1,
        "requests": nreq,
        "warmup_requests": warm,
        "measured_requests": int(meas.size),
        "rate_req_per_s": round(lam, 4),
        "wall_s": round(wall, 2),
        "higher_is_better": False,
        "sweeps": st["sweeps"],
        "mix_vs_alone_checked": len(results),
        "mix_vs_alone_max_rel_err": worst,
        "data": "synthetic (seeded generators)",
        "config": {"workload": f"serving: {WORKLOADS['serving']}",
                   "order": "fewest left first" if args.order == 1 else "oldest first",
                   "graph_order": "least work left first",
                   "starve_after_s": serve_opts["starve_after_s"],
                   "wg_threads": serve_opts["wg_threads"],
                   "graphs": [f"{g.name} n={g.n} m={g.m}" for g in graphs]},
    }
    print(json.dumps(rec), flush=True)


HBM_PEAK_GBS = 8000.0

def tuned_settings() -> dict:
    """Pinned launch settings per workload (shared with the full-size parity tests)."""
    from paper_1701_05975_amd.launch import LAUNCH
    return LAUNCH


MALL_BYTES = 256 << 20  # MI355X Infinity Cache


def copy_bandwidth_gbs(torch, stream, nbytes: int = 1 << 30, reps: int = 5) -> float:
    """Device-to-device copy rate on this GPU (read + write bytes per second,
    best of reps), the practical ceiling the roofline fraction is also
    reported against."""
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    best = 0.0
    with torch.cuda.stream(stream):
        for _ in range(reps):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            b.copy_(a)
            e1.record(stream)
            e1.synchronize()
            best = max(best, 2.0 * nbytes / (e0.elapsed_time(e1) * 1e-3) / 1e9)
    del a, b
    torch.cuda.empty_cache()
    return best


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ["kernels.hip", "passes.h", "dev_common.h", "shared_types.h", "kernels.h"]:
        with open(os.path.join(HERE, "paper_1701_05975_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profiled_traffic(config: str, key: str = "traffic_bytes_per_launch"):
    """HBM bytes per launch from the committed rocprofv3 counter summary of
    this workload (FETCH_SIZE scaled by the copy calibration, plus WRITE_SIZE;
    with key "traffic_unscaled_bytes_per_launch" the raw FETCH_SIZE, which
    counts 64 bytes per request), or None when the kernel sources changed
    since."""
    path = os.path.join(HERE, "profiles", f"k_batched_{config}.md")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        if ":" in line and not line.startswith(("|", "#")):
            name, _, val = line.partition(":")
            fields[name.strip()] = val.strip()
    if fields.get("kernel_source_hash") != kernel_source_hash():
        return None
    try:
        return float(fields[key])
    except (KeyError, ValueError):
        return None


def ensure_built():
    lib = os.path.join(HERE, "paper_1701_05975_amd", "libbcgpu.so")
    if not os.path.exists(lib):
        from paper_1701_05975_amd import build
        build.build()


def cpu_baseline(g, sources, target_s: float = 15.0, seed: int = 7):
    """The oracle timed on every host core over a seeded sample of the same
    source list: a first slice of one source per thread sizes a second slice
    so that the two together take about target_s seconds (capped at the whole
    list).  The oracle is compiled for this host (-O3 -march=native) into a
    temporary directory; the parity tests use the portable build."""
    import tempfile

    import oracle
    threads = oracle.host_threads()
    tmp = tempfile.mkdtemp(prefix="bc_oracle_")
    lib = oracle.build(extra_flags=("-march=native",), out=os.path.join(tmp, "liboracle.so"))
    rng = np.random.default_rng(seed)
    order = rng.permutation(np.asarray(sources, dtype=np.int32))
    k = order.shape[0]
    first = order[: min(threads, k)]
    t0 = time.perf_counter()
    oracle.oracle_bc(g, first, threads=threads, lib=lib)
    t1 = time.perf_counter() - t0
    done, total = first.shape[0], t1
    if done < k and t1 < target_s:
        more = int((target_s - t1) / max(t1, 1e-6)) * threads
        more = min(k - done, max(more, 0))
        if more > 0:
            t0 = time.perf_counter()
            oracle.oracle_bc(g, order[done: done + more], threads=threads, lib=lib)
            total += time.perf_counter() - t0
            done += more
    return {
        "value": round(done * g.m / total / 1e9, 6),
        "unit": "GTEPS",
        "cores": threads,
        "kind": "oracle",
        "extrapolated": done < k,
        "sample": f"{done} of the {k} sources (seed {seed}), {total:.2f} s wall on {threads} "
                  f"threads (every host core), gcc -O3 -march=native"
                  + ("; rate over the sample, applied to the whole list" if done < k else ""),
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="rmat22", choices=sorted(WORKLOADS))
    ap.add_argument("--plain-sources", type=int, default=64)
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="wall time the CPU-baseline sample aims at")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--autotune", action="store_true",
                    help="let the library's autotuner choose the settings during warm-up")
    ap.add_argument("--delta", type=int, default=0)
    ap.add_argument("--wg", type=int, default=0)
    ap.add_argument("--lane-max", type=int, default=0)
    ap.add_argument("--batch", type=int, default=0)
    ap.add_argument("--accumulate", type=int, default=0)
    ap.add_argument("--dep-mode", type=int, default=0)
    ap.add_argument("--lds-bits", type=int, default=0, help="LDS distance entry width (8, 16, 32)")
    ap.add_argument("--lds-vertices", type=int, default=0,
                    help="LDS-resident distances (-1: none; 0: as many as fit)")
    ap.add_argument("--far-buckets", type=int, default=0,
                    help="far values: 0 auto, 1 bucket ring, 2 two-tier pile")
    ap.add_argument("--edges", action="store_true",
                    help="time node + edge betweenness (bc_compute_edges_device)")
    ap.add_argument("--interleaved-sources", type=int, default=256,
                    help="sources timed in the source-interleaved form (0: skip)")
    ap.add_argument("--ablation-sources", type=int, default=256)
    ap.add_argument("--variants", default="", help="ablation: comma-separated name parts to run")
    ap.add_argument("--requests", type=int, default=0,
                    help="serving: requests in the run (0 = the stored setting, 512)")
    ap.add_argument("--order", type=int, default=1,
                    help="serving: 1 = fewest sources left first within a graph, 0 = oldest first")
    ap.add_argument("--serve-warmup", type=int, default=-1,
                    help="serving: warm-up requests left out of the percentiles (-1 = stored, 32)")
    ap.add_argument("--serve-checks", type=int, default=32,
                    help="serving: measured requests whose result is compared with a lone run")
    ap.add_argument("--calibrate", action="store_true",
                    help="serving: measure capacity and print the arrival rate for a load")
    ap.add_argument("--load", type=float, default=0.7, help="serving --calibrate: offered load")
    ap.add_argument("--rate", type=float, default=0.0,
                    help="serving: arrival rate (0 = the stored rate)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU form "
              "(sources sharded over GPUs, one all-reduce of the centralities) is not built.",
              file=sys.stderr)
        sys.exit(2)

    ensure_built()
    if args.config == "serving":
        run_serving(args)
        return
    if args.config == "ablation":
        run_ablation(args)
        return
    if args.config == "dynamic":
        run_dynamic(args)
        return
    import torch

    from paper_1701_05975_amd import bc, graphgen as gg

    t_gen = time.perf_counter()
    g = gg.config_graph(args.config)
    sources = gg.config_sources(args.config, g)
    t_gen = time.perf_counter() - t_gen
    print(f"# graph {g.name}: n={g.n} m={g.m} nnz={g.nnz} k={len(sources)} "
          f"(generated in {t_gen:.1f}s)", file=sys.stderr, flush=True)

    torch.cuda.init()
    stream = torch.cuda.current_stream()
    copy_gbs = copy_bandwidth_gbs(torch, stream)
    G = bc.Graph(g, edges=args.edges)
    src_dev = torch.from_numpy(sources).to("cuda")
    out = torch.empty(g.n, dtype=torch.float64, device="cuda")
    eout = torch.empty(max(g.nnz, 1), dtype=torch.float64, device="cuda") if args.edges else None
    k = int(len(sources))

    def run(o):
        if args.edges:
            return bc.bc_compute_edges_device(G.handle, src_dev.data_ptr(), k, out.data_ptr(),
                                              eout.data_ptr(), o)
        return bc.bc_compute_device(G.handle, src_dev.data_ptr(), k, out.data_ptr(), o)

    pinned = {} if args.autotune else tuned_settings().get(args.config, {})

    def opts(**kw):
        base = dict(delta=args.delta or pinned.get("delta", 0),
                    wg_threads=args.wg or pinned.get("wg_threads", 0),
                    lane_max_deg=args.lane_max or pinned.get("lane_max_deg", 0),
                    dep_mode=args.dep_mode or pinned.get("dep_mode", 0),
                    lds_bits=args.lds_bits or pinned.get("lds_bits", 0),
                    lds_vertices=args.lds_vertices or pinned.get("lds_vertices", 0),
                    batch=args.batch or pinned.get("batch", 0), accumulate=args.accumulate,
                    far_buckets=args.far_buckets or pinned.get("far_buckets", 0),
                    expand_lane_deg=pinned.get("expand_lane_deg", 0),
                    wave_max_deg=pinned.get("wave_max_deg", 0),
                    wg_min_deg=pinned.get("wg_min_deg", 0),
                    stream=stream.cuda_stream)
        base.update(kw)
        return bc.make_options(**base)

    # warm-up (with --autotune the first call searches and caches the settings)
    o = opts(autotune=1 if args.autotune else 0)
    for i in range(args.warmup):
        st = run(o)
        print(f"# warmup {i}: {st.ms:.1f} ms (delta={st.delta} wg={st.wg_threads} "
              f"lane_max={st.lane_max_deg} batch={st.batch} expand_lane_deg={st.expand_lane_deg} "
              f"wave_max_deg={st.wave_max_deg} wg_min_deg={st.wg_min_deg} "
              f"far_buckets={st.far_buckets})", file=sys.stderr, flush=True)

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for i in range(args.steps):
        st = run(o)
        stats.append(st)
        print(f"# step {i}: {st.ms:.1f} ms", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    ms_per_step = t / args.steps * 1e3
    gteps = k * g.m * args.steps / t / 1e9
    last = stats[-1]

    kernel_ms = float(np.mean([s.kernel_ms for s in stats]))
    achieved = last.algo_bytes / (kernel_ms * 1e-3) / 1e9
    # graph plus the distance arrays of the sources in flight: below the
    # Infinity Cache's size the HBM roofline does not bind
    working_set = G.info()["device_bytes"] + 4 * g.n * last.batch
    roofline = {
        "bound": "hbm",
        "achieved": round(achieved, 2),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 5),
        "traffic": profiled_traffic(args.config),
        "traffic_unscaled": profiled_traffic(args.config, "traffic_unscaled_bytes_per_launch"),
        "kernel": "k_batched",
        "kernel_ms": round(kernel_ms, 3),
        "algo_bytes_per_launch": last.algo_bytes,
        "copy_gbs": round(copy_gbs, 1),
        "frac_of_copy": round(achieved / copy_gbs, 5) if copy_gbs > 0 else None,
        "cache_resident": bool(working_set <= MALL_BYTES),
    }

    plain = None
    if not args.no_plain and not args.edges:
        ps = sources[: min(args.plain_sources, k)]
        ps_dev = torch.from_numpy(np.ascontiguousarray(ps)).to("cuda")
        po = opts(mode=bc.BC_MODE_PLAIN)
        bc.bc_compute_device(G.handle, ps_dev.data_ptr(), min(4, len(ps)), out.data_ptr(), po)
        torch.cuda.synchronize()
        tp0 = time.perf_counter()
        pst = bc.bc_compute_device(G.handle, ps_dev.data_ptr(), len(ps), out.data_ptr(), po)
        torch.cuda.synchronize()
        tp = time.perf_counter() - tp0
        plain = {"value": round(len(ps) * g.m / tp / 1e9, 6), "unit": "GTEPS",
                 "sources": int(len(ps)), "ms": round(tp * 1e3, 2),
                 "batched_over_plain": round(gteps / (len(ps) * g.m / tp / 1e9), 2)}

    interleaved = None
    if args.interleaved_sources > 0 and not args.edges:
        # the source-interleaved form (64 sources per wave) on the first sources
        isrc = sources[: min(args.interleaved_sources, k)]
        i_dev = torch.from_numpy(np.ascontiguousarray(isrc)).to("cuda")
        io = bc.make_options(mode=bc.BC_MODE_INTERLEAVED, stream=stream.cuda_stream)
        torch.cuda.synchronize()
        ti0 = time.perf_counter()
        ist = bc.bc_compute_device(G.handle, i_dev.data_ptr(), len(isrc), out.data_ptr(), io)
        torch.cuda.synchronize()
        ti = time.perf_counter() - ti0
        iv = len(isrc) * g.m / ti / 1e9
        interleaved = {"value": round(iv, 6), "unit": "GTEPS", "sources": int(len(isrc)),
                       "ms": round(ti * 1e3, 2), "delta": ist.delta, "rounds": ist.iterations,
                       "bands": ist.bands, "batched_over_interleaved": round(gteps / iv, 2)}
        print(f"# interleaved: {json.dumps(interleaved)}", file=sys.stderr, flush=True)

    cpu = None if args.no_cpu else cpu_baseline(g, sources, args.cpu_seconds)

    rec = {
        "metric": ("weighted node+edge BC GTEPS (sources x m / s), batched" if args.edges
                   else "weighted-BC GTEPS (sources x m / s), batched"),
        "value": round(gteps, 4),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "ms_median": round(float(np.median([s.ms for s in stats])), 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "i32/u64/f64",
        "data": "synthetic (seeded generator, paper-style random weights)",
        "config": {
            "workload": f"{args.config}: {WORKLOADS[args.config]}",
            "n": g.n, "m": g.m, "k": k,
            "delta": last.delta, "wg_threads": last.wg_threads, "lane_max_deg": last.lane_max_deg,
            "batch": last.batch, "accumulate": last.accumulate, "dep_mode": last.dep_mode,
            "lds_vertices": last.lds_vertices,
            "lds_bits": last.lds_bits, "far_buckets": last.far_buckets,
            "expand_lane_deg": last.expand_lane_deg, "wave_max_deg": last.wave_max_deg,
            "wg_min_deg": last.wg_min_deg,
            "reached": last.reached, "arcs_out_reached": last.arcs_out_reached,
            "dag_arcs": last.dag_arcs, "improvements": last.improvements,
            "bands": last.bands, "iterations": last.iterations,
            "sigma_rounds": last.sigma_rounds, "delta_rounds": last.delta_rounds,
            "phase_share": {k: round(v / max(1, sum(last.phase_ticks)), 4) for k, v in
                            zip(["init", "expand", "counts", "dependencies", "split"],
                                list(last.phase_ticks))},
        },
        "roofline": roofline,
        "plain": plain,
        "interleaved": interleaved,
        "cpu_baseline": cpu,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
