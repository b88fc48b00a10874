#!/usr/bin/env python3
"""HyperBall benchmark on one MI355X.

Workload (default): directed R-MAT, scale 24 (16,777,216 nodes), edge factor
16, (a,b,c,d) = (.57,.19,.19,.05), generator seed 3, nodes relabelled by a
seeded permutation, self-loops and duplicates removed, run on the transposed
CSR (int64 offsets, int32 indices), log2m = 7 (128 registers), hash seed 42,
modified-node frontier on.

One step = one whole HyperBall computation on that graph: reset (counters of
radius 0), passes until a pass changes no counter, and the centralities
written to device memory.  The graph is resident in HBM before timing starts.

Printed (one JSON line): `value` = edge visits per second, counting the arcs
each pass actually scans (a pass of the frontier skips rows none of whose
successors changed), summed over the passes of a step and divided by the step
time; beside it `nominal_edge_visits_per_s` = m x passes / step time, the
paper's time-per-arc convention (every arc counted in every pass).  Also the
roofline of the dominant kernel (algorithmic bytes per launch / mean launch
time from HIP events, against 8 TB/s; measured HBM traffic from committed
rocprofv3 counters, raw and scaled), and the CPU oracle timed on a sample of
the same graph (one core, and all cores).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "edge visits/s per iteration + % HBM peak (R-MAT s24); batched graphs/s vs plain"

WORKLOADS = {
    "rmat-s24": dict(scale=24, ef=16, gen_seed=3, log2m=7, offsets=64),
    # the same graph without the seeded relabelling (R-MAT's own id locality)
    "rmat-s24-raw": dict(scale=24, ef=16, gen_seed=3, log2m=7, offsets=64, relabel=False),
    "rmat-s20": dict(scale=20, ef=16, gen_seed=2, log2m=6, offsets=32),
    "rmat-s10u": dict(scale=10, ef=8, gen_seed=1, log2m=4, offsets=32, undirected=True),
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def make_graph(w):
    import graphgen

    t = time.time()
    if w.get("undirected"):
        off, idx = graphgen.rmat(w["scale"], w["ef"], seed=w["gen_seed"], directed=False)
    else:
        off, idx = graphgen.rmat(w["scale"], w["ef"], seed=w["gen_seed"], transpose=True,
                                 relabel=w.get("relabel", True))
    log(f"graph: n={len(off) - 1} m={len(idx)} generated in {time.time() - t:.1f}s")
    return off, idx


# Kernel launched by each pass mode (first, dense, sparse, slice, edge).
KERNEL_OF_MODE = {0: "k_expand<{b}>", 1: "k_expand<{b}>", 2: "k_expand_q<{b}>", 3: "k_expand_q<{b}>",
                  4: "k_expand_q<{b}>"}


def kernel_hash():
    """Hash of the kernel sources; HBM traffic figures are valid only for it."""
    h = hashlib.sha256()
    for f in ("hb_kernels.hip", "hb_internal.h"):
        h.update(open(os.path.join(ROOT, "paper_1308_2144_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def read_traffic(kname, workload):
    """HBM traffic per launch of `kname` from the committed rocprofv3 counter
    summary: the raw FETCH_SIZE and WRITE_SIZE (KiB per dispatch), the scale
    factors a plain device copy of known size gives them, and the scaled
    total in bytes; None if there is no summary for this kernel and workload
    or the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.txt")
    if not os.path.exists(path):
        return None
    rec = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            rec[k.strip()] = v.strip()
    if rec.get("kernel_hash") != kernel_hash() or rec.get("kernel") != kname:
        return None
    return {"bytes": int(rec["hbm_bytes_per_launch"]), "fetch_kib": float(rec["fetch_kib_per_launch"]),
            "write_kib": float(rec["write_kib_per_launch"]), "fetch_scale": float(rec["fetch_scale"]),
            "write_scale": float(rec["write_scale"])}


def kernel_of(ps, b):
    """Expand kernel of a pass: path 1 is the first pass from node hashes,
    path 2 a sparse pass from pair lists."""
    if ps["path"] == 1:
        return f"k_expand_codes<{b}>"
    if ps["path"] == 2:
        return f"k_pair_expand<{b}, 0>"
    return KERNEL_OF_MODE[ps["mode"]].format(b=b)


def pass_bytes(ps, listed, p):
    """Algorithmic HBM bytes of one pass's expand kernel.

    Every listed (non-empty) row: list entry, two offsets and its change-bit
    word (28 B; plus a 4 B activation stamp in sparse passes).  Every row
    that runs: own counter (p B) and the cached estimate and two accumulators
    (24 B).  Every scanned arc: its successor id (4 B).  Every gathered
    successor in a slice pass: its 2 B slice mask.  Every gathered 16-byte
    counter slice: 16 B.  Every written counter: p B.  Every changed row:
    estimate, accumulators and slice mask written back (26 B).  A first pass
    from node hashes reads no counter: its rows read only the estimate and
    accumulators, its arcs only the successor id.  A pair-list pass reads per
    row (run) a 32 B work item and no list entry, per pair a 4 B successor id."""
    per_row = 28 + (4 if ps["mode"] == 2 else 0)
    if ps["path"] == 1:
        return (per_row * listed + 24 * ps["rows_loaded"] + 4 * ps["arcs_scanned"]
                + p * ps["rows_written"] + 26 * ps["rows_changed"])
    if ps["path"] == 2:
        return ((32 + p + 24) * ps["rows_loaded"] + 4 * ps["arcs_scanned"] + 16 * ps["slices_gathered"]
                + p * ps["rows_written"] + 26 * ps["rows_changed"])
    per_arc = 4
    return (per_row * listed + (p + 24) * ps["rows_loaded"] + per_arc * ps["arcs_scanned"]
            + 16 * ps["slices_gathered"] + 2 * (ps["counters_gathered"] if ps["mode"] == 3 else 0)
            + p * ps["rows_written"] + 26 * ps["rows_changed"])


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(off, idx, w, seed, target_s: float = 20.0):
    """The oracle on a bounded sample of the benchmark graph itself: pass 0
    (every arc of a row gathered) over a contiguous range of rows, timed in a
    child process pinned to one core, then the OpenMP build of the same pass
    loop over the same rows on every core the process may use, checked equal
    to the single-core result.  Rows are in a random order (the graph is
    relabelled), so a range of rows is a uniform sample of them; the range is
    sized from a short calibration run to about target_s seconds on one
    core."""
    import subprocess
    import tempfile

    d = "/dev/shm" if os.path.isdir("/dev/shm") else None
    with tempfile.TemporaryDirectory(dir=d) as tmp:
        np.save(os.path.join(tmp, "off.npy"), np.asarray(off, dtype=np.int64))
        np.save(os.path.join(tmp, "idx.npy"), np.asarray(idx, dtype=np.int32))
        r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-baseline-child", tmp,
                            "--child-log2m", str(w["log2m"]), "--child-seed", str(seed),
                            "--child-target-s", str(target_s)],
                           stdout=subprocess.PIPE, check=True, text=True)
    res = json.loads(r.stdout.strip().splitlines()[-1])
    res["sample"] = (f"pass 0 of the {w.get('name', 'benchmark')} graph itself (log2m={w['log2m']}, hash seed {seed}) "
                     f"over rows [0, {res.pop('rows')}) of {res.pop('n')} ({res['arcs']} of {res.pop('m')} arcs), "
                     "C oracle built with gcc -O3 (no contraction, no fast-math); counters of every node set "
                     "to radius 0 first (not timed)")
    return res


def cpu_baseline_child(args):
    """Child process of cpu_baseline (no GPU use)."""
    import oracle

    off = np.load(os.path.join(args.cpu_baseline_child, "off.npy"))
    idx = np.load(os.path.join(args.cpu_baseline_child, "idx.npy"))
    n, m = len(off) - 1, len(idx)
    b, seed = args.child_log2m, args.child_seed
    allowed = sorted(os.sched_getaffinity(0))
    os.sched_setaffinity(0, {allowed[0]})
    cal_rows = max(1, n // 512)
    cal = oracle.first_pass_rows(off, idx, b, seed, 0, cal_rows)
    rate = max(int(off[cal_rows]), 1) / max(cal["seconds"], 1e-6)
    want_arcs = rate * args.child_target_s
    rows = int(np.searchsorted(off, min(want_arcs, m), side="left"))
    rows = min(max(rows, cal_rows), n)
    one = oracle.first_pass_rows(off, idx, b, seed, 0, rows)
    arcs = int(off[rows])
    os.sched_setaffinity(0, set(allowed))
    allc = oracle.first_pass_rows(off, idx, b, seed, 0, rows, all_cores=True)
    same = (one["changed"] == allc["changed"] and np.array_equal(one["next"], allc["next"])
            and np.array_equal(one["S"], allc["S"]) and np.array_equal(one["H"], allc["H"]))
    print(json.dumps({
        "value": arcs / one["seconds"], "unit": "edge visits/s", "cores": 1, "kind": "oracle",
        "seconds": round(one["seconds"], 2), "arcs": arcs, "rows": rows, "n": n, "m": m,
        "pinned_cpu": allowed[0], "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
        "usable_cpus": len(allowed),
        "all_cores": {"value": arcs / allc["seconds"], "unit": "edge visits/s", "cores": allc["threads"],
                      "seconds": round(allc["seconds"], 2), "identical_to_single_core": bool(same)}}),
        flush=True)


def bench_streamed(args, torch, hb, off, idx, w, seed, resident_ms, steps: int = 3,
                   budget: int = 512 << 20):
    """The same workload with the CSR kept in pinned host memory and streamed
    to the device in row chunks every pass (graph budget `budget` bytes: two
    staging buffers of budget/2), against the resident run: each step =
    reset + passes to convergence + centralities into device memory.  Run
    with the arcs as they are and kept compressed (decoded on the device),
    and a plain pinned-host-to-device copy of 1 GiB, the host link's
    reference rate."""
    n, m = len(off) - 1, len(idx)
    dev = torch.device("cuda:0")
    outs = [torch.empty(n, dtype=torch.float64, device=dev) for _ in range(4)]
    stream = torch.cuda.current_stream().cuda_stream

    def leg(compress):
        t = time.perf_counter()
        g = hb.HyperBall(off, idx, w["log2m"], seed, stream=stream, stream_graph=1, graph_budget=budget,
                         stream_compress=compress, timing=1)
        init_s = time.perf_counter() - t
        st = g.stats()

        def step():
            g.reset(seed)
            p = g.run()
            hb.hb_centralities(g._ctx, *outs, True)
            return p

        step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        host = 0
        scanned = 0
        for _ in range(steps):
            passes = step()
            ps = [g.pass_stats(t) for t in range(passes)]
            host += sum(p["host_bytes"] for p in ps)
            scanned += sum(p["arcs_scanned"] for p in ps)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        cen = [o.cpu() for o in outs]
        g.close()
        return cen, {"chunks": st["chunks"], "init_s": round(init_s, 2), "passes": passes,
                     "host_graph_bytes": st["host_graph_bytes"],
                     "chunks_run_per_pass": [p["chunks_run"] for p in ps],
                     "ms_per_step": dt * 1e3, "slowdown_vs_resident": dt * 1e3 / resident_ms,
                     "edge_visits_per_s": scanned / steps / dt,
                     "host_bytes_per_step": host // steps, "host_link_GBps": host / steps / dt / 1e9,
                     "pass_ms": [round(p["expand_ms"] + p["push_ms"], 3) for p in ps]}

    raw_cen, raw = leg(0)
    zip_cen, comp = leg(1)
    comp["centralities_identical_to_raw"] = all(torch.equal(a, b) for a, b in zip(raw_cen, zip_cen))
    comp["bytes_per_arc"] = round((comp["host_graph_bytes"] - 8 * (n + 1)) / max(m, 1), 3)
    del outs, raw_cen, zip_cen
    src = torch.empty(1 << 30, dtype=torch.uint8).pin_memory()
    dst = torch.empty(1 << 30, dtype=torch.uint8, device=dev)
    dst.copy_(src, non_blocking=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(3):
        dst.copy_(src, non_blocking=True)
    torch.cuda.synchronize()
    h2d = 3 * (1 << 30) / (time.perf_counter() - t0) / 1e9
    del src, dst
    return {"workload": f"{args.workload} with the CSR in pinned host memory, streamed in row chunks "
                        f"(graph budget {budget >> 20} MiB: two staging buffers of {budget >> 21} MiB)",
            **raw, "resident_ms_per_step": resident_ms, "h2d_copy_GBps": h2d,
            "compressed": comp}


def batch_roofline(recs, b):
    """Roofline of the batched dense passes (persistent k_expand_p<b, false>)
    from a pass-by-pass run: algorithmic bytes of each dense pass over the
    rows it ran (list entry, offsets and change word: 28 B; own counter and
    E, S, H: p + 24 B) and arcs scanned (id 4 B + successor counter p B),
    plus p B per counter written and 26 B per changed row, divided by the
    pass time (every kernel of the device pass, so a lower bound on the
    expand kernel's rate).  Measured HBM traffic per dispatch from the
    committed counters, when they match the kernel sources."""
    p = 1 << b
    dense = [r for r in recs if r["mode"] == 1]
    if not dense:
        return None
    byts = [(28 + p + 24) * r["rows_loaded"] + (4 + p) * r["arcs_scanned"] + p * r["rows_written"]
            + 26 * r["rows_changed"] for r in dense]
    ms = [r["expand_ms"] for r in dense]
    achieved = sum(byts) / (sum(ms) * 1e-3) / 1e9
    kname = f"k_expand_p<{b}, false>"
    tr = read_traffic(kname, "batch-4096")
    return {"bound": "hbm", "kernel": kname, "launches": len(dense), "achieved": round(achieved, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
            "algorithmic_bytes_per_launch": sum(byts) // len(dense), "mean_pass_ms": round(sum(ms) / len(ms), 4),
            "traffic": None if tr is None else tr["bytes"],
            "traffic_counters": None if tr is None else {k: tr[k] for k in ("fetch_kib", "write_kib", "fetch_scale",
                                                                            "write_scale")},
            "traffic_over_algorithmic": None if tr is None else round(tr["bytes"] / (sum(byts) / len(dense)), 3),
            "passes": [{"mode": r["mode"], "ms": round(r["expand_ms"], 3), "rows": r["rows_loaded"],
                        "arcs": r["arcs_scanned"], "changed": r["rows_changed"]} for r in recs]}


def bench_batch(args, torch, hb, plain_sample: int = 512):
    """Batched form on the 4096-graph workload: graphs/s of one batched
    context (reset + passes to convergence for every graph + centralities,
    inputs resident) against repeated plain per-graph runs on the same GPU,
    with identical results required."""
    import graphgen

    t = time.time()
    graphs = graphgen.batch_workload()
    k = len(graphs)
    seeds = np.arange(k, dtype=np.uint64) + 42
    b = 5
    log(f"batch: {k} graphs, n={sum(len(o) - 1 for o, _ in graphs)}, m={sum(len(i) for _, i in graphs)}, "
        f"generated in {time.time() - t:.1f}s")
    t = time.time()
    opt, tune = hb.hb_batch_autotune(graphs, b, seeds, sample=256, cache_path=args.tune_cache or None)
    tuned = hb.options_dict(opt)
    log(f"batch: autotune {tune} -> {tuned} in {time.time() - t:.1f}s")
    torch.cuda.synchronize()
    t = time.perf_counter()
    opt.timing = 1  # pass times for hb_iterate passes (no effect on hb_run's graph replays)
    bt = hb.Batch(graphs, b, seeds, options=opt)
    torch.cuda.synchronize()
    init_s = time.perf_counter() - t
    log(f"batch: context built in {init_s:.2f}s; stats {bt.stats()}")
    outs = [torch.empty(max(bt.total, 1), dtype=torch.float64, device="cuda") for _ in range(4)]

    def bstep():
        bt.reset()
        passes = bt.run()
        hb.hb_centralities(bt._ctx, *outs, True)
        return passes

    bstep()
    steps = max(args.steps, 2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        engine_passes = bstep()
    torch.cuda.synchronize()
    bdt = (time.perf_counter() - t0) / steps
    passes = bt.passes()
    regs = bt.split(bt.registers())
    harm = bt.split(outs[2].cpu().numpy())
    # One more run pass by pass (hb_iterate): every pass's work counts over
    # all graphs and its time (all kernels of the device pass, HIP events on
    # the batch's stream), for the roofline of the dense passes.
    bt.reset()
    while not hb.hb_stats(bt._ctx)["converged"]:
        hb.hb_iterate(bt._ctx)
    recs = [hb.hb_pass_stats(bt._ctx, t) for t in range(hb.hb_stats(bt._ctx)["passes"])]
    broof = batch_roofline(recs, b)
    bt.close()
    del outs
    row_opts = {}  # plain contexts keep the single-graph defaults (faster for them than the batch's tuning)
    # Plain runs: one context per graph (created before timing), each reset,
    # run and finalised in turn; a seeded sample of the graphs, scaled to all.
    rng = np.random.default_rng(7)
    sample = np.sort(rng.choice(k, size=min(plain_sample, k), replace=False))
    ctxs = []
    for i in sample:
        o, x = graphs[i]
        ctxs.append(hb.HyperBall(torch.from_numpy(o).cuda(), torch.from_numpy(x).cuda(), b, int(seeds[i]),
                                 stream=torch.cuda.current_stream().cuda_stream, **row_opts))
    pouts = [torch.empty(200_001, dtype=torch.float64, device="cuda") for _ in range(4)]
    plain_passes = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for j, i in enumerate(sample):
        g = ctxs[j]
        g.reset(int(seeds[i]))
        plain_passes.append(g.run())
        hb.hb_centralities(g._ctx, *pouts, True)
    torch.cuda.synchronize()
    pdt = (time.perf_counter() - t0) / len(sample) * k
    mismatch = {"passes": 0, "registers": 0, "harmonic": 0}
    for j, i in enumerate(sample):
        g = ctxs[j]
        mismatch["passes"] += int(plain_passes[j] != int(passes[i]))
        mismatch["registers"] += int(not np.array_equal(g.registers(), regs[i]))
        mismatch["harmonic"] += int(not np.array_equal(g.centralities()["harmonic"], harm[i]))
        g.close()
    identical = not any(mismatch.values())
    # Cold plain runs (init, passes, centralities, free) on a smaller sample.
    cold = sample[:min(64, len(sample))]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in cold:
        o, x = graphs[i]
        with hb.HyperBall(o, x, b, int(seeds[i]), **row_opts) as g:
            g.run()
            g.centralities()
    torch.cuda.synchronize()
    cdt = (time.perf_counter() - t0) / len(cold) * k
    return {"workload": "4096 graphs: 2048 Barabasi-Albert (m=4) + 2048 Watts-Strogatz (k=10, beta=0.1), "
                        "n log-uniform in [1000, 200000], log2m=5, hash seeds 42+i",
            "graphs": k, "batched_graphs_per_s": k / bdt, "batched_ms": bdt * 1e3,
            "init_s": init_s, "batched_graphs_per_s_with_init": k / (init_s + bdt),
            "engine_passes": int(engine_passes), "max_graph_passes": int(passes.max()),
            "plain_graphs_per_s": k / pdt, "plain_ms_estimated": pdt * 1e3,
            "plain_sample": int(len(sample)),
            "plain_cold_graphs_per_s": k / cdt, "plain_cold_sample": int(len(cold)),
            "speedup_vs_plain": pdt / bdt, "identical_on_sample": bool(identical),
            "autotune": {"options": {k: tuned[k] for k in ("light_max", "heavy_min", "chunk", "wgs_per_cu",
                                                            "graph_passes", "dense_pct", "sparse_pct", "qdense", "push")},
                         **tune},
            "mismatches_on_sample": mismatch, "roofline": broof}


def bench_ensemble(args, torch, hb, K: int = 8, b: int = 4, steps: int = 3):
    """Multi-seed ensemble: K hash seeds on R-MAT scale 20 (edge factor 16,
    transposed, gen seed 2) in one context against K plain runs one after
    another; inputs resident, each step = reset + passes to convergence +
    centralities and the ensemble summary into device memory."""
    w = WORKLOADS["rmat-s20"]
    off, idx = make_graph(w)
    n, m = len(off) - 1, len(idx)
    dev = torch.device("cuda:0")
    o = torch.from_numpy(off.astype(np.int32)).to(dev)
    x = torch.from_numpy(idx).to(dev)
    seeds = [42 + k for k in range(K)]
    stream = torch.cuda.current_stream().cuda_stream
    ens = hb.Ensemble(o, x, b, seeds, stream=stream)
    outs = [torch.empty(n * K, dtype=torch.float64, device=dev) for _ in range(4)]
    summ = [torch.empty(n, dtype=torch.float64, device=dev) for _ in range(2)]

    def estep():
        ens.reset(seeds)
        total = ens.run()
        hb.hb_centralities(ens._ctx, *outs, True)
        hb.hb_ensemble_summary(ens._ctx, "harmonic", *summ, True)
        return total

    estep()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        estep()
    torch.cuda.synchronize()
    edt = (time.perf_counter() - t0) / steps
    passes = ens.passes()
    eregs = ens.registers()
    ens.close()
    plain = hb.HyperBall(o, x, b, seeds[0], stream=stream)
    pouts = [torch.empty(n, dtype=torch.float64, device=dev) for _ in range(4)]
    ppasses = []
    same = True
    for k in range(K):  # warm-up and check
        plain.reset(seeds[k])
        ppasses.append(plain.run())
        same &= bool(np.array_equal(plain.registers(), eregs[:, k]))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        for k in range(K):
            plain.reset(seeds[k])
            plain.run()
            hb.hb_centralities(plain._ctx, *pouts, True)
    torch.cuda.synchronize()
    pdt = (time.perf_counter() - t0) / steps
    plain.close()
    same &= [int(v) for v in passes] == ppasses
    visits = m * int(np.sum(passes))
    return {"workload": f"R-MAT scale 20, edge factor 16, transposed, int32 CSR, log2m={b}, {K} seeds 42..{41 + K}",
            "n": n, "m": m, "seeds": K, "passes": [int(v) for v in passes],
            "ensemble_ms": edt * 1e3, "plain_ms": pdt * 1e3, "speedup_vs_plain": pdt / edt,
            "ensemble_edge_visits_per_s": visits / edt, "plain_edge_visits_per_s": visits / pdt,
            "identical": bool(same)}


def bench_extensions(args, torch, hb, steps: int = 3):
    """Cost of node weights (1..4), the logarithmic discount and the
    neighbourhood function on R-MAT scale 20 (edge factor 16, transposed,
    log2m 6), against the plain computation; inputs resident, each step =
    reset + passes + centralities (+ discounted sums and N(t))."""
    w = WORKLOADS["rmat-s20"]
    off, idx = make_graph(w)
    n, m = len(off) - 1, len(idx)
    dev = torch.device("cuda:0")
    o = torch.from_numpy(off.astype(np.int32)).to(dev)
    x = torch.from_numpy(idx).to(dev)
    stream = torch.cuda.current_stream().cuda_stream
    outs = [torch.empty(n, dtype=torch.float64, device=dev) for _ in range(5)]
    weights = torch.from_numpy(np.random.default_rng(9).integers(1, 5, size=n).astype(np.int32)).to(dev)
    res = {}
    for name in ("plain", "extended"):
        ext = name == "extended"
        g = hb.HyperBall(o, x, w["log2m"], 42, stream=stream, neighbourhood=int(ext))
        if ext:
            g.set_weights(weights)
            g.set_discount(hb.discount_table("logarithmic", 64))

        def step():
            g.reset(42)
            p = g.run()
            hb.hb_centralities(g._ctx, *outs[:4], True)
            if ext:
                hb.hb_get_discounted(g._ctx, outs[4], True)
                hb.hb_neighbourhood(g._ctx)
            return p

        step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            passes = step()
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        res[name] = {"ms": dt * 1e3, "passes": passes, "edge_visits_per_s": m * passes / dt}
        if ext:
            N = g.neighbourhood()
            res[name]["N_last"] = float(N[-1])
            res[name]["distance_stats"] = hb.hb_distance_stats(N)
        g.close()
    return {"workload": "R-MAT scale 20, edge factor 16, transposed, log2m=6; extended = node weights "
                        "uniform in 1..4 + logarithmic discount + neighbourhood function",
            **res, "overhead": res["extended"]["ms"] / res["plain"]["ms"] - 1.0}


class PinnedArena:
    """First-fit allocator over one pinned host buffer (result buffers of
    served requests, so that their copies run asynchronously)."""

    def __init__(self, torch, nbytes: int):
        self.buf = torch.empty(nbytes, dtype=torch.uint8).pin_memory()
        self.np = self.buf.numpy()
        self.free = [(0, nbytes)]

    def alloc(self, nbytes: int):
        nbytes = (nbytes + 255) // 256 * 256
        for k, (s, ln) in enumerate(self.free):
            if ln >= nbytes:
                self.free[k] = (s + nbytes, ln - nbytes)
                if self.free[k][1] == 0:
                    del self.free[k]
                return s, nbytes
        return None

    def release(self, s: int, nbytes: int):
        self.free.append((s, nbytes))
        self.free.sort()
        merged = []
        for a, ln in self.free:
            if merged and merged[-1][0] + merged[-1][1] == a:
                merged[-1] = (merged[-1][0], merged[-1][1] + ln)
            else:
                merged.append((a, ln))
        self.free = merged


SERVE_OUTS = ("closeness", "lin", "harmonic")


def serve_pool(torch, count: int, seed: int = 5):
    """Request pool of the serving workload: directed R-MAT graphs, scale
    uniform in 10..20, edge factor uniform in 4..32, transposed, int32 CSR,
    in pinned host memory."""
    import graphgen

    rng = np.random.default_rng(seed)
    pool = []
    for j in range(count):
        sc = int(rng.integers(10, 21))
        ef = int(rng.integers(4, 33))
        off, idx = graphgen.rmat(sc, ef, seed=1000 + j, transpose=True)
        o = torch.from_numpy(off.astype(np.int32)).pin_memory()
        x = torch.from_numpy(idx).pin_memory()
        pool.append(dict(scale=sc, ef=ef, n=len(off) - 1, m=len(idx), off=o.numpy(), idx=x.numpy(),
                         _t=(o, x)))
    return pool


def bench_serve(args, torch, hb, n_requests: int = 2000, rate: float = 500.0, pool_size: int = 32):
    """Serving form under Poisson arrivals: requests (pool graph, log2m in
    {4, 6, 8}, hash seed) arrive at `rate` per second; latency is arrival to
    outputs in host memory on the server's clock.  Also: throughput with all
    requests queued at once, repeated plain per-request runs on a sample, and
    a bit-for-bit check of served against plain outputs on a sample."""
    import threading

    t = time.time()
    pool = serve_pool(torch, pool_size)
    log(f"serve: pool of {pool_size} graphs, n={sum(g['n'] for g in pool)} m={sum(g['m'] for g in pool)}, "
        f"generated in {time.time() - t:.1f}s")
    rng = np.random.default_rng(5)
    gaps = rng.exponential(1.0 / rate, size=n_requests)
    arrivals = np.cumsum(gaps) - gaps[0]
    which = rng.integers(0, pool_size, size=n_requests)
    classes = rng.choice([4, 6, 8], size=n_requests)
    hseeds = rng.integers(0, 1 << 40, size=n_requests)
    arena = PinnedArena(torch, 4 << 30)
    # requests whose registers and finalized outputs are compared bit for bit
    # with a solo run (the pass counts of all of them are compared)
    check_ids = set(rng.choice(n_requests, size=min(200, n_requests), replace=False).tolist())

    def run_stream(times, tag):
        srv = hb.Server(validate=0)
        # engines (one per log2m) are created on first use: warm them up
        for b in (4, 6, 8):
            g = pool[0]
            srv.wait(srv.submit(g["off"], g["idx"], b, 1, outputs=()))
        st0 = srv.stats()
        done_q = []
        lock = threading.Lock()
        kept = {}
        infos = [None] * n_requests

        def waiter():
            while True:
                with lock:
                    item = done_q.pop(0) if done_q else None
                if item is None:
                    time.sleep(0.0002)
                    continue
                if item == "end":
                    return
                i, req, alloc = item
                infos[i] = srv.wait(req)
                if i in check_ids:
                    kept[i] = {k: v.copy() for k, v in req.outputs.items()}
                with lock:
                    arena.release(*alloc)

        th = threading.Thread(target=waiter)
        th.start()
        t0 = time.perf_counter()
        for i in range(n_requests):
            g = pool[which[i]]
            n = g["n"]
            rbytes = n << int(classes[i]) if i in check_ids else 0
            while True:
                with lock:
                    a = arena.alloc(24 * n + rbytes)
                if a is not None:
                    break
                time.sleep(0.0005)
            base = a[0]
            outs = {k: arena.np[base + 8 * n * j: base + 8 * n * (j + 1)].view(np.float64)
                    for j, k in enumerate(SERVE_OUTS)}
            if rbytes:
                outs["registers"] = arena.np[base + 24 * n: base + 24 * n + rbytes].reshape(n, -1)
            if times is not None:
                dt = times[i] - (time.perf_counter() - t0)
                if dt > 0.002:
                    time.sleep(dt - 0.001)
                while time.perf_counter() - t0 < times[i]:
                    pass
            req = srv.submit(g["off"], g["idx"], int(classes[i]), int(hseeds[i]), outputs=(), out=outs)
            with lock:
                done_q.append((i, req, a))
        with lock:
            done_q.append("end")
        th.join()
        st = srv.stats()
        srv.stop()
        lat = np.array([f["t_done"] - f["t_submit"] for f in infos]) * 1e3
        first = min(f["t_submit"] for f in infos)
        last = max(f["t_done"] for f in infos)
        window = last - first
        passes = np.array([f["passes"] for f in infos])
        visits = float(sum(pool[which[i]]["m"] * passes[i] for i in range(n_requests)))
        res = {"requests": n_requests, "graphs_per_s": n_requests / window, "window_s": window,
               "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
               "mean_ms": float(lat.mean()), "max_ms": float(lat.max()),
               "edge_visits_per_s": visits / window,
               "gpu_busy_frac": (st["busy_s"] - st0["busy_s"]) / window,
               "engine_passes": st["engine_passes"] - st0["engine_passes"],
               "request_passes": int(passes.sum()),
               "peak_resident_bytes": st["peak_resident_bytes"]}
        log(f"serve {tag}: {json.dumps(res)}")
        return res, infos, kept

    poisson, infos, kept = run_stream(arrivals, "poisson")
    burst, binfos, bkept = run_stream(None, "burst")
    # Plain: the same requests one after another through hb_init / hb_run /
    # hb_centralities / hb_free (host CSR, outputs to host), on a sample.
    sample = sorted(set(range(0, n_requests, max(1, n_requests // 100))))
    plain_t = 0.0
    for i in sample:
        g = pool[which[i]]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        with hb.HyperBall(g["off"], g["idx"], int(classes[i]), int(hseeds[i]), validate=0) as ctx:
            ctx.run()
            ctx.centralities()
        plain_t += time.perf_counter() - t0
    plain_gps = len(sample) / plain_t
    # Every request solo (one plain context per pool graph and log2m, reset
    # to the request's seed): its pass count against both served streams,
    # and for the checked requests registers and outputs bit for bit.
    mism = {"passes": 0, "registers": 0, "outputs": 0}
    t0 = time.perf_counter()
    order = sorted(range(n_requests), key=lambda i: (which[i], classes[i]))
    ctx, key = None, None
    for i in order:
        g = pool[which[i]]
        if key != (which[i], classes[i]):
            if ctx is not None:
                ctx.close()
            key = (which[i], classes[i])
            ctx = hb.HyperBall(g["off"], g["idx"], int(classes[i]), int(hseeds[i]), validate=0)
        ctx.reset(int(hseeds[i]))
        passes = ctx.run()
        mism["passes"] += int(passes != infos[i]["passes"]) + int(passes != binfos[i]["passes"])
        if i in check_ids:
            regs = ctx.registers()
            cen = ctx.centralities()
            for kk in (kept[i], bkept[i]):
                mism["registers"] += int(not np.array_equal(regs, kk["registers"]))
                mism["outputs"] += int(not all(np.array_equal(cen[k], kk[k]) for k in SERVE_OUTS))
    if ctx is not None:
        ctx.close()
    solo_s = time.perf_counter() - t0
    return {"workload": f"Poisson arrivals {rate:g}/s (seed 5), {n_requests} requests over a pool of "
                        f"{pool_size} directed R-MAT graphs (scale U{{10..20}}, edge factor U{{4..32}}, "
                        "transposed, int32 CSR, pinned host memory), log2m U{4,6,8}, budget 64 GiB",
            "poisson": poisson, "burst": burst,
            "plain_graphs_per_s": plain_gps, "plain_sample": len(sample),
            "burst_speedup_vs_plain": burst["graphs_per_s"] / plain_gps,
            "checked_pass_counts": 2 * n_requests, "checked_registers_and_outputs": 2 * len(check_ids),
            "solo_check_s": round(solo_s, 1), "mismatches": mism,
            "identical": not any(mism.values())}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="rmat-s24", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--light-max", type=int, default=0)
    ap.add_argument("--heavy-min", type=int, default=0)
    ap.add_argument("--chunk", type=int, default=0)
    ap.add_argument("--frontier", type=int, default=1)
    ap.add_argument("--dense-pct", type=int, default=-1)
    ap.add_argument("--push", type=int, default=1)
    ap.add_argument("--sparse-pct", type=int, default=-1)
    ap.add_argument("--qdense", type=int, default=0)
    ap.add_argument("--slice", type=int, default=0)
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-vs-plain measurement")
    ap.add_argument("--no-streamed", action="store_true", help="skip the host-streamed graph measurement")
    ap.add_argument("--plain-sample", type=int, default=512,
                    help="graphs of the batch also run one by one through plain contexts")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving measurement")
    ap.add_argument("--no-ensemble", action="store_true", help="skip the multi-seed ensemble measurement")
    ap.add_argument("--ensemble-only", action="store_true", help="only the ensemble measurement (its own line)")
    ap.add_argument("--no-extensions", action="store_true", help="skip the weights/discount/N(t) measurement")
    ap.add_argument("--tune-cache", default=os.path.join(ROOT, "paper_1308_2144_amd", "tune_cache.txt"),
                    help="autotuner cache of the batched form ('' for none: tune every run)")
    ap.add_argument("--batch-only", action="store_true", help="only the batched measurement (its own line)")
    ap.add_argument("--serve-only", action="store_true", help="only the serving measurement (its own line)")
    ap.add_argument("--copy-calib", action="store_true",
                    help="also run a plain 1 GiB device copy (torch) 3 times, to scale HBM counters")
    ap.add_argument("--cpu-baseline-child", default="", help=argparse.SUPPRESS)
    ap.add_argument("--child-log2m", type=int, default=7, help=argparse.SUPPRESS)
    ap.add_argument("--child-seed", type=int, default=42, help=argparse.SUPPRESS)
    ap.add_argument("--child-target-s", type=float, default=20.0, help=argparse.SUPPRESS)
    args = ap.parse_args()
    if args.cpu_baseline_child:
        cpu_baseline_child(args)
        return
    if args.gpus != 1:
        print(json.dumps({"error": "one GPU per run: sharding a graph over several GPUs is not implemented, so --gpus must be 1"}))
        sys.exit(2)

    import torch

    import paper_1308_2144_amd as hb

    if args.serve_only:
        print(json.dumps({"serving": bench_serve(args, torch, hb)}), flush=True)
        return
    if args.batch_only:
        print(json.dumps({"batched": bench_batch(args, torch, hb, plain_sample=args.plain_sample)}), flush=True)
        return
    if args.ensemble_only:
        print(json.dumps({"ensemble": bench_ensemble(args, torch, hb)}), flush=True)
        return
    w = WORKLOADS[args.workload]
    off, idx = make_graph(w)
    n, m = len(off) - 1, len(idx)
    p = 1 << w["log2m"]
    seed = 42
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    o_d = torch.from_numpy(off.astype(np.int64 if w["offsets"] == 64 else np.int32)).to(dev)
    i_d = torch.from_numpy(idx).to(dev)
    outs = [torch.empty(n, dtype=torch.float64, device=dev) for _ in range(4)]
    stream = torch.cuda.current_stream().cuda_stream
    g = hb.HyperBall(o_d, i_d, w["log2m"], seed, stream=stream, timing=1, frontier=args.frontier,
                     light_max=args.light_max, heavy_min=args.heavy_min, chunk=args.chunk,
                     dense_pct=args.dense_pct, push=args.push, sparse_pct=args.sparse_pct,
                     qdense=args.qdense, slice=args.slice)
    st0 = g.stats()
    listed = st0["light_rows"] + st0["medium_rows"] + st0["heavy_rows"]
    log(f"rows: light={st0['light_rows']} medium={st0['medium_rows']} heavy={st0['heavy_rows']} "
        f"chunks={st0['heavy_chunks']} reverse={st0['reverse_built']}")

    def step():
        g.reset(seed)
        passes = g.run()
        hb.hb_centralities(g._ctx, *outs, True)
        return passes

    for i in range(args.warmup):
        passes = step()
        log(f"warmup {i}: {passes} passes")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    step_passes = []
    scanned = 0
    per_kernel = {}  # kernel name -> [ms, algorithmic bytes, launches]
    first = None
    step_pass_ms = []  # per timed step: device time of each pass (push + expand + merge), ms
    for k in range(args.steps):
        passes = step()
        step_passes.append(passes)
        infos = [g.pass_stats(t) for t in range(passes)]
        step_pass_ms.append([ps["push_ms"] + ps["expand_ms"] + ps["merge_ms"] for ps in infos])
        scanned += sum(ps["arcs_scanned"] for ps in infos)
        for ps in infos:
            kname = kernel_of(ps, w["log2m"])
            acc = per_kernel.setdefault(kname, [0.0, 0, 0])
            acc[0] += ps["expand_ms"]
            acc[1] += pass_bytes(ps, listed, p)
            acc[2] += 1
        if first is None:
            first = infos
        log(f"step {k}: {passes} passes")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ms_per_step = 1e3 * dt / args.steps
    scanned_per_s = scanned / dt
    nominal = m * sum(step_passes)  # every arc of every pass, as the paper counts time per arc

    for t, ps in enumerate(first):
        log(f"  pass {t:2d} mode {ps['mode']}: arcs={ps['arcs_scanned']:>10d} "
            f"gathered={ps['counters_gathered']:>10d} slices={ps['slices_gathered']:>11d} "
            f"loaded={ps['rows_loaded']:>8d} "
            f"written={ps['rows_written']:>8d} changed={ps['rows_changed']:>8d} "
            f"sch={ps['slices_changed']:>9d} "
            f"push={ps['push_ms']:.3f} expand={ps['expand_ms']:.3f} merge={ps['merge_ms']:.3f} ms "
            f"{pass_bytes(ps, listed, p) / (ps['expand_ms'] * 1e6):.0f} GB/s")

    # Roofline of the dominant kernel (most total time).
    kname, (k_ms, k_bytes, launches) = max(per_kernel.items(), key=lambda kv: kv[1][0])
    mean_ms = k_ms / launches
    achieved = k_bytes / launches / (mean_ms * 1e-3) / 1e9
    tr = read_traffic(kname, args.workload)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None if tr is None else tr["bytes"],
            "traffic_counters": None if tr is None else {k: tr[k] for k in ("fetch_kib", "write_kib",
                                                                            "fetch_scale", "write_scale")},
            "kernel": kname, "launches": launches, "mean_launch_ms": round(mean_ms, 4),
            "algorithmic_bytes_per_launch": k_bytes // launches}
    others = {kn: {"launches": v[2], "mean_launch_ms": round(v[0] / v[2], 4),
                   "achieved_GBps": round(v[1] / v[2] / (v[0] / v[2] * 1e-3) / 1e9, 1)}
              for kn, v in per_kernel.items() if kn != kname}
    p0 = first[0]
    out = {
        "metric": METRIC, "value": scanned_per_s, "unit": "edge visits/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "m": m, "log2m": w["log2m"], "p": p,
                   "passes": step_passes[0], "frontier": bool(args.frontier), "hash_seed": seed,
                   "generator": "rmat a=.57 b=.19 c=.19 d=.05, gen seed %d" % w["gen_seed"],
                   "offsets": f"int{w['offsets']}"},
        "first_pass": {"ms": p0["expand_ms"] + p0["merge_ms"],
                       "edge_visits_per_s": m / ((p0["expand_ms"] + p0["merge_ms"]) * 1e-3),
                       "GBps": pass_bytes(p0, listed, p) / (p0["expand_ms"] * 1e6)},
        # Timing protocol: each pass's device time and the sum over a run's
        # passes, medians over the timed steps (every step runs the same passes).
        "pass_ms_median": [round(float(np.median([sp[t] for sp in step_pass_ms])), 4)
                           for t in range(min(len(sp) for sp in step_pass_ms))] if step_pass_ms else [],
        "passes_ms_median_of_run": round(float(np.median([sum(sp) for sp in step_pass_ms])), 4)
                                   if step_pass_ms else None,
        "nominal_edge_visits_per_s": nominal / dt,
        "arcs_scanned_per_step": scanned // args.steps,
        "roofline": roof,
        "other_kernels": others,
    }
    g.close()
    del o_d, i_d, outs
    torch.cuda.empty_cache()
    if not args.no_streamed:
        log("streamed graph ...")
        out["streamed"] = bench_streamed(args, torch, hb, off, idx, w, seed, ms_per_step)
        log(f"streamed: {out['streamed']}")
        torch.cuda.empty_cache()
    if not args.no_batch:
        log("batched form ...")
        out["batched"] = bench_batch(args, torch, hb, plain_sample=args.plain_sample)
        torch.cuda.empty_cache()
    if not args.no_extensions:
        log("weights, discount, neighbourhood function ...")
        out["extensions"] = bench_extensions(args, torch, hb)
        torch.cuda.empty_cache()
    if not args.no_ensemble:
        log("multi-seed ensemble ...")
        out["ensemble"] = bench_ensemble(args, torch, hb)
        torch.cuda.empty_cache()
    if not args.no_serve:
        log("serving form ...")
        out["serving"] = bench_serve(args, torch, hb)
        torch.cuda.empty_cache()
    if args.copy_calib:
        src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        cdt = (time.perf_counter() - t0) / 3
        out["copy_calib"] = {"bytes_read": 1 << 30, "bytes_written": 1 << 30, "ms": cdt * 1e3,
                             "GBps_rw": 2 * (1 << 30) / cdt / 1e9}
        del src, dst
        # Random row gathers of known size (torch index_select over 2 GiB of
        # 128-byte and 32-byte rows, 2^23 uniform row ids, int64): how
        # FETCH_SIZE counts scattered reads of counter-sized rows.
        table = torch.empty(1 << 31, dtype=torch.uint8, device=dev).fill_(1)
        for width in (128, 32):
            rows = table.view(-1, width)
            ids = torch.randint(0, rows.shape[0], (1 << 23,), device=dev, generator=torch.Generator(device=dev).manual_seed(11))
            got = torch.index_select(rows, 0, ids)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(3):
                got = torch.index_select(rows, 0, ids)
            torch.cuda.synchronize()
            gdt = (time.perf_counter() - t0) / 3
            out["copy_calib"][f"gather{width}"] = {"rows": 1 << 23, "row_bytes": width,
                                                   "bytes_read": (1 << 23) * (width + 8),
                                                   "bytes_written": (1 << 23) * width, "ms": gdt * 1e3}
            del got, ids
        del table
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle pass 0 on a sample of rows ...")
        out["cpu_baseline"] = cpu_baseline(off, idx, dict(w, name=args.workload), seed)
        log(f"cpu baseline: {out['cpu_baseline']}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
