#!/usr/bin/env python3
"""Writes the full-size expected values of the GPU parity tests.

Every value written here comes from the CPU oracle (``oracle/``) run on the
seeded inputs of ``graphgen/``; nothing else is imported.  Run on the CPU:

    python tests/golden/make_fullsize.py rmat-s24     # ~15 min, ~7 GB
    python tests/golden/make_fullsize.py batch-4096   # all 4096 graphs, parallel
    python tests/golden/make_fullsize.py serve-targets

Files written next to this script:

* ``fullsize_rmat-s24.txt`` - directed R-MAT scale 24, edge factor 16,
  generator seed 3, relabelled, transposed CSR, log2m 7, hash seed 42: the
  pass count, the counters changed by every pass, sha256 digests of the final
  registers (n*p bytes, node-major), of S and H and of the four finalized
  outputs (float64, little-endian), and the exact values (hex floats) at a
  seeded sample of nodes that includes every node changed in the last two
  passes, the heaviest rows and some degree-1 and empty rows.
* ``fullsize_batch-4096.txt`` - the 4096-graph batch (``graphgen.batch_workload``,
  hash seed 42+i): per graph its size, pass count and digests of its
  registers, S, H and of its per-pass change counts.
* ``fullsize_serve-targets.txt`` - the three served target requests of the
  serving workload's pool (largest with log2m 8, smallest with log2m 4, the
  middle one with log2m 6; hash seed 42+j for pool graph j): pass count,
  per-pass change counts and digests of registers, S, H and the finalized
  outputs.

Digests: sha256 over the raw bytes (uint8 registers; float64 little-endian).
The batch file truncates each digest to 16 hex digits; the change counts are
hashed as their decimal values joined by commas.
"""
from __future__ import annotations

import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import graphgen  # noqa: E402
import oracle  # noqa: E402

OUTS = ("closeness", "lin", "harmonic", "coreach")


def sha(a) -> str:
    a = np.ascontiguousarray(a)
    if a.dtype == np.float64:
        a = a.astype("<f8", copy=False)
    return hashlib.sha256(a.tobytes()).hexdigest()


def seq_sha(xs) -> str:
    return hashlib.sha256(",".join(str(int(x)) for x in xs).encode()).hexdigest()


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def rmat_s24():
    b, seed = 7, 42
    t = time.time()
    off, idx = graphgen.rmat(24, 16, seed=3, transpose=True, relabel=True)
    n, m = len(off) - 1, len(idx)
    log(f"s24: n={n} m={m} generated in {time.time() - t:.0f}s")
    t = time.time()
    r = oracle.run(off, idx, b, seed, lastmod=True)
    log(f"s24: oracle {r['passes']} passes in {time.time() - t:.0f}s, changes {list(r['nmod'])}")
    fin = oracle.finalize(r["regs"], b, r["S"], r["H"])
    T = r["passes"]
    lm = r["lastmod"]
    deg = np.diff(off)
    rng = np.random.default_rng(2024)
    pick = set(rng.choice(n, size=1024, replace=False).tolist())
    pick |= set(np.flatnonzero(lm >= T - 1).tolist())                 # changed in the last two passes
    late = np.flatnonzero(lm == T - 2)
    pick |= set(rng.choice(late, size=min(256, len(late)), replace=False).tolist())
    pick |= set(np.argsort(deg, kind="stable")[-16:].tolist())         # heaviest rows
    for d in (0, 1):
        cand = np.flatnonzero(deg == d)
        pick |= set(rng.choice(cand, size=min(16, len(cand)), replace=False).tolist())
    path = os.path.join(HERE, "fullsize_rmat-s24.txt")
    with open(path, "w") as f:
        f.write("# Oracle values for directed R-MAT scale 24, edge factor 16 (a,b,c,d = .57,.19,.19,.05),\n"
                "# generator seed 3, relabelled, transposed CSR, log2m 7, hash seed 42.\n"
                "# Written by tests/golden/make_fullsize.py rmat-s24 (oracle/ and graphgen/ only).\n"
                "# node lines: id lastmod S H closeness lin harmonic coreach (hex floats);\n"
                "# lastmod = 1 + the last pass that changed the node's counter (0: never).\n")
        f.write(f"n {n}\nm {m}\nlog2m {b}\nseed {seed}\npasses {T}\n")
        f.write("nmod " + " ".join(str(int(x)) for x in r["nmod"]) + "\n")
        f.write(f"sha256 registers {sha(r['regs'])}\n")
        f.write(f"sha256 S {sha(r['S'])}\nsha256 H {sha(r['H'])}\n")
        for k in OUTS:
            f.write(f"sha256 {k} {sha(fin[k])}\n")
        for v in sorted(pick):
            vals = [r["S"][v], r["H"][v]] + [fin[k][v] for k in OUTS]
            f.write(f"node {v} {int(lm[v])} " + " ".join(float(x).hex() for x in vals) + "\n")
    log(f"wrote {path}: {len(pick)} nodes")


def _batch_one(args):
    g, off, idx, seed = args
    r = oracle.run(off, idx, 5, seed)
    return (g, len(off) - 1, len(idx), r["passes"], sha(r["regs"])[:16], sha(r["S"])[:16], sha(r["H"])[:16],
            seq_sha(r["nmod"])[:16])


def batch_4096(workers: int):
    import multiprocessing as mp

    t = time.time()
    graphs = graphgen.batch_workload()
    k = len(graphs)
    log(f"batch: {k} graphs generated in {time.time() - t:.0f}s")
    # largest first, so that the pool drains evenly
    order = sorted(range(k), key=lambda g: -len(graphs[g][1]))
    jobs = [(g, graphs[g][0], graphs[g][1], 42 + g) for g in order]
    rows = {}
    t = time.time()
    with mp.get_context("fork").Pool(workers) as pool:
        for j, row in enumerate(pool.imap_unordered(_batch_one, jobs, chunksize=1)):
            rows[row[0]] = row
            if (j + 1) % 256 == 0:
                log(f"batch: {j + 1}/{k} graphs in {time.time() - t:.0f}s")
    path = os.path.join(HERE, "fullsize_batch-4096.txt")
    with open(path, "w") as f:
        f.write("# Oracle values for the 4096-graph batch (graphgen.batch_workload(): 2048 Barabasi-Albert\n"
                "# m=4 then 2048 Watts-Strogatz k=10 beta=0.1, n log-uniform in [1000, 200000], seed 4),\n"
                "# log2m 5, hash seed 42+g.  Written by tests/golden/make_fullsize.py batch-4096.\n"
                "# g n m passes sha256[:16](registers) sha256[:16](S) sha256[:16](H) sha256[:16](changes)\n")
        for g in range(k):
            f.write(" ".join(str(x) for x in rows[g]) + "\n")
    log(f"wrote {path}")


def serve_targets():
    """The serving workload's pool recipe: 32 graphs, scale U{10..20} and edge
    factor U{4..32} drawn with PCG64 seed 5, generator seed 1000+j,
    transposed."""
    rng = np.random.default_rng(5)
    pool = [(int(rng.integers(10, 21)), int(rng.integers(4, 33)), j) for j in range(32)]
    by_size = sorted(pool, key=lambda t: (t[0], t[1]))
    targets = [(by_size[-1], 8), (by_size[0], 4), (by_size[len(by_size) // 2], 6)]
    path = os.path.join(HERE, "fullsize_serve-targets.txt")
    with open(path, "w") as f:
        f.write("# Oracle values for the served target requests: pool graph j (directed R-MAT scale sc,\n"
                "# edge factor ef, generator seed 1000+j, transposed), log2m b, hash seed 42+j.\n"
                "# Written by tests/golden/make_fullsize.py serve-targets.\n"
                "# target j sc ef b n m passes; then nmod and sha256 lines for that target\n")
        for (sc, ef, j), b in targets:
            t = time.time()
            off, idx = graphgen.rmat(sc, ef, seed=1000 + j, transpose=True)
            r = oracle.run(off, idx, b, 42 + j)
            fin = oracle.finalize(r["regs"], b, r["S"], r["H"])
            log(f"serve target j={j} sc={sc} ef={ef} b={b}: {r['passes']} passes in {time.time() - t:.0f}s")
            f.write(f"target {j} {sc} {ef} {b} {len(off) - 1} {len(idx)} {r['passes']}\n")
            f.write("nmod " + " ".join(str(int(x)) for x in r["nmod"]) + "\n")
            f.write(f"sha256 registers {sha(r['regs'])}\nsha256 S {sha(r['S'])}\nsha256 H {sha(r['H'])}\n")
            for k in OUTS:
                f.write(f"sha256 {k} {sha(fin[k])}\n")
    log(f"wrote {path}")


def main():
    what = sys.argv[1:] or ["serve-targets", "batch-4096", "rmat-s24"]
    for w in what:
        if w == "rmat-s24":
            rmat_s24()
        elif w == "batch-4096":
            batch_4096(int(os.environ.get("GOLDEN_WORKERS", "6")))
        elif w == "serve-targets":
            serve_targets()
        else:
            raise SystemExit(f"unknown workload {w}")


if __name__ == "__main__":
    main()
