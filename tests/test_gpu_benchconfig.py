"""Parity in the configurations the benchmark times, at their full sizes:
sampled nodes evaluated one by one by the oracle's breadth-first path (the
counter of x after t passes is the HyperLogLog state of the ball B(x, t)),
plus properties that hold at any size.

* batched: the 4096-graph Barabasi-Albert / Watts-Strogatz batch, log2m 5,
  hash seeds 42+i, options from the committed autotuner cache: every graph's
  pass count and the digests of its registers, S and H against the whole
  oracle run of that graph (tests/golden/fullsize_batch-4096.txt, written by
  tests/golden/make_fullsize.py from the oracle alone); the same with the
  library's default options and with other forced configurations;
* serving: the largest, smallest and a middle request of the served R-MAT
  pool (scale 10..20, edge factor 4..32, log2m 4/6/8) in a mix: pass counts,
  and digests of registers, S, H and the finalized outputs against the whole
  oracle runs in tests/golden/fullsize_serve-targets.txt; the plain path's
  per-pass change counts against the same runs;
* ensemble: R-MAT scale 20, 8 seeds 42..49, log2m 4;
* weights + logarithmic discount + neighbourhood function: R-MAT scale 20,
  log2m 6, weights uniform in 1..4 (PCG64 seed 9).
"""
import math
import os

import numpy as np
import pytest

import graphgen as gg
import oracle
from hbcheck import CENTRALITIES, assert_fp, load_golden_batch, load_golden_targets, sha256_of

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _log(*a):
    print(*a, flush=True)


def _pick(off, k, seed):
    rng = np.random.default_rng(seed)
    n = len(off) - 1
    deg = np.diff(off)
    picks = set(rng.choice(n, size=min(k, n), replace=False).tolist())
    picks.add(int(np.argmax(deg)))
    return sorted(picks)


def _check_node(off, idx, b, seed, x, regs, S, H, what, D=None, **kw):
    q = oracle.node(off, idx, b, seed, x, **kw)
    assert np.array_equal(regs, q["regs"]), f"{what} node {x}: registers"
    assert_fp([S], [q["S"]], f"{what} S[{x}]")
    assert_fp([H], [q["H"]], f"{what} H[{x}]")
    if D is not None:
        assert_fp([D], [q["D"]], f"{what} D[{x}]")
    return q


@pytest.mark.timeout(900)
def test_batch_bench_config():
    import torch

    import paper_1308_2144_amd as hb

    graphs = gg.batch_workload()
    k = len(graphs)
    seeds = np.arange(k, dtype=np.uint64) + 42
    opt, rep = hb.hb_batch_autotune(graphs, 5, seeds, sample=256,
                                    cache_path=os.path.join(ROOT, "paper_1308_2144_amd", "tune_cache.txt"))
    _log("batch: autotune", rep)
    with hb.Batch(graphs, 5, seeds, options=opt) as bt:
        bt.run()
        passes = bt.passes()
        regs = torch.empty((bt.total, 32), dtype=torch.uint8, device="cuda")
        S = torch.empty(bt.total, dtype=torch.float64, device="cuda")
        H = torch.empty(bt.total, dtype=torch.float64, device="cuda")
        hb.hb_get_registers(bt._ctx, regs, True)
        hb.hb_get_accumulators(bt._ctx, S, H, True)
        bounds = bt.bounds
    assert np.all(passes > 0)
    sizes = np.array([len(o) - 1 for o, _ in graphs])
    gold = load_golden_batch("fullsize_batch-4096.txt")
    assert len(gold) == k
    bad = {"passes": [], "registers": [], "S": [], "H": []}
    regs_h, S_h, H_h = regs.cpu().numpy(), S.cpu().numpy(), H.cpu().numpy()
    for g in range(k):
        base, n = int(bounds[g]), int(sizes[g])
        ref = gold[g]
        assert (ref["n"], ref["m"]) == (n, len(graphs[g][1])), f"graph {g}: input differs from the golden's"
        if int(passes[g]) != ref["passes"]:
            bad["passes"].append(g)
        for key, arr in (("registers", regs_h), ("S", S_h), ("H", H_h)):
            if sha256_of(arr[base:base + n])[:16] != ref["regs" if key == "registers" else key]:
                bad[key].append(g)
    assert not any(bad.values()), {k: v[:10] for k, v in bad.items()}
    _log("batch: all", k, "graphs equal the oracle runs (pass counts, registers, S, H)")
    half = k // 2
    ba, ws = np.arange(half), np.arange(half, k)
    chosen = {int(ba[np.argmin(sizes[ba])]), int(ba[np.argmax(sizes[ba])]), int(ws[np.argmin(sizes[ws])]),
              int(ws[np.argmax(sizes[ws])]), 17, 3001}
    for g in sorted(chosen):
        off, idx = graphs[g]
        base, n = int(bounds[g]), int(sizes[g])
        what = f"graph {g} (n={n})"
        xs = _pick(off, 4, g)
        rows = torch.tensor([base + x for x in xs], device="cuda")
        r_regs, r_S, r_H = regs[rows].cpu().numpy(), S[rows].cpu().numpy(), H[rows].cpu().numpy()
        last = 0
        for j, x in enumerate(xs):
            q = _check_node(off, idx, 5, int(seeds[g]), x, r_regs[j], r_S[j], r_H[j], what)
            last = max(last, q["last_change"])
        assert passes[g] >= last + 1, what
        if n <= 5000:                           # whole-graph oracle run for the small ones
            ref = oracle.run(off.astype(np.int64), idx, 5, int(seeds[g]))
            assert passes[g] == ref["passes"], what
            assert np.array_equal(regs[base:base + n].cpu().numpy(), ref["regs"]), what
            assert_fp(S[base:base + n].cpu().numpy(), ref["S"], what + " S")
        _log("batch ok:", what, "passes", int(passes[g]))


@pytest.mark.timeout(900)
@pytest.mark.parametrize("opts", [
    dict(),                                          # library defaults, not the tuned ones
    dict(frontier=0),                                # every device pass dense
    dict(push=1, graph_passes=2, light_max=32),      # reverse CSR for sparse passes, other split
])
def test_batch_all_graphs_in_other_configurations(opts):
    """The 4096-graph batch with untuned and forced options: every graph's
    pass count and register, S and H digests equal its stored oracle run."""
    import paper_1308_2144_amd as hb

    graphs = gg.batch_workload()
    k = len(graphs)
    seeds = np.arange(k, dtype=np.uint64) + 42
    opt = hb.default_options(**opts)
    with hb.Batch(graphs, 5, seeds, options=opt) as bt:
        bt.run()
        passes = bt.passes()
        regs, S, H = bt.registers(), *bt.accumulators()
        bounds = bt.bounds
    gold = load_golden_batch("fullsize_batch-4096.txt")
    bad = []
    for g in range(k):
        base, n = int(bounds[g]), len(graphs[g][0]) - 1
        ref = gold[g]
        if (int(passes[g]) != ref["passes"] or sha256_of(regs[base:base + n])[:16] != ref["regs"]
                or sha256_of(S[base:base + n])[:16] != ref["S"] or sha256_of(H[base:base + n])[:16] != ref["H"]):
            bad.append(g)
    assert not bad, (opts, bad[:10])
    _log("batch", opts, ": all", k, "graphs equal the oracle runs")


@pytest.mark.timeout(900)
def test_serving_bench_config():
    import paper_1308_2144_amd as hb

    # the request pool recipe of the serving benchmark
    rng = np.random.default_rng(5)
    pool = []
    for j in range(32):
        sc, ef = int(rng.integers(10, 21)), int(rng.integers(4, 33))
        pool.append((sc, ef, j))
    by_size = sorted(pool, key=lambda t: (t[0], t[1]))
    targets = [(by_size[-1], 8), (by_size[0], 4), (by_size[len(by_size) // 2], 6)]
    mix = [by_size[i] for i in range(0, 32, 3)]
    graphs = {}
    for (sc, ef, j) in {t for t, _ in targets} | set(mix):
        off, idx = gg.rmat(sc, ef, seed=1000 + j, transpose=True)
        graphs[j] = (off.astype(np.int32), idx)
    with hb.Server(validate=0) as srv:
        reqs = []
        for i, (sc, ef, j) in enumerate(mix):             # background load
            reqs.append(srv.submit(*graphs[j], [4, 6, 8][i % 3], 1000 + i, outputs=("harmonic",)))
        tr = []
        for (sc, ef, j), b in targets:
            tr.append((j, b, srv.submit(*graphs[j], b, 42 + j, registers=True)))
        gold = {(t["j"], t["b"]): t for t in load_golden_targets("fullsize_serve-targets.txt")}
        for j, b, r in tr:
            info = srv.wait(r, 300.0)
            assert info["state_name"] == "done"
            off, idx = graphs[j]
            what = f"served pool graph {j} (n={len(off) - 1}, m={len(idx)}, log2m={b})"
            ref = gold[(j, b)]
            assert (ref["n"], ref["m"]) == (len(off) - 1, len(idx)), what
            assert info["passes"] == ref["passes"], (what, info["passes"], ref["passes"])
            out = r.outputs
            for key in ("registers", "S", "H") + CENTRALITIES:
                assert sha256_of(out[key]) == ref["sha256"][key], f"{what}: {key} differs from the oracle run"
            with hb.HyperBall(off, idx, b, 42 + j) as g:          # the plain path's per-pass changes
                assert g.run() == ref["passes"], what
                assert [g.pass_stats(t)["rows_changed"] for t in range(ref["passes"])] == ref["nmod"], what
            for x in _pick(off, 4, j):
                _check_node(off, idx, b, 42 + j, x, r.outputs["registers"][x], r.outputs["S"][x],
                            r.outputs["H"][x], what)
            _log("serve ok:", what, "passes", info["passes"], "latency ms", (info["t_done"] - info["t_submit"]) * 1e3)
        for r in reqs:
            assert srv.wait(r, 300.0)["state_name"] == "done"


@pytest.mark.timeout(900)
def test_ensemble_bench_config():
    import torch

    import paper_1308_2144_amd as hb

    off, idx = gg.rmat(20, 16, seed=2, transpose=True, relabel=True)     # the benchmark's graph
    seeds = [42 + k for k in range(8)]
    o = torch.from_numpy(off.astype(np.int32)).cuda()
    i = torch.from_numpy(idx).cuda()
    with hb.Ensemble(o, i, 4, seeds) as e:
        e.run()
        passes = e.passes()
        regs = e.registers()
        S, H = e.accumulators()
    xs = _pick(off, 3, 20)
    for k, sd in enumerate(seeds):
        last = 0
        for x in xs:
            q = _check_node(off, idx, 4, sd, x, regs[x, k], S[x, k], H[x, k], f"ensemble seed {sd}")
            last = max(last, q["last_change"])
        assert passes[k] >= last + 1
    with hb.HyperBall(o, i, 4, seeds[0]) as g:
        assert g.run() == passes[0]
        assert np.array_equal(g.registers(), regs[:, 0])
    _log("ensemble ok, passes", passes)


@pytest.mark.timeout(900)
def test_extensions_bench_config():
    import torch

    import paper_1308_2144_amd as hb

    off, idx = gg.rmat(20, 16, seed=2, transpose=True, relabel=True)     # the benchmark's graph
    n = len(off) - 1
    w = np.random.default_rng(9).integers(1, 5, size=n).astype(np.int32)
    table = hb.discount_table("logarithmic", 64)
    otable = oracle.discount_table("logarithmic", 64)
    o = torch.from_numpy(off.astype(np.int32)).cuda()
    i = torch.from_numpy(idx).cuda()
    with hb.HyperBall(o, i, 6, 42, neighbourhood=1) as g:
        g.set_weights(torch.from_numpy(w).cuda())
        g.set_discount(table)
        passes = g.run()
        regs = g.registers()
        S, H = g.accumulators()
        D = g.discounted()
        cen = g.centralities()
        N = g.neighbourhood()
    last = 0
    for x in _pick(off, 6, 21):
        q = _check_node(off, idx, 6, 42, x, regs[x], S[x], H[x], "extensions", D=D[x], weights=w, discount=otable)
        last = max(last, q["last_change"])
        fin = oracle.finalize(q["regs"][None, :], 6, np.array([q["S"]]), np.array([q["H"]]))
        for key in ("closeness", "lin", "harmonic", "coreach"):
            assert_fp([cen[key][x]], fin[key], f"extensions {key}[{x}]")
    assert passes >= last + 1 and len(N) == passes + 1
    # N(T) is the sum of the final estimates, correctly rounded (single
    # estimates may dip where linear counting hands over to the raw
    # estimator, so N is not asserted monotone pass by pass)
    assert N[-1] == math.fsum(cen["coreach"].tolist())
    assert N[0] < N[-1]
    _log("extensions ok, passes", passes, "N", N[:3], "...", N[-1])
