"""Batched form: many graphs in one context must give, graph by graph, the
same registers, pass counts and FP64 results as running each graph alone
(and hence as the oracle)."""
import numpy as np
import pytest

import graphgen as gg
from hbcheck import assert_fp, run_hb, run_oracle

pytestmark = pytest.mark.gpu


def _log(*a):
    print(*a, flush=True)


def mixed_graphs(seed=0, count=24):
    rng = np.random.default_rng(seed)
    out = [gg.empty(0), gg.empty(1), gg.from_edges(2, [(0, 1)]), gg.directed_cycle(70), gg.star(130)]
    while len(out) < count:
        kind = len(out) % 4
        n = int(rng.integers(50, 3000))
        s = int(rng.integers(1 << 30))
        if kind == 0:
            out.append(gg.ba(n, 4, seed=s))
        elif kind == 1:
            out.append(gg.ws(n, 10, 0.1, seed=s))
        elif kind == 2:
            out.append(gg.random_digraph(n, 6 * n, seed=s))
        else:
            sc = int(rng.integers(6, 12))
            out.append(gg.rmat(sc, 8, seed=s, transpose=True))
    return out


def compare_batch(graphs, b, seeds, max_passes=0, **opts):
    import paper_1308_2144_amd as hb

    with hb.Batch(graphs, b, seeds, **opts) as bt:
        bt.run(max_passes)
        regs = bt.split(bt.registers())
        S, H = (bt.split(x) for x in bt.accumulators())
        cen = {k: bt.split(v) for k, v in bt.centralities().items()}
        passes = bt.passes()
        infos = [bt.graph(i) for i in range(len(graphs))]
    for i, (off, idx) in enumerate(graphs):
        solo = run_hb(off, idx, b, int(seeds[i]), max_passes=max_passes, **opts)
        what = f"graph {i} (n={len(off) - 1})"
        if max_passes == 0:
            assert passes[i] == solo["passes"], (what, passes[i], solo["passes"])
            assert infos[i]["converged"] == 1 and infos[i]["n"] == len(off) - 1
        assert np.array_equal(regs[i], solo["regs"]), what
        assert_fp(S[i], solo["S"], what + " S")
        assert_fp(H[i], solo["H"], what + " H")
        for k in ("closeness", "lin", "harmonic", "coreach"):
            assert_fp(cen[k][i], solo[k], what + " " + k)


@pytest.mark.parametrize("b", [4, 5, 7, 8])
def test_batch_equals_solo(b):
    graphs = mixed_graphs(b)
    seeds = np.arange(len(graphs), dtype=np.uint64) + 42
    _log("batch of", len(graphs), "b", b)
    compare_batch(graphs, b, seeds)


@pytest.mark.parametrize("opts", [
    dict(light_max=2, heavy_min=6, chunk=3),
    dict(frontier=0),
    dict(dense_pct=101, sparse_pct=0),     # edge passes
    dict(dense_pct=101, sparse_pct=101),   # sparse passes
    dict(push=0, dense_pct=101),
])
def test_batch_row_paths_and_modes(opts):
    graphs = mixed_graphs(11, count=14)
    seeds = np.arange(len(graphs), dtype=np.uint64) * 7 + 1
    _log("opts", opts)
    compare_batch(graphs, 5, seeds, **opts)


@pytest.mark.parametrize("b", [4, 6, 8])
def test_batch_medium_rows_of_many_graphs(b):
    """Every row with 2+ arcs a medium row: first passes take several medium
    rows to a wavefront (8, or 4 at p = 256), rows of different graphs among
    them, each hashed with its own graph's seed and node numbering."""
    graphs = mixed_graphs(13, count=12)
    seeds = np.arange(len(graphs), dtype=np.uint64) * 3 + 11
    _log("medium rows, b", b)
    compare_batch(graphs, b, seeds, light_max=1, heavy_min=100000)


def test_batch_partial_runs_and_reset():
    import paper_1308_2144_amd as hb

    graphs = mixed_graphs(3, count=10)
    seeds = np.arange(10, dtype=np.uint64) + 5
    for t in (1, 2, 4):
        compare_batch(graphs, 6, seeds, max_passes=t)
    # reset with new seeds equals a fresh batch with those seeds
    seeds2 = seeds + 100
    with hb.Batch(graphs, 6, seeds) as bt:
        bt.run()
        bt.reset(seeds2)
        bt.run()
        regs = bt.split(bt.registers())
        passes = bt.passes()
    for i, (off, idx) in enumerate(graphs):
        ref = run_oracle(off, idx, 6, int(seeds2[i]))
        assert passes[i] == ref["passes"] and np.array_equal(regs[i], ref["regs"]), i


def test_batch_against_oracle_directly():
    graphs = mixed_graphs(7, count=8)
    seeds = np.arange(8, dtype=np.uint64) * 3 + 9
    import paper_1308_2144_amd as hb

    with hb.Batch(graphs, 5, seeds) as bt:
        bt.run()
        regs = bt.split(bt.registers())
        cen = {k: bt.split(v) for k, v in bt.centralities().items()}
        passes = bt.passes()
    for i, (off, idx) in enumerate(graphs):
        ref = run_oracle(off, idx, 5, int(seeds[i]))
        assert passes[i] == ref["passes"]
        assert np.array_equal(regs[i], ref["regs"])
        for k in ("closeness", "lin", "harmonic", "coreach"):
            assert_fp(cen[k][i], ref[k], f"{i} {k}")


def test_batch_device_outputs_are_packed_and_bounded():
    # Device destinations get the packed layout (sum of n_i entries) and
    # nothing past it: a guard region after the packed size stays untouched.
    import torch

    import paper_1308_2144_amd as hb

    graphs = mixed_graphs(5, count=12)
    seeds = np.arange(12, dtype=np.uint64) + 77
    with hb.Batch(graphs, 6, seeds) as bt:
        bt.run()
        total = bt.total
        guard = 4096
        outs = [torch.full((total + guard,), -7.0, dtype=torch.float64, device="cuda") for _ in range(4)]
        hb.hb_centralities(bt._ctx, *outs, True)
        host = bt.centralities()
        for o, key in zip(outs, ("closeness", "lin", "harmonic", "coreach")):
            o = o.cpu().numpy()
            assert np.array_equal(o[:total], host[key]), key
            assert np.all(o[total:] == -7.0), key
        S = torch.full((total + guard,), -7.0, dtype=torch.float64, device="cuda")
        H = torch.full((total + guard,), -7.0, dtype=torch.float64, device="cuda")
        hb.hb_get_accumulators(bt._ctx, S, H, True)
        hS, hH = bt.accumulators()
        assert np.array_equal(S.cpu().numpy()[:total], hS) and np.all(S.cpu().numpy()[total:] == -7.0)
        assert np.array_equal(H.cpu().numpy()[:total], hH) and np.all(H.cpu().numpy()[total:] == -7.0)
        R = torch.full(((total + guard) * bt.p,), 251, dtype=torch.uint8, device="cuda")
        hb.hb_get_registers(bt._ctx, R, True)
        R = R.cpu().numpy()
        assert np.array_equal(R[: total * bt.p].reshape(total, bt.p), bt.registers())
        assert np.all(R[total * bt.p:] == 251)


def test_autotune_picks_candidates_and_caches(tmp_path):
    """The tuner returns options from its candidate sets, a second call with
    the same batch is served from the cache, and a batch built with the tuned
    options still equals solo runs."""
    import paper_1308_2144_amd as hb

    graphs = mixed_graphs(seed=5, count=40)
    seeds = np.arange(len(graphs), dtype=np.uint64) + 3
    cache = str(tmp_path / "tune.txt")
    opt, rep = hb.hb_batch_autotune(graphs, 5, seeds, sample=16, cache_path=cache)
    _log("autotune:", rep, hb.options_dict(opt))
    assert rep["from_cache"] == 0 and rep["candidates"] > 10 and rep["sample_graphs"] == 16
    assert rep["best_ms"] <= rep["start_ms"]
    assert opt.light_max in (16, 32, 64, 128, 256) and opt.heavy_min > opt.light_max
    assert opt.wgs_per_cu in (2, 3, 4, 5, 6, 8) and opt.graph_passes in (1, 2, 4, 8, 16)
    opt2, rep2 = hb.hb_batch_autotune(graphs, 5, seeds, sample=16, cache_path=cache)
    assert rep2["from_cache"] == 1 and hb.options_dict(opt2) == hb.options_dict(opt)
    tuned = hb.options_dict(opt)
    compare_batch(graphs, 5, seeds, **{k: tuned[k] for k in ("light_max", "heavy_min", "chunk", "wgs_per_cu",
                                                            "graph_passes", "dense_pct", "sparse_pct", "qdense")})


def test_mostly_empty_batches():
    """Empty graphs beside one non-empty graph: the batch equals solo runs, and
    an autotune sample of one graph takes the non-empty graph (a batch of empty
    graphs only is refused at init)."""
    import paper_1308_2144_amd as hb

    graphs = [gg.empty(0), gg.empty(0), gg.empty(5), gg.directed_cycle(70), gg.empty(0)]
    seeds = np.arange(len(graphs), dtype=np.uint64) + 11
    compare_batch(graphs, 5, seeds)
    opt, rep = hb.hb_batch_autotune([gg.empty(0)] * 6 + [gg.star(40)], 5, np.arange(7, dtype=np.uint64), sample=1)
    _log("autotune:", rep)
    assert rep["sample_graphs"] == 1


def test_batch_pass_records_equal_the_oracle_sums():
    """Passes run one by one (hb_iterate) keep per-pass records on a batched
    context: pass t's changed counters are the sum over the graphs of the
    oracle's changes in their pass t, and a dense pass scans every arc of
    the graphs that have not converged."""
    import paper_1308_2144_amd as hb

    graphs = mixed_graphs(seed=7, count=16)
    b = 5
    seeds = np.arange(len(graphs), dtype=np.uint64) + 3
    refs = [run_oracle(o, x, b, int(s)) for (o, x), s in zip(graphs, seeds)]
    with hb.Batch(graphs, b, seeds, timing=1) as bt:
        while not hb.hb_stats(bt._ctx)["converged"]:
            hb.hb_iterate(bt._ctx)
        T = hb.hb_stats(bt._ctx)["passes"]
        recs = [hb.hb_pass_stats(bt._ctx, t) for t in range(T)]
        assert list(bt.passes()) == [r["passes"] for r in refs]
    assert T == max(r["passes"] for r in refs)
    for t, rec in enumerate(recs):
        want = sum(int(r["nmod"][t]) for r in refs if t < r["passes"])
        assert rec["rows_changed"] == want, (t, rec["rows_changed"], want)
        if rec["mode"] == 1:
            arcs = sum(len(x) for (o, x), r in zip(graphs, refs) if t < r["passes"])
            assert rec["arcs_scanned"] == arcs, t
        assert rec["expand_ms"] > 0.0
    _log("batch pass records:", [(r["mode"], r["rows_changed"]) for r in recs])
