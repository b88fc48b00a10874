"""Serving form: a request's outputs are the same alone and in a mix of
other requests that arrive, run and retire around it (different sizes,
log2m classes and pass counts), and both equal the plain single-graph
path bit for bit (and hence the oracle, checked directly on a few).

Limits are set small in some cases so that requests wait for budget, slots
and pool regions, and regions, slots and list segments are reused."""
import time

import numpy as np
import pytest

import graphgen as gg
from hbcheck import assert_fp, run_hb, run_oracle

pytestmark = pytest.mark.gpu

OUTS = ("closeness", "lin", "harmonic", "coreach", "S", "H")


def _log(*a):
    print(*a, flush=True)


def request_pool(seed=0, count=18):
    """Small stand-ins of the served workload (directed R-MAT, transposed,
    scale and edge factor drawn per request) plus degenerate graphs and one
    with a heavy row."""
    rng = np.random.default_rng(seed)
    out = [gg.empty(0), gg.empty(5), gg.from_edges(2, [(0, 1)]), gg.directed_cycle(70),
           gg.star(9000)]                              # centre row: 8999 arcs, cut into chunks
    while len(out) < count:
        sc = int(rng.integers(6, 13))
        ef = int(rng.integers(4, 33))
        out.append(gg.rmat(sc, ef, seed=int(rng.integers(1 << 30)), transpose=True))
    return out


def check_same(res, ref, what):
    assert res["passes"] == ref["passes"], (what, res["passes"], ref["passes"])
    assert np.array_equal(res["registers"], ref["regs"]), what + ": registers"
    for k in OUTS:
        assert_fp(res[k], ref[k], f"{what} {k}")


def serve_all(srv, graphs, classes, seeds, gap_s=0.0, order=None):
    order = range(len(graphs)) if order is None else order
    reqs = {}
    for i in order:
        off, idx = graphs[i]
        reqs[i] = srv.submit(off, idx, classes[i], seeds[i], registers=True)
        if gap_s:
            time.sleep(gap_s)
    out = {}
    for i, r in reqs.items():
        info = srv.wait(r, 120.0)
        assert info["state_name"] == "done", (i, info)
        out[i] = dict(r.outputs, passes=info["passes"], info=info)
        out[i]["registers"] = r.outputs["registers"]
    return out


def plain(graphs, classes, seeds):
    return [run_hb(off, idx, classes[i], seeds[i]) for i, (off, idx) in enumerate(graphs)]


@pytest.fixture(scope="module")
def workload():
    graphs = request_pool(1)
    rng = np.random.default_rng(2)
    classes = [int(c) for c in rng.choice([4, 6, 8], size=len(graphs))]
    classes[4] = 4                                     # the star under the cheapest class
    seeds = [int(s) for s in rng.integers(0, 1 << 40, size=len(graphs))]
    _log("workload:", [(len(o) - 1, len(x), c) for (o, x), c in zip(graphs, classes)])
    return graphs, classes, seeds, plain(graphs, classes, seeds)


def test_alone_equals_plain(workload):
    import paper_1308_2144_amd as hb

    graphs, classes, seeds, ref = workload
    for i in range(len(graphs)):
        with hb.Server() as srv:
            res = serve_all(srv, [graphs[i]], [classes[i]], [seeds[i]])[0]
            st = srv.stats()
        check_same(res, ref[i], f"alone {i}")
        assert st["completed"] == 1 and st["resident"] == 0 and st["resident_bytes"] == 0


@pytest.mark.parametrize("mode", ["burst", "staggered", "tight", "ticks3"])
def test_mix_equals_alone(workload, mode):
    import paper_1308_2144_amd as hb

    graphs, classes, seeds, ref = workload
    kw, gap = {}, 0.0
    order = list(range(len(graphs)))
    if mode == "staggered":
        gap = 0.002                                   # later requests join engines mid-flight
        order = order[::-1]
    elif mode == "tight":
        # requests wait for budget, slots and pool room; regions get reused
        biggest = max(2 * (len(o) - 1) * (1 << c) for (o, _), c in zip(graphs, classes))
        kw = dict(budget_bytes=biggest + 4096, max_resident=3, max_nodes=1 << 14, max_arcs=1 << 18)
    elif mode == "ticks3":
        kw = dict(passes_per_tick=3)
        gap = 0.001
    with hb.Server(**kw) as srv:
        t0 = time.time()
        res = serve_all(srv, graphs, classes, seeds, gap, order)
        st = srv.stats()
    _log(mode, f"{time.time() - t0:.3f}s", st)
    for i in range(len(graphs)):
        check_same(res[i], ref[i], f"{mode} {i}")
    assert st["completed"] == len(graphs) and st["resident"] == 0 and st["queued"] == 0
    assert st["peak_resident_bytes"] <= (kw.get("budget_bytes") or 64 << 30)
    if mode == "burst":
        assert st["peak_resident_bytes"] > 0 and st["engine_passes"] < sum(r["passes"] for r in ref)


def test_served_matches_oracle():
    import paper_1308_2144_amd as hb

    graphs = [gg.rmat(9, 8, seed=11, directed=False), gg.rmat(8, 16, seed=12, transpose=True)]
    classes, seeds = [4, 6], [42, 7]
    with hb.Server() as srv:
        res = serve_all(srv, graphs, classes, seeds)
    for i, (off, idx) in enumerate(graphs):
        ref = run_oracle(off, idx, classes[i], seeds[i])
        assert res[i]["passes"] == ref["passes"]
        assert np.array_equal(res[i]["registers"], ref["regs"])
        for k in OUTS:
            assert_fp(res[i][k], ref[k], f"oracle {i} {k}")


def test_many_small_requests_reuse_slots():
    """More requests than slots: every slot and region is used many times."""
    import paper_1308_2144_amd as hb

    rng = np.random.default_rng(9)
    graphs = [gg.random_digraph(int(rng.integers(1, 400)), int(rng.integers(0, 2000)), seed=k)
              for k in range(60)]
    seeds = [int(s) for s in rng.integers(0, 1 << 30, size=len(graphs))]
    classes = [5] * len(graphs)
    with hb.Server(max_resident=4, max_nodes=4096) as srv:
        res = serve_all(srv, graphs, classes, seeds, gap_s=0.0005)
        st = srv.stats()
    assert st["completed"] == len(graphs)
    for i, (off, idx) in enumerate(graphs):
        ref = run_hb(off, idx, 5, seeds[i])
        check_same(res[i], ref, f"small {i}")
