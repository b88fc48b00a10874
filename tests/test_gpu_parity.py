"""GPU parity: the HIP library against the oracle, element by element.

Registers and pass counts must be bit-exact; FP64 accumulators and
centralities must agree to 1e-12 relative (the implementation is designed to
be bit-identical, and the checks below report any inexact entry).
"""
import numpy as np
import pytest

import graphgen as gg
import oracle
from hbcheck import assert_fp, check, run_hb, run_oracle

pytestmark = pytest.mark.gpu


def _log(*a):
    print(*a, flush=True)


def test_rmat_s10_undirected_p16():
    # R-MAT scale 10, edge factor 8, undirected, int32 CSR, log2m = 4, seed 42.
    off, idx = gg.rmat(10, 8, seed=1, directed=False)
    _log("rmat s10 undirected n=1024 m=", len(idx))
    got, ref = check(off.astype(np.int32), idx, 4, 42, "s10")
    assert got["passes"] >= 3


def random_cases():
    yield "single", gg.empty(1)
    yield "pair", gg.from_edges(2, [(0, 1)])
    yield "self-loop", (np.array([0, 1], dtype=np.int64), np.array([0], dtype=np.int32))
    yield "isolated100", gg.empty(100)
    yield "cycle65", gg.directed_cycle(65)
    yield "path130", gg.directed_path(130)
    yield "star200", gg.star(200)
    for s, (n, m) in enumerate([(63, 200), (64, 64), (65, 500), (200, 50), (1000, 8000), (3001, 30000)]):
        yield f"rand{n}_{m}", gg.random_digraph(n, m, seed=10 + s, self_loops=bool(s % 2))
    yield "rmat12t", gg.rmat(12, 16, seed=7, transpose=True, relabel=True)
    yield "ba2000", gg.ba(2000, 4, seed=3)
    yield "ws2000", gg.ws(2000, 10, 0.1, seed=3)


@pytest.mark.parametrize("b", [4, 5, 6, 7, 8])
def test_parity_small_graphs(b):
    for name, (off, idx) in random_cases():
        _log("case", name, "b", b)
        check(off, idx, b, 1000 + b, f"{name}/b{b}")


def test_duplicate_arcs_and_unsorted_rows():
    # A CSR with repeated successors and unsorted rows is still a valid input.
    off = np.array([0, 4, 6, 6, 9], dtype=np.int64)
    idx = np.array([3, 1, 3, 1, 0, 0, 2, 1, 2], dtype=np.int32)
    for b in (4, 7):
        check(off, idx, b, 5, f"dups/b{b}")


def test_every_pass_matches():
    off, idx = gg.rmat(11, 8, seed=9, transpose=True, relabel=True)
    full = run_oracle(off, idx, 6, 77)
    for t in range(1, full["passes"] + 1):
        _log("pass", t)
        check(off, idx, 6, 77, f"t={t}", max_passes=t)


@pytest.mark.parametrize("opts", [
    dict(light_max=2, heavy_min=6, chunk=3),      # many heavy chunks
    dict(light_max=1, heavy_min=100000),          # every row with 2+ arcs is medium
    dict(light_max=4, heavy_min=40, chunk=17),
    dict(frontier=0),
    dict(frontier=0, light_max=2, heavy_min=6, chunk=5),
    dict(dense_pct=0),                            # every pass after the first is dense
    dict(dense_pct=0, qdense=1),                  # dense passes through the queued gather
    dict(dense_pct=101, sparse_pct=0),            # every pass after the first is an edge pass
    dict(dense_pct=101, sparse_pct=0, slice=1),   # edge passes with slice masks
    dict(dense_pct=101, sparse_pct=101),          # every pass after the first is sparse
    dict(dense_pct=101),                          # edge passes, then sparse ones
    dict(dense_pct=101, push=0),                  # edge passes only (no reverse CSR)
    dict(dense_pct=101, slice=1),                 # edge passes with slice masks, then sparse pair passes
    dict(dense_pct=101, sparse_pct=101, slice=1),  # sparse pair passes writing slice masks
    dict(dense_pct=101, sparse_pct=101, pairs=0),  # sparse passes from activation stamps
    dict(dense_pct=101, sparse_pct=101, pairs=0, light_max=2, heavy_min=6, chunk=3),
    dict(dense_pct=101, sparse_pct=0, slice=1, light_max=2, heavy_min=6, chunk=3),
    dict(dense_pct=101, sparse_pct=101, light_max=2, heavy_min=6, chunk=3),
    dict(slice=1),                                # default planning with slice masks
])
def test_parity_every_row_path(opts):
    graphs = [("rmat11", gg.rmat(11, 16, seed=4, transpose=True)),
              ("rmat10u", gg.rmat(10, 8, seed=5, directed=False)),
              ("star300", gg.star(300))]
    for name, (off, idx) in graphs:
        for b in (4, 6, 8):
            _log("opts", opts, name, "b", b)
            check(off, idx, b, 31, f"{name}/b{b}/{opts}", **opts)


def test_registers_before_the_first_pass_and_after_a_reset():
    """Registers read after a reset, before any pass, are every node's
    singleton counter; runs from a fresh context, after such a read and after
    a second reset all equal the oracle, heavy rows (merged from partial
    counters) and rows without successors included."""
    import paper_1308_2144_amd as hb

    off, idx = gg.rmat(9, 6, seed=3, transpose=True, relabel=True)
    n = len(off) - 1
    assert (np.diff(off) == 0).any() and np.diff(off).max() > 6
    for b in (5, 7):
        ref = run_oracle(off, idx, b, 17)
        init = np.stack([oracle.counter_of([v], b, 17) for v in range(n)])
        with hb.HyperBall(off, idx, b, 17, light_max=2, heavy_min=6, chunk=3) as g:
            g.run()
            assert np.array_equal(g.registers(), ref["regs"]), b
            g.reset(17)
            assert np.array_equal(g.registers(), init), b
            g.run()
            assert np.array_equal(g.registers(), ref["regs"]), b
            g.reset(17)
            g.run()
            assert np.array_equal(g.registers(), ref["regs"]), b
            assert np.array_equal(g.centralities()["harmonic"], ref["H"]), b


@pytest.mark.parametrize("b,n,m", [(9, 300, 2000), (10, 200, 1500), (12, 90, 600)])
def test_wide_counters(b, n, m):
    off, idx = gg.random_digraph(n, m, seed=b)
    check(off, idx, b, 11, f"wide b{b}")


def test_exact_regime_p65536():
    # p = 2^16, at most 48 nodes: linear counting is exact enough to recover
    # distance sums; the GPU must match the oracle bit for bit here too.
    for name, (off, idx) in [("cycle24", gg.directed_cycle(24)), ("grid", gg.grid(4, 6)),
                             ("rand", gg.random_digraph(40, 120, seed=2))]:
        check(off, idx, 16, 3, f"exact {name}")


def test_device_inputs_borrowed():
    import torch

    off, idx = gg.rmat(12, 8, seed=12, transpose=True, relabel=True)
    ref = run_oracle(off, idx, 7, 42)
    for bits in (32, 64):
        o = torch.from_numpy(off.astype(np.int32 if bits == 32 else np.int64)).cuda()
        i = torch.from_numpy(idx).cuda()
        got = run_hb(o, i, 7, 42)
        assert got["passes"] == ref["passes"]
        assert np.array_equal(got["regs"], ref["regs"])
        assert_fp(got["S"], ref["S"], "S")
        assert_fp(got["harmonic"], ref["harmonic"], "harmonic")
        want = off.astype(np.int32 if bits == 32 else np.int64)
        assert np.array_equal(o.cpu().numpy(), want)  # borrowed input left untouched


def test_device_centralities_and_stream():
    import torch

    import paper_1308_2144_amd as hb

    off, idx = gg.rmat(10, 8, seed=1, directed=False)
    ref = run_oracle(off, idx, 5, 8)
    s = torch.cuda.Stream()
    with hb.HyperBall(off, idx, 5, 8, stream=s.cuda_stream) as g:
        g.run()
        cen = g.centralities(device=True)
        for k in ("closeness", "lin", "harmonic", "coreach"):
            assert_fp(cen[k].cpu().numpy(), ref[k], k)


def test_edge_cases():
    import paper_1308_2144_amd as hb

    # n = 0
    with hb.HyperBall(np.zeros(1, dtype=np.int64), np.zeros(0, dtype=np.int32), 4, 1) as g:
        assert g.run() == 1 and g.iterate() == 0
        assert g.registers().shape == (0, 16)
    # converged contexts are inert; reset restarts with a new seed
    off, idx = gg.rmat(9, 8, seed=2, transpose=True)
    with hb.HyperBall(off, idx, 5, 100) as g:
        T = g.run()
        regs = g.registers()
        S, H = g.accumulators()
        assert g.iterate() == 0 and g.run() == T
        assert np.array_equal(g.registers(), regs)
        assert np.array_equal(g.accumulators()[0], S)
        g.reset(101)
        T2 = g.run()
        ref = run_oracle(off, idx, 5, 101)
        assert T2 == ref["passes"] and np.array_equal(g.registers(), ref["regs"])
        assert_fp(g.accumulators()[0], ref["S"], "S after reset")


def test_determinism():
    off, idx = gg.rmat(12, 16, seed=21, transpose=True)
    a = run_hb(off, idx, 6, 9, light_max=8, heavy_min=64, chunk=32)
    b = run_hb(off, idx, 6, 9, light_max=8, heavy_min=64, chunk=32)
    assert np.array_equal(a["regs"], b["regs"])
    assert np.array_equal(a["S"], b["S"]) and np.array_equal(a["H"], b["H"])


def test_pass_counters():
    off, idx = gg.rmat(11, 8, seed=4, transpose=True)
    m = len(idx)
    nonempty = int((np.diff(off) > 0).sum())
    b = 6
    G = (1 << b) // 16
    sparse = run_hb(off, idx, b, 3, dense_pct=101, sparse_pct=101)
    sliced = run_hb(off, idx, b, 3, dense_pct=101, sparse_pct=0, slice=1)
    edge = run_hb(off, idx, b, 3, dense_pct=101, sparse_pct=0)
    dense = run_hb(off, idx, b, 3, frontier=0)
    assert sparse["passes"] == dense["passes"] == sliced["passes"] == edge["passes"]
    # the arcs into counters changed by pass t are exactly what edge pass t+1 gathers
    es = edge["pass_stats"]
    for t in range(1, edge["passes"]):
        assert es[t]["mode"] == 4 and es[t]["counters_gathered"] == es[t - 1]["arcs_to_changed"]
        assert es[t]["slices_gathered"] == G * es[t]["counters_gathered"]
    for t, (a, b_, c) in enumerate(zip(sparse["pass_stats"], dense["pass_stats"], sliced["pass_stats"])):
        assert b_["mode"] == (0 if t == 0 else 1)
        assert a["mode"] == (0 if t == 0 else 2) and c["mode"] == (0 if t == 0 else 3)
        assert b_["arcs_scanned"] == m and b_["counters_gathered"] == m and b_["rows_loaded"] == nonempty
        # the first pass recomputes singleton counters instead of reading slices
        assert b_["slices_gathered"] == (0 if t == 0 else m * G)
        # slice passes scan every row but read a row's own counter only when a
        # changed slice turned up or the row changed before
        assert c["arcs_scanned"] == m and c["rows_changed"] <= c["rows_loaded"] <= nonempty
        assert c["slices_gathered"] <= G * c["counters_gathered"] and c["counters_gathered"] <= m
        assert a["arcs_scanned"] <= m and a["counters_gathered"] <= a["arcs_scanned"]
        assert a["rows_changed"] == b_["rows_changed"] == c["rows_changed"]
        assert a["slices_changed"] == b_["slices_changed"] == c["slices_changed"]
        assert b_["rows_changed"] <= b_["slices_changed"] <= G * b_["rows_changed"]
        assert a["rows_written"] >= a["rows_changed"]
        assert a["rows_loaded"] >= a["rows_changed"]
    assert sparse["pass_stats"][0]["counters_gathered"] == m
    assert sum(p["arcs_scanned"] for p in sparse["pass_stats"]) < sparse["passes"] * m
    assert sum(p["slices_gathered"] for p in sliced["pass_stats"]) < sliced["passes"] * m * G
    # the last pass visits only rows next to the previous pass's changes
    assert sparse["pass_stats"][-1]["rows_loaded"] < nonempty


def _k_medium_graph(n, k, seed):
    """n nodes; k rows of 2-40 successors (the medium rows when light_max is
    1), every other row 0 or 1 successor, all successors uniform."""
    rng = np.random.default_rng(seed)
    deg = rng.integers(0, 2, size=n)
    deg[rng.choice(n, size=k, replace=False)] = rng.integers(2, 41, size=k)
    off = np.zeros(n + 1, dtype=np.int64)
    off[1:] = np.cumsum(deg)
    idx = rng.integers(0, n, size=int(off[-1])).astype(np.int32)
    return off, idx


@pytest.mark.parametrize("k", [1, 3, 8, 9, 33])
def test_medium_rows_finished_together(k):
    """Medium rows are taken several to a wavefront (8, or 4 at p = 256) in
    first passes and in the queued passes of plain single-graph contexts, and
    finished together.  Ragged counts of medium rows, rows that skip a pass
    (sparse passes) and rows that keep their counter (lazy rows of edge
    passes), for every register count, in every pass mode: equal to the
    oracle."""
    off, idx = _k_medium_graph(400, k, 60 + k)
    for b in (4, 5, 6, 7, 8):
        for opts in (dict(), dict(dense_pct=0), dict(dense_pct=101, sparse_pct=0),
                     dict(dense_pct=101, sparse_pct=0, slice=1), dict(dense_pct=101, sparse_pct=101, pairs=0)):
            _log("k", k, "b", b, opts)
            got, _ = check(off, idx, b, 40 + b, f"k{k}/b{b}/{opts}", light_max=1, heavy_min=100000, **opts)
            assert got["pass_stats"][0]["mode"] == 0


@pytest.mark.parametrize("b", [4, 5, 6, 7, 8])
@pytest.mark.parametrize("opts", [dict(), dict(light_max=2, heavy_min=6, chunk=3),
                                  dict(light_max=1, heavy_min=100000), dict(light_max=4, heavy_min=40, chunk=17)])
def test_first_pass_from_hashes(b, opts):
    """Pass 0 of a plain context recomputes the successors' singleton counters
    from their hashes and folds them in LDS (light rows by lane groups, medium
    rows by wavefronts, heavy chunks by workgroups): equal to the oracle's
    pass 0, with no counter slice read."""
    for name, (off, idx) in [("rmat10t", gg.rmat(10, 12, seed=31, transpose=True)), ("star700", gg.star(700)),
                             ("rand3001", gg.random_digraph(3001, 30000, seed=32, self_loops=True)),
                             ("isolated70", gg.empty(70))]:
        got, _ = check(off, idx, b, 900 + b, f"{name}/b{b}/{opts}", max_passes=1, **opts)
        p0 = got["pass_stats"][0]
        assert p0["mode"] == 0 and p0["path"] == 1 and p0["slices_gathered"] == 0
        assert p0["counters_gathered"] == p0["arcs_scanned"] == len(idx)


def test_first_pass_reads_counters_when_weighted():
    """Weighted counters start with several items, so pass 0 gathers counter
    slices (only singletons are recomputed from hashes); the result equals the
    oracle's, and an unweighted reset afterwards recomputes them again."""
    import paper_1308_2144_amd as hb

    off, idx = gg.rmat(9, 8, seed=33, transpose=True)
    n = len(off) - 1
    w = np.random.default_rng(34).integers(1, 4, size=n).astype(np.int32)
    with hb.HyperBall(off, idx, 6, 5) as g:
        g.set_weights(w)
        g.reset(5)
        g.run(1)
        assert g.pass_stats(0)["slices_gathered"] == 4 * len(idx) and g.pass_stats(0)["path"] == 0
        regs = g.registers()
        g.set_weights(None)
        g.reset(5)
        g.run(1)
        assert g.pass_stats(0)["slices_gathered"] == 0
        plain = g.registers()
    ref = oracle.run_ext(off.astype(np.int64), idx, 6, 5, max_passes=1, weights=w)
    assert np.array_equal(regs, ref["regs"])
    assert np.array_equal(plain, oracle.run(off.astype(np.int64), idx, 6, 5, max_passes=1)["regs"])


@pytest.mark.parametrize("b", [4, 7, 8])
def test_sparse_pair_lists_long_runs(b):
    """Sparse passes from pair lists: the hub's 3000 successors all change in
    pass 0, so in pass 1 its run of 3000 pairs is cut into items whose
    partial counters are merged.  Equal to the oracle, and to the
    activation-stamp path, pass by pass."""
    k = 3000
    edges = [(0, i) for i in range(1, k + 1)] + [(i, k + i) for i in range(1, k + 1)]
    off, idx = gg.from_edges(2 * k + 1, edges)
    for opts in (dict(dense_pct=101, sparse_pct=101), dict(dense_pct=101, sparse_pct=101, pairs=0)):
        got, _ = check(off, idx, b, 77, f"hub{k}/b{b}/{opts}", **opts)
        modes = [p["mode"] for p in got["pass_stats"]]
        assert modes[0] == 0 and all(m == 2 for m in modes[1:]), modes
        paths = [p["path"] for p in got["pass_stats"][1:]]
        if opts.get("pairs", 1):
            # pair passes scan only arcs into changed counters
            assert all(p["arcs_scanned"] == p["counters_gathered"] for p in got["pass_stats"][1:])
            assert paths == [2] * len(paths)
        else:
            assert paths == [0] * len(paths)


def test_sparse_passes_mix_stamps_and_pair_lists():
    """R-MAT scale 15 (m + n > 2^16, so the pair lists hold (m + n) / 16
    pairs) with every pass after the first sparse: the early passes have
    more pairs than fit and run from activation stamps, the later ones from
    pair lists; the run equals the oracle pass by pass."""
    off, idx = gg.rmat(15, 16, seed=35, transpose=True, relabel=True)
    got, _ = check(off, idx, 6, 41, "rmat15 sparse", dense_pct=101, sparse_pct=101)
    paths = [p["path"] for p in got["pass_stats"][1:]]
    assert 0 in paths and 2 in paths, paths
    assert paths.index(2) > paths.index(0)


def test_validation_rejects_bad_indices():
    import paper_1308_2144_amd as hb

    off = np.array([0, 2, 3], dtype=np.int64)
    for bad in ([0, 2, 1], [0, -1, 1]):
        with pytest.raises(hb.HBError) as e:
            hb.HyperBall(off, np.array(bad, dtype=np.int32), 4, 1)
        assert e.value.status == hb.HB_EINVAL
    with pytest.raises(hb.HBError) as e:
        hb.HyperBall(np.array([0, 2, 1, 3], dtype=np.int64), np.array([0, 1, 2], dtype=np.int32), 4, 1)
    assert e.value.status == hb.HB_EINVAL
