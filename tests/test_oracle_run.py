"""Pins for the oracle's HyperBall loop (Sec. 4.2 Algorithm 2, Sec. 5, Sec. 3).

The recurrence is pinned to its definition: after t passes, the counter of x
is exactly the HyperLogLog state of the ball B(x, t), with balls computed by
scipy's breadth-first shortest paths (independent of the oracle).  The
accumulators and centralities are pinned to exact distance sums on graphs in
the exact-counting regime (p = 2^16, at most ~48 nodes), and to closed forms
on cycles, paths, stars and complete graphs.
"""
import math

import numpy as np
import pytest
from scipy.sparse import csr_matrix
from scipy.sparse.csgraph import shortest_path


def bfs_dist(offsets, indices):
    n = offsets.shape[0] - 1
    A = csr_matrix((np.ones(indices.shape[0]), indices, offsets), shape=(n, n))
    return shortest_path(A, method="D", directed=True, unweighted=True)


def ball_counters(orc, D, b, seed, t):
    n = D.shape[0]
    out = np.zeros((n, 1 << b), dtype=np.uint8)
    for x in range(n):
        out[x] = orc.counter_of(np.flatnonzero(D[x] <= t), b, seed)
    return out


def small_graphs(gg):
    yield "path", gg.directed_path(9)
    yield "cycle", gg.directed_cycle(11)
    yield "star", gg.star(10)
    yield "grid", gg.grid(4, 5)
    yield "empty", gg.empty(6)
    for s in range(6):
        n = [12, 20, 33, 40, 50, 64][s]
        m = [10, 30, 60, 120, 80, 400][s]
        yield f"rand{s}", gg.random_digraph(n, m, seed=100 + s, self_loops=(s % 2 == 1))
    yield "rmat6", gg.rmat(6, 4, seed=5, transpose=True)
    yield "rmat6u", gg.rmat(6, 4, seed=6, directed=False)


@pytest.mark.parametrize("b", [4, 5, 7])
def test_counters_are_hll_of_balls(orc, gg, b):
    seed = 42 + b
    for name, (o, i) in small_graphs(gg):
        D = bfs_dist(o, i)
        full = orc.run(o, i, b, seed)
        T = full["passes"]
        for t in range(1, T + 1):
            r = orc.run(o, i, b, seed, max_passes=t)
            assert np.array_equal(r["regs"], ball_counters(orc, D, b, seed, t)), (name, t)
        # radius 0 through the per-node path: {x}
        for x in range(min(5, D.shape[0])):
            assert np.array_equal(orc.node(o, i, b, seed, x, radius=0)["regs"],
                                  orc.counter_of([x], b, seed))


@pytest.mark.parametrize("b", [4, 6])
def test_termination_count(orc, gg, b):
    # Algorithm 2 stops after the first pass that changes no counter; that
    # pass is counted.  From balls: passes = 1 + max_x L(x), where L(x) is
    # the last t with HLL(B(x,t)) != HLL(B(x,t-1)).
    seed = 9
    for name, (o, i) in small_graphs(gg):
        D = bfs_dist(o, i)
        n = D.shape[0]
        finite = D[np.isfinite(D)]
        diam = int(finite.max()) if finite.size else 0
        prev = ball_counters(orc, D, b, seed, 0)
        L = np.zeros(n, dtype=int)
        for t in range(1, diam + 1):
            cur = ball_counters(orc, D, b, seed, t)
            L[(cur != prev).any(axis=1)] = t
            prev = cur
        r = orc.run(o, i, b, seed)
        expect = 1 + (int(L.max()) if n else 0)
        assert r["passes"] == expect, name
        assert r["passes"] <= diam + 1
        assert r["nmod"][-1] == 0 and (r["nmod"][:-1] > 0).all()
        # the per-node evaluation reports the same L(x)
        for x in range(n):
            assert orc.node(o, i, b, seed, x)["last_change"] == L[x]


def test_node_evaluation_matches_run_bitwise(orc, gg):
    for b in (4, 6, 8):
        for name, (o, i) in small_graphs(gg):
            r = orc.run(o, i, b, 77)
            n = o.shape[0] - 1
            for x in range(n):
                q = orc.node(o, i, b, 77, x)
                assert q["S"] == r["S"][x] and q["H"] == r["H"][x], (name, x)
                assert np.array_equal(q["regs"], r["regs"][x])


def exact_seed(orc, n, b=16):
    # a seed for which the n node ids fill n distinct registers
    for seed in range(1000):
        if np.count_nonzero(orc.counter_of(range(n), b, seed)) == n:
            return seed
    raise AssertionError("no collision-free seed")


def test_accumulators_match_exact_distances(orc, gg):
    # With p = 2^16 and <= 64 nodes, counters count exactly (no collisions),
    # so S ~ sum of distances, H ~ sum of reciprocal distances, coreach ~
    # reachable-set size (Sec. 5), up to the linear-counting bias k^2/2p.
    b = 16
    for name, (o, i) in small_graphs(gg):
        n = o.shape[0] - 1
        seed = exact_seed(orc, n)
        D = bfs_dist(o, i)
        r = orc.run(o, i, b, seed)
        f = orc.finalize(r["regs"], b, r["S"], r["H"])
        for x in range(n):
            d = D[x][np.isfinite(D[x]) & (D[x] > 0)]
            S, H, R = d.sum(), (1.0 / d).sum(), 1 + d.size
            tol = 2e-3 * max(1.0, S)
            assert abs(r["S"][x] - S) < tol, (name, x)
            assert abs(r["H"][x] - H) < 2e-3 * max(1.0, H), (name, x)
            assert abs(f["coreach"][x] - R) < 2e-3 * R, (name, x)
            if d.size == 0:
                assert r["S"][x] == 0.0 and f["closeness"][x] == 0.0 and f["lin"][x] == 1.0
            else:
                assert abs(f["closeness"][x] - 1.0 / S) < 3e-3 / S
                assert abs(f["lin"][x] - R * R / S) < 6e-3 * R * R / S
            assert f["harmonic"][x] == r["H"][x]


def test_closed_forms(orc, gg):
    b = 16
    # directed cycle C_n: every node reaches the n-1 others at distances 1..n-1
    n = 24
    o, i = gg.directed_cycle(n)
    r = orc.run(o, i, b, exact_seed(orc, n))
    f = orc.finalize(r["regs"], b, r["S"], r["H"])
    Hn = sum(1.0 / k for k in range(1, n))
    assert np.allclose(r["S"], n * (n - 1) / 2, rtol=3e-3)
    assert np.allclose(r["H"], Hn, rtol=3e-3)
    assert np.allclose(f["coreach"], n, rtol=3e-3)
    assert r["passes"] == n  # distances up to n-1, plus the unchanged pass
    # complete digraph K_n: S = H = n-1, two passes
    n = 30
    o, i = gg.complete(n)
    r = orc.run(o, i, b, exact_seed(orc, n))
    assert np.allclose(r["S"], n - 1, rtol=3e-3) and np.allclose(r["H"], n - 1, rtol=3e-3)
    assert r["passes"] == 2
    # undirected star: centre S = H = n-1; leaf S = 2n-3, H = 1 + (n-2)/2
    n = 20
    o, i = gg.star(n)
    r = orc.run(o, i, b, exact_seed(orc, n))
    assert abs(r["S"][0] - (n - 1)) < 3e-3 * n and abs(r["H"][0] - (n - 1)) < 3e-3 * n
    assert np.allclose(r["S"][1:], 2 * n - 3, rtol=3e-3)
    assert np.allclose(r["H"][1:], 1 + (n - 2) / 2, rtol=3e-3)
    # directed path 0->1->...->n-1: node 0 has S = n(n-1)/2, the sink S = 0
    n = 16
    o, i = gg.directed_path(n)
    r = orc.run(o, i, b, exact_seed(orc, n))
    f = orc.finalize(r["regs"], b, r["S"], r["H"])
    assert abs(r["S"][0] - n * (n - 1) / 2) < 3e-3 * n * n
    assert r["S"][-1] == 0.0 and f["closeness"][-1] == 0.0 and f["lin"][-1] == 1.0


def test_graph_without_arcs(orc, gg):
    for b in (4, 8):
        o, i = gg.empty(7)
        r = orc.run(o, i, b, 1)
        assert r["passes"] == 1 and (r["S"] == 0).all() and (r["H"] == 0).all()
        f = orc.finalize(r["regs"], b, r["S"], r["H"])
        p = 1 << b
        assert np.all(f["coreach"] == p * math.log(p / (p - 1)))
    o, i = gg.empty(0)
    assert orc.run(o, i, 4, 1)["passes"] == 1


def test_invariants_on_rmat(orc, gg):
    # Registers never decrease; a pass that reports a change changed some
    # register; once a pass changes nothing, further passes change nothing.
    o, i = gg.rmat(9, 8, seed=11, transpose=True)
    b = 5
    full = orc.run(o, i, b, 3)
    prev = orc.run(o, i, b, 3, max_passes=1)["regs"]
    for t in range(2, full["passes"] + 3):
        cur = orc.run(o, i, b, 3, max_passes=t)["regs"]
        assert (cur >= prev).all()
        nchg = int((cur != prev).any(axis=1).sum())
        if t <= full["passes"]:
            assert nchg == full["nmod"][t - 1]
        else:
            assert nchg == 0
        prev = cur


def test_ensemble_summary_against_numpy_and_closed_forms(orc):
    rng = np.random.default_rng(3)
    for K in (2, 4, 8, 16):
        x = rng.lognormal(2.0, 1.0, size=(500, K))
        m, sd = orc.ensemble_summary(x)
        assert np.allclose(m, x.mean(axis=1), rtol=1e-14, atol=0)
        assert np.allclose(sd, x.std(axis=1, ddof=1), rtol=1e-12, atol=1e-300)
    # equal integer values (every partial sum exact): mean exact, spread exactly zero
    x = np.repeat(rng.integers(1, 1 << 20, size=(50, 1)).astype(np.float64), 8, axis=1)
    m, sd = orc.ensemble_summary(x)
    assert np.array_equal(m, x[:, 0]) and np.all(sd == 0.0)
    # two values a, b: sd = |a - b| / sqrt(2)
    a, b = rng.lognormal(size=200), rng.lognormal(size=200)
    m, sd = orc.ensemble_summary(np.stack([a, b], axis=1))
    assert np.allclose(sd, np.abs(a - b) / np.sqrt(2.0), rtol=1e-14)
    # arithmetic progression c, c+h, ..., c+(K-1)h: sd = h * sqrt(K (K+1) / 12)
    for K in (4, 16):
        c, h = 10.0, 0.5
        x = (c + h * np.arange(K))[None, :].repeat(3, axis=0)
        m, sd = orc.ensemble_summary(x)
        assert np.allclose(m, c + h * (K - 1) / 2, rtol=1e-15)
        assert np.allclose(sd, h * np.sqrt(K * (K + 1) / 12.0), rtol=1e-14)


def test_ensemble_is_independent_runs(orc, gg):
    off, idx = gg.rmat(7, 8, seed=5, transpose=True)
    runs = orc.ensemble(off, idx, 4, [3, 9])
    for sd, r in zip([3, 9], runs):
        ref = orc.run(off, idx, 4, sd)
        assert r["passes"] == ref["passes"] and np.array_equal(r["regs"], ref["regs"])
    assert not np.array_equal(runs[0]["regs"], runs[1]["regs"])   # different seeds differ


def exact_replica_seed(orc, weights, b=16):
    # a seed for which all replicas of all nodes fill distinct registers
    items = [orc.replica_item(x, j) for x in range(len(weights)) for j in range(int(weights[x]))]
    for seed in range(2000):
        if np.count_nonzero(orc.counter_of(items, b, seed)) == len(items):
            return seed
    raise AssertionError("no collision-free seed")


def test_run_ext_reduces_to_run(orc, gg):
    off, idx = gg.rmat(8, 8, seed=31, transpose=True)
    n = len(off) - 1
    a = orc.run(off, idx, 6, 5)
    table = [float(d) for d in range(1, 40)]
    b = orc.run_ext(off, idx, 6, 5, weights=np.ones(n, dtype=np.int32), discount=table, trace=True)
    assert a["passes"] == b["passes"] and np.array_equal(a["regs"], b["regs"])
    assert np.array_equal(a["S"], b["S"]) and np.array_equal(a["H"], b["H"])
    assert np.array_equal(b["D"], b["S"])          # f(d) = d is S's own weighting, same arithmetic
    # the trace's last row is the size of the final counters
    fin = orc.finalize(a["regs"], 6, a["S"], a["H"])
    assert np.array_equal(b["etrace"][-1], fin["coreach"])
    assert b["etrace"].shape == (a["passes"] + 1, n)


def test_weighted_counter_is_hll_of_replicas(orc, gg):
    n = 9
    o, i = gg.empty(n)
    w = np.array([1, 2, 3, 5, 8, 1, 1, 4, 2], dtype=np.int32)
    r = orc.run_ext(o, i, 7, 13, weights=w)
    for x in range(n):
        items = [orc.replica_item(x, j) for j in range(w[x])]
        assert np.array_equal(r["regs"][x], orc.counter_of(items, 7, 13))


def test_weights_and_discounts_match_exact_distances(orc, gg):
    # Sec. 6 and Sec. 7 in the exact-counting regime: S ~ sum_y w(y) d(x,y),
    # H ~ sum_y w(y)/d(x,y), D ~ sum_y w(y) f(d(x,y)), coreach ~ sum of the
    # weights of the reachable set (x included).
    b = 16
    rng = np.random.default_rng(17)
    tables = {"quadratic": [1.0 / d ** 2 for d in range(1, 65)],
              "logarithmic": [1.0 / math.log2(d + 1) for d in range(1, 65)],
              "short": [1.0, 0.5, 0.25]}                     # f(d) = 1/4 beyond d = 3
    for name, (o, i) in small_graphs(gg):
        n = o.shape[0] - 1
        w = rng.integers(1, 4, size=n).astype(np.int32)
        seed = exact_replica_seed(orc, w)
        Dist = bfs_dist(o, i)
        for tname, table in tables.items():
            r = orc.run_ext(o, i, b, seed, weights=w, discount=table)
            core = orc.finalize(r["regs"], b, r["S"], r["H"])["coreach"]
            for x in range(n):
                mask = np.isfinite(Dist[x]) & (Dist[x] > 0)
                d, wy = Dist[x][mask], w[mask]
                fd = np.array([table[min(int(k), len(table)) - 1] for k in d])
                S, H, Dd, R = (wy * d).sum(), (wy / d).sum(), (wy * fd).sum(), w[x] + wy.sum()
                assert abs(r["S"][x] - S) < 3e-3 * max(1.0, S), (name, tname, x)
                assert abs(r["H"][x] - H) < 3e-3 * max(1.0, H), (name, tname, x)
                assert abs(r["D"][x] - Dd) < 3e-3 * max(1.0, Dd), (name, tname, x)
                assert abs(core[x] - R) < 3e-3 * R, (name, tname, x)


def test_neighbourhood_function_matches_ball_sizes(orc, gg):
    # N(t) ~ sum over x of the weight of B(x, t), exact regime
    b = 16
    rng = np.random.default_rng(19)
    for name, (o, i) in small_graphs(gg):
        n = o.shape[0] - 1
        w = rng.integers(1, 3, size=n).astype(np.int32)
        seed = exact_replica_seed(orc, w)
        Dist = bfs_dist(o, i)
        r = orc.run_ext(o, i, b, seed, weights=w, trace=True)
        N = orc.neighbourhood(r["etrace"])
        assert len(N) == r["passes"] + 1
        for t in range(len(N)):
            exact = sum(w[(Dist[x] <= t)].sum() for x in range(n))
            assert abs(N[t] - exact) < 3e-3 * exact, (name, t)
        assert np.all(np.diff(N) >= -1e-9 * N[-1])          # balls only grow


def test_distance_stats_closed_forms(orc):
    # directed path on n nodes: n - d pairs at distance d, average (n+1)/3
    n = 40
    N = [n + sum(n - d for d in range(1, t + 1)) for t in range(n)]
    st = orc.distance_stats(N)
    assert st["pairs"] == n * (n - 1) / 2
    assert abs(st["average_distance"] - (n + 1) / 3) < 1e-12
    # directed cycle: n pairs at each distance 1..n-1, N(t) = n (t+1) linear,
    # average n/2, effective diameter 0.9 n - 1 exactly by interpolation
    n = 50
    N = [n * (t + 1) for t in range(n)]
    st = orc.distance_stats(N)
    assert abs(st["average_distance"] - n / 2) < 1e-12
    assert abs(st["effective_diameter"] - (0.9 * n - 1)) < 1e-12
    assert orc.distance_stats([7.0])["effective_diameter"] == 0.0     # no arcs


def test_node_ext_matches_run_ext_bitwise(orc, gg):
    table = [1.0 / math.log2(d + 1) for d in range(1, 20)]
    for name, (o, i) in small_graphs(gg):
        n = o.shape[0] - 1
        w = np.random.default_rng(n).integers(1, 6, size=n).astype(np.int32)
        r = orc.run_ext(o, i, 6, 21, weights=w, discount=table)
        for x in range(0, n, max(1, n // 7)):
            q = orc.node(o, i, 6, 21, x, weights=w, discount=table)
            assert np.array_equal(q["regs"], r["regs"][x]), (name, x)
            assert q["S"] == r["S"][x] and q["H"] == r["H"][x] and q["D"] == r["D"][x], (name, x)


def test_discount_tables_exact_values(orc):
    """Sec. 7 discounts at distances where they are exact in binary: 1/d and
    1/d^2 at powers of two, 1/log2(d+1) at d = 2^k - 1 (= 1/k), constant 1;
    and everywhere non-increasing with f(1) = 1."""
    L = 64
    h, q, lg, c = (orc.discount_table(k, L) for k in ("harmonic", "quadratic", "logarithmic", "constant"))
    for k in range(0, 6):
        d = 1 << k
        assert h[d - 1] == 1.0 / d and q[d - 1] == 1.0 / (d * d)
    for k in range(1, 7):
        assert lg[(1 << k) - 2] == 1.0 / k
    assert np.all(c == 1.0)
    for f in (h, q, lg, c):
        assert f[0] == 1.0 and np.all(np.diff(f) <= 0.0)
    with pytest.raises(KeyError):
        orc.discount_table("exponential", 4)


def test_first_pass_rows_is_pass_zero_and_openmp_build_agrees(orc, gg):
    """The bounded pass behind the CPU baseline: over every row it is pass 0 of
    the oracle run (counters at radius 1, S, H and the change count), over a
    sub-range it is that range of the same pass, and the OpenMP build of the
    same loop (several threads) gives identical counters, sums and count."""
    off, idx = gg.rmat(12, 8, seed=7, transpose=True, relabel=True)
    n = len(off) - 1
    b, seed = 6, 9
    one = orc.run(off, idx, b, seed, max_passes=1)
    full = orc.first_pass_rows(off, idx, b, seed, 0, n)
    assert np.array_equal(full["next"], one["regs"])
    assert np.array_equal(full["S"], one["S"]) and np.array_equal(full["H"], one["H"])
    assert full["changed"] == one["nmod"][0] and full["threads"] == 1
    v0, v1 = 100, 3000
    part = orc.first_pass_rows(off, idx, b, seed, v0, v1)
    par = orc.first_pass_rows(off, idx, b, seed, v0, v1, all_cores=True)
    assert np.array_equal(part["next"], full["next"][v0:v1])
    assert np.array_equal(part["S"], full["S"][v0:v1]) and np.array_equal(part["H"], full["H"][v0:v1])
    for key in ("next", "S", "H"):
        assert np.array_equal(par[key], part[key]), key
    assert par["changed"] == part["changed"]
    with pytest.raises(ValueError):
        orc.first_pass_rows(off, idx, b, seed, 5, n + 1)
