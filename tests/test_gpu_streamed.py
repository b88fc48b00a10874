"""Graphs streamed from host memory (Sec. 5.1 keeps the graph out of the
memory that holds the counters): the CSR in pinned host memory, uploaded in
row chunks every pass, against the oracle element by element and against the
same graph resident in device memory; chunk selection in sparse passes; and
the refusals."""
import numpy as np
import pytest

import graphgen as gg
from hbcheck import check, compare, run_hb, run_oracle

pytestmark = pytest.mark.gpu


def _log(*a):
    print(*a, flush=True)


def _streamed(off, idx, b, seed, budget, **opt):
    got = run_hb(off, idx, b, seed, stream_graph=1, graph_budget=budget, timing=1, **opt)
    st = got["stats"]
    assert st["streamed"] == 1 and st["chunk_bytes"] == budget // 2 // 256 * 256
    assert st["compressed"] == int(bool(opt.get("stream_compress", 0)))
    return got


@pytest.fixture(scope="module")
def s20():
    off, idx = gg.rmat(20, 16, seed=2, transpose=True, relabel=True)
    return off, idx, run_oracle(off, idx, 6, 42)


@pytest.mark.timeout(600)
def test_streamed_rmat_s20_against_oracle(s20):
    """R-MAT scale 20 (edge factor 16, relabelled, transposed), log2m 6, in
    chunks of 4 MiB (about 18 chunks), against the whole oracle run."""
    off, idx, ref = s20
    got = _streamed(off, idx, 6, 42, 8 << 20)
    compare(got, ref, "streamed s20")
    ps = got["pass_stats"]
    chunks = got["stats"]["chunks"]
    _log("streamed s20: chunks", chunks, "passes", got["passes"], "modes", [p["mode"] for p in ps],
         "chunks run", [p["chunks_run"] for p in ps], "host MB", [round(p["host_bytes"] / 1e6, 1) for p in ps])
    assert chunks > 8
    csr = 8 * (len(off)) + 4 * len(idx)
    # first and dense passes stream every chunk: the whole CSR once, plus the
    # 256-byte alignment of each chunk's offsets
    assert ps[0]["chunks_run"] == chunks and csr <= ps[0]["host_bytes"] <= csr + 8 * chunks


@pytest.mark.timeout(600)
def test_streamed_compressed_rmat_s20_against_oracle(s20):
    """The same graph with the streamed arcs kept compressed (rows sorted,
    blocks of 32 arcs coded as differences) and decoded on the device: the
    oracle's results, fewer bytes over the host link."""
    off, idx, ref = s20
    got = _streamed(off, idx, 6, 42, 8 << 20, stream_compress=1)
    compare(got, ref, "streamed compressed s20")
    st = got["stats"]
    csr = 8 * len(off) + 4 * len(idx)
    ps = got["pass_stats"]
    _log("compressed s20: host bytes", st["host_graph_bytes"], "of", csr, "; first pass sent", ps[0]["host_bytes"])
    assert st["host_graph_bytes"] < 0.9 * csr
    assert ps[0]["chunks_run"] == st["chunks"] and ps[0]["host_bytes"] < 0.9 * csr


@pytest.mark.timeout(600)
def test_streamed_skips_chunks_in_sparse_passes():
    """Unrelabelled R-MAT keeps its hubs at low ids, so the late passes'
    changes sit in few chunks: the selection must skip chunks and still give
    the oracle's results; and a graph with a long tail (a directed path) has
    passes that need a single chunk."""
    off, idx = gg.rmat(16, 8, seed=5, transpose=True)
    got = _streamed(off, idx, 5, 9, 1 << 20)
    compare(got, run_oracle(off, idx, 5, 9), "streamed raw s16")
    off, idx = gg.directed_path(3000)        # pass t changes nodes 0 .. n-t-2 only
    got = _streamed(off, idx, 4, 3, 16 << 10)
    compare(got, run_oracle(off, idx, 4, 3), "streamed path")
    compare(_streamed(off, idx, 4, 3, 16 << 10, stream_compress=1), run_oracle(off, idx, 4, 3), "compressed path")
    ps = got["pass_stats"]
    assert got["stats"]["chunks"] >= 4
    assert min(p["chunks_run"] for p in ps[1:]) <= 2, [p["chunks_run"] for p in ps]


@pytest.mark.timeout(600)
@pytest.mark.parametrize("b", [4, 7, 8])
def test_streamed_equals_resident(b):
    """Every row class (light, medium, heavy rows cut into items) and both
    offset widths: streamed and resident runs agree bit for bit, with the
    oracle too."""
    off, idx = gg.rmat(14, 24, seed=40 + b, transpose=True)
    opt = dict(light_max=8, heavy_min=200, chunk=64)
    for o in (off, off.astype(np.int32)):
        got = _streamed(o, idx, b, 5, 256 << 10, **opt)
        res = run_hb(o, idx, b, 5, **opt)
        assert got["passes"] == res["passes"] and np.array_equal(got["regs"], res["regs"])
        for k in ("S", "H", "closeness", "lin", "harmonic", "coreach"):
            assert np.array_equal(got[k], res[k]), k
        assert [p["rows_changed"] for p in got["pass_stats"]] == [p["rows_changed"] for p in res["pass_stats"]]
    check(off, idx, b, 5, "streamed rmat14", stream_graph=1, graph_budget=256 << 10, **opt)
    check(off, idx, b, 5, "compressed rmat14", stream_graph=1, graph_budget=256 << 10, stream_compress=1, **opt)


def test_streamed_compressed_unsorted_rows_and_duplicates():
    """Compression sorts each row's successors and codes differences, zero
    for repeated arcs and negative across row and block boundaries: rows
    given in shuffled order with duplicate arcs and self-loops, and ids near
    2^31 / 64 apart, give the oracle's results."""
    rng = np.random.default_rng(17)
    n = 5000
    off, idx = gg.random_digraph(n, 14 * n, seed=18, self_loops=True, dedup=False)
    idx = idx.copy()
    for v in range(0, n, 3):                       # shuffle some rows in place
        a, b_ = off[v], off[v + 1]
        idx[a:b_] = rng.permutation(idx[a:b_])
    for cmp in (0, 1):
        got = _streamed(off, idx, 5, 2, 64 << 10, stream_compress=cmp)
        compare(got, run_oracle(off, idx, 5, 2), f"unsorted compress={cmp}")


def test_streamed_budget_decides_and_refusals():
    import torch

    import paper_1308_2144_amd as hb

    off, idx = gg.rmat(10, 8, seed=1, directed=False)
    csr = 8 * len(off) + 4 * len(idx)
    with hb.HyperBall(off, idx, 4, 42, graph_budget=csr - 1) as g:     # over budget: streamed
        assert g.stats()["streamed"] == 1
        g.run()
    with hb.HyperBall(off, idx, 4, 42, graph_budget=csr) as g:         # fits: resident
        assert g.stats()["streamed"] == 0
    with hb.HyperBall(off, idx, 4, 42, stream_graph=-1, graph_budget=16) as g:
        assert g.stats()["streamed"] == 0
    with pytest.raises(hb.HBError) as e:                                # a row larger than a staging buffer
        hb.HyperBall(*gg.star(3000), 4, 1, stream_graph=1, graph_budget=4096)
    assert e.value.status == hb.HB_ENOMEM and "staging buffer" in str(e.value)
    with pytest.raises(hb.HBError) as e:
        hb.HyperBall(off, idx, 9, 1, stream_graph=1)
    assert e.value.status == hb.HB_EINVAL
    with pytest.raises(hb.HBError) as e:
        hb.HyperBall(torch.from_numpy(off).cuda(), torch.from_numpy(idx).cuda(), 4, 1, stream_graph=1)
    assert e.value.status == hb.HB_EINVAL
    with pytest.raises(hb.HBError) as e:                                # validation on the host
        hb.HyperBall(np.array([0, 1, 3], dtype=np.int64), np.array([1, 5, 0], dtype=np.int32), 4, 1,
                     stream_graph=1)
    assert e.value.status == hb.HB_EINVAL
    for o, x in (gg.empty(0), gg.empty(50)):                           # no arcs at all
        got = _streamed(o, x, 4, 1, 1 << 16)
        compare(got, run_oracle(o, x, 4, 1), "streamed empty")
