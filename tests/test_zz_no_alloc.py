"""hb_run_static, the entry point that allocates no device memory (its state
lives in the library's fixed scratch array), against hb_init + hb_run +
hb_centralities on the same graphs: pass count, registers and the four
outputs bit for bit, on calls in a row that reuse the scratch (the second
graph smaller than the first, so stale contents of a larger call sit past
the smaller one's data), and the refusal of a graph that does not fit."""
import numpy as np
import pytest

import graphgen as gg
import oracle

pytestmark = pytest.mark.gpu

OUTS = ("closeness", "lin", "harmonic", "coreach")


def _log(*a):
    print(*a, flush=True)


def _static(off, idx, b, seed, offsets_dtype):
    import torch

    import paper_1308_2144_amd as hb

    n = len(off) - 1
    o = torch.from_numpy(off.astype(offsets_dtype)).cuda()
    x = torch.from_numpy(idx).cuda()
    outs = {k: torch.full((max(n, 1),), -7.0, dtype=torch.float64, device="cuda") for k in OUTS}
    regs = torch.full((max(n, 1), 1 << b), 0xAB, dtype=torch.uint8, device="cuda")
    passes = hb.hb_run_static(o, x, b, seed, **outs, registers=regs,
                              stream=torch.cuda.current_stream().cuda_stream)
    torch.cuda.synchronize()
    res = {k: v[:n].cpu().numpy() for k, v in outs.items()}
    res["registers"] = regs[:n].cpu().numpy()
    res["passes"] = passes
    return res


def _plain(off, idx, b, seed):
    import paper_1308_2144_amd as hb

    with hb.HyperBall(off, idx, b, seed) as g:
        passes = g.run()
        res = dict(g.centralities())
        res["registers"] = g.registers()
        res["passes"] = passes
    return res


def _same(a, b, what):
    assert a["passes"] == b["passes"], (what, a["passes"], b["passes"])
    assert np.array_equal(a["registers"], b["registers"]), what + ": registers"
    for k in OUTS:
        assert np.array_equal(a[k], b[k]), f"{what}: {k} not bit-identical"


def test_static_equals_context_path_on_calls_in_a_row():
    big = gg.rmat(15, 8, seed=61, transpose=True, relabel=True)     # 32768 nodes, some isolated
    small = gg.rmat(11, 12, seed=62, transpose=True)                 # 2048 nodes
    cases = [("rmat15 b6 int64", big, 6, 11, np.int64), ("rmat11 b8 int32", small, 8, 12, np.int32),
             ("rmat11 b4 int64", small, 4, 13, np.int64)]
    for what, (off, idx), b, seed, dt in cases:
        _log("case", what, "n", len(off) - 1, "m", len(idx))
        got = _static(off, idx, b, seed, dt)
        _same(got, _plain(off, idx, b, seed), what)
        _log("  ok, passes", got["passes"])
    # and the smallest against the oracle directly
    off, idx = small
    got = _static(off, idx, 4, 13, np.int64)
    ref = oracle.run(off, idx, 4, 13)
    fin = oracle.finalize(ref["regs"], 4, ref["S"], ref["H"])
    assert got["passes"] == ref["passes"] and np.array_equal(got["registers"], ref["regs"])
    for k in OUTS:
        assert np.array_equal(got[k], fin[k]), k


def test_static_degenerate_graphs():
    for what, (off, idx) in (("no arcs", gg.empty(100)), ("one node", gg.empty(1)), ("cycle", gg.directed_cycle(77)),
                             ("star", gg.star(3000))):
        got = _static(off, idx, 5, 3, np.int64)
        _same(got, _plain(off, idx, 5, 3), what)


def test_static_refuses_a_graph_over_its_scratch():
    import torch

    import paper_1308_2144_amd as hb

    n = 1 << 20                                   # 2^20 nodes at log2m 8 need ~0.5 GiB
    o = torch.zeros(n + 1, dtype=torch.int64, device="cuda")
    x = torch.zeros(1, dtype=torch.int32, device="cuda")[:0]
    with pytest.raises(hb.HBError) as e:
        hb.hb_run_static(o, x, 8, 1)
    assert e.value.status == hb.HB_ENOMEM and "scratch" in str(e.value)
    with pytest.raises(hb.HBError) as e:
        hb.hb_run_static(o, x, 9, 1)
    assert e.value.status == hb.HB_EINVAL
