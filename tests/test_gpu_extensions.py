"""Node weights (Sec. 6), discounted-gain sums (Sec. 7) and the
neighbourhood function against the oracle's run_ext: registers, pass counts,
S, H, D, centralities and N(t) bit for bit, in every pass mode and row
class, and the distance statistics from N(t)."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from hbcheck import assert_fp

pytestmark = pytest.mark.gpu

CEN = ("closeness", "lin", "harmonic", "coreach")


def _log(*a):
    print(*a, flush=True)


def _tables(table):
    """A discount given as (kind, length) is computed on each side on its own
    (hb_discount_table for the library, the oracle's for the oracle); an
    explicit list of values goes to both."""
    import paper_1308_2144_amd as hb

    if isinstance(table, tuple):
        return hb.discount_table(*table), oracle.discount_table(*table)
    return table, table


def run_gpu(off, idx, b, seed, weights=None, table=None, **opt):
    import paper_1308_2144_amd as hb

    table = _tables(table)[0]
    with hb.HyperBall(off, idx, b, seed, neighbourhood=1, **opt) as g:
        if weights is not None:
            g.set_weights(weights)
        if table is not None:
            g.set_discount(table)
        passes = g.run()
        out = dict(passes=passes, regs=g.registers(), N=g.neighbourhood())
        out["S"], out["H"] = g.accumulators()
        out.update(g.centralities())
        if table is not None:
            out["D"] = g.discounted()
    return out


def check(off, idx, b, seed, what, weights=None, table=None, **opt):
    got = run_gpu(off, idx, b, seed, weights=weights, table=table, **opt)
    ref = oracle.run_ext(off, idx, b, seed, weights=weights, discount=_tables(table)[1], trace=True)
    ref.update(oracle.finalize(ref["regs"], b, ref["S"], ref["H"]))
    assert got["passes"] == ref["passes"], (what, got["passes"], ref["passes"])
    assert np.array_equal(got["regs"], ref["regs"]), what + ": registers"
    for k in ("S", "H") + CEN:
        assert_fp(got[k], ref[k], f"{what} {k}")
    if table is not None:
        assert_fp(got["D"], ref["D"], f"{what} D")
    N = oracle.neighbourhood(ref["etrace"])
    assert_fp(got["N"], N, f"{what} N(t)")
    import paper_1308_2144_amd as hb

    st, rst = hb.hb_distance_stats(got["N"]), oracle.distance_stats(N)
    for k in rst:
        assert_fp([st[k]], [rst[k]], f"{what} {k}")
    return got


GRAPHS = {
    "rmat8t": lambda: gg.rmat(8, 8, seed=41, transpose=True),
    "rmat9u": lambda: gg.rmat(9, 6, seed=42, directed=False),
    "star": lambda: gg.star(9000),
    "cycle": lambda: gg.directed_cycle(120),
    "empty0": lambda: gg.empty(0),
    "isolated": lambda: gg.empty(23),
}


@pytest.mark.parametrize("b", [4, 6, 8, 10])
@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_weights_equal_oracle(name, b):
    off, idx = GRAPHS[name]()
    n = len(off) - 1
    w = np.random.default_rng(b).integers(1, 6, size=n).astype(np.int32)
    check(off, idx, b, 7, f"{name} b={b}", weights=w)


@pytest.mark.parametrize("kind", ["quadratic", "logarithmic", "constant", "short", "identity"])
@pytest.mark.parametrize("name", ["rmat8t", "rmat9u", "star", "cycle", "isolated"])
def test_discounts_equal_oracle(name, kind):
    off, idx = GRAPHS[name]()
    table = {"short": [1.0, 0.5, 0.25], "identity": list(np.arange(1.0, 200.0))}.get(kind, (kind, 48))
    w = np.random.default_rng(3).integers(1, 4, size=len(off) - 1).astype(np.int32)
    got = check(off, idx, 6, 11, f"{name} {kind}", weights=w, table=table)
    if kind == "identity":                      # f(d) = d is S's own weighting
        assert np.array_equal(got["D"], got["S"])


@pytest.mark.parametrize("opt", [dict(frontier=0), dict(qdense=1), dict(push=0), dict(slice=1),
                                 dict(light_max=4, heavy_min=40, chunk=16), dict(dense_pct=101)])
def test_extensions_in_every_mode(opt):
    off, idx = gg.rmat(10, 12, seed=43, transpose=True)
    w = np.random.default_rng(5).integers(1, 9, size=len(off) - 1).astype(np.int32)
    check(off, idx, 5, 3, f"opts {opt}", weights=w, table=("quadratic", 30), **opt)


def test_unit_weights_change_nothing_and_device_weights():
    import torch

    import paper_1308_2144_amd as hb

    off, idx = gg.rmat(12, 10, seed=44, transpose=True, relabel=True)
    n = len(off) - 1
    a = run_gpu(off, idx, 7, 9)
    b = run_gpu(off, idx, 7, 9, weights=np.ones(n, dtype=np.int32))
    assert a["passes"] == b["passes"] and np.array_equal(a["regs"], b["regs"])
    for k in ("S", "H", "N"):
        assert np.array_equal(a[k], b[k]), k
    w = np.random.default_rng(6).integers(1, 30, size=n).astype(np.int32)
    with hb.HyperBall(off, idx, 7, 9) as g:
        g.set_weights(torch.from_numpy(w).cuda())
        g.run()
        regs = g.registers()
        g.set_weights(None)                    # back to unit weights, pass 0
        g.run()
        assert np.array_equal(g.registers(), a["regs"])
        bad = w.copy()
        bad[17] = 0
        with pytest.raises(hb.HBError) as e:
            g.set_weights(bad)
        assert e.value.status == hb.HB_EINVAL
        with pytest.raises(hb.HBError) as e:
            g.set_weights(torch.from_numpy(bad).cuda())
        assert e.value.status == hb.HB_EINVAL
    ref = oracle.run_ext(off, idx, 7, 9, weights=w)
    assert np.array_equal(regs, ref["regs"])


def test_refusals():
    import paper_1308_2144_amd as hb

    off, idx = gg.directed_cycle(30)
    with hb.HyperBall(off, idx, 9, 1) as g:              # p = 512: wide kernel
        with pytest.raises(hb.HBError):
            g.set_discount([1.0])
        with pytest.raises(hb.HBError):
            hb.hb_neighbourhood(g._ctx)                  # not enabled at init
    with hb.Ensemble(off, idx, 4, [1, 2]) as e:
        with pytest.raises(hb.HBError):
            hb.hb_set_weights(e._ctx, np.ones(30, dtype=np.int32))
        with pytest.raises(hb.HBError):
            hb.hb_set_discount(e._ctx, [1.0])


def test_extensions_at_scale_18():
    """R-MAT scale 18 with weights 1..4, the logarithmic discount and N(t),
    whole oracle run."""
    off, idx = gg.rmat(18, 8, seed=45, transpose=True, relabel=True)
    w = np.random.default_rng(7).integers(1, 5, size=len(off) - 1).astype(np.int32)
    got = check(off, idx, 6, 13, "s18", weights=w, table=("logarithmic", 64))
    _log("s18 passes", got["passes"], "N", got["N"][:4], "...", got["N"][-1])
