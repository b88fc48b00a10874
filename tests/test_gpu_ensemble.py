"""Multi-seed ensembles: K runs with different hash seeds on one graph in one
context.  Every run must equal the oracle's independent run with that seed
(registers, pass count, FP64 accumulators and centralities), and the per-node
mean and empirical standard deviation must equal the oracle's, in every pass
mode and row class."""
import numpy as np
import pytest

import graphgen as gg
import oracle
from hbcheck import assert_fp, run_hb

pytestmark = pytest.mark.gpu

CEN = ("closeness", "lin", "harmonic", "coreach")


def _log(*a):
    print(*a, flush=True)


def run_ens(off, idx, b, seeds, max_passes=0, **opt):
    import paper_1308_2144_amd as hb

    with hb.Ensemble(off, idx, b, seeds, **opt) as e:
        total = e.run(max_passes)
        out = dict(total=total, passes=e.passes(), regs=e.registers(), cen=e.centralities())
        out["S"], out["H"] = e.accumulators()
        out["summary"] = {w: e.summary(w) for w in CEN}
    return out


def check_vs_oracle(off, idx, b, seeds, what, max_passes=0, **opt):
    got = run_ens(off, idx, b, seeds, max_passes=max_passes, **opt)
    ref = oracle.ensemble(off, idx, b, seeds, max_passes=max_passes)
    K = len(seeds)
    assert got["total"] == max(r["passes"] for r in ref), what
    for k, r in enumerate(ref):
        w = f"{what} seed {k}"
        if max_passes == 0:
            assert got["passes"][k] == r["passes"], (w, got["passes"], [x["passes"] for x in ref])
        assert np.array_equal(got["regs"][:, k], r["regs"]), w + ": registers"
        assert_fp(got["S"][:, k], r["S"], w + " S")
        assert_fp(got["H"][:, k], r["H"], w + " H")
        for c in CEN:
            assert_fp(got["cen"][c][:, k], r[c], f"{w} {c}")
    for c in CEN:
        vals = np.stack([r[c] for r in ref], axis=1) if len(off) > 1 else np.zeros((0, K))
        m, sd = oracle.ensemble_summary(vals)
        assert_fp(got["summary"][c][0], m, f"{what} mean {c}")
        assert_fp(got["summary"][c][1], sd, f"{what} sd {c}")
    return got


GRAPHS = {
    "rmat8t": lambda: gg.rmat(8, 8, seed=21, transpose=True),
    "rmat9u": lambda: gg.rmat(9, 6, seed=22, directed=False),
    "star": lambda: gg.star(9000),             # heavy row cut into chunks
    "cycle": lambda: gg.directed_cycle(150),   # long tail of sparse passes
    "empty0": lambda: gg.empty(0),
    "isolated": lambda: gg.empty(37),
}


@pytest.mark.parametrize("b,K", [(4, 2), (4, 16), (5, 8), (6, 4), (7, 2)])
@pytest.mark.parametrize("name", sorted(GRAPHS))
def test_ensemble_equals_oracle_runs(name, b, K):
    off, idx = GRAPHS[name]()
    seeds = [int(s) for s in np.random.default_rng(b * 100 + K).integers(0, 1 << 40, size=K)]
    check_vs_oracle(off, idx, b, seeds, f"{name} b={b} K={K}")


@pytest.mark.parametrize("opt", [dict(frontier=0), dict(qdense=1), dict(push=0), dict(slice=1),
                                 dict(dense_pct=101, sparse_pct=101), dict(dense_pct=101, sparse_pct=101, pairs=0),
                                 dict(light_max=4, heavy_min=40, chunk=16), dict(dense_pct=101)])
def test_ensemble_modes_and_row_classes(opt):
    off, idx = gg.rmat(9, 12, seed=23, transpose=True)
    check_vs_oracle(off, idx, 5, [7, 8, 9, 10], f"opts {opt}", **opt)


def test_ensemble_partial_runs_and_reset():
    import paper_1308_2144_amd as hb

    off, idx = gg.rmat(8, 10, seed=24, transpose=True)
    check_vs_oracle(off, idx, 4, [1, 2, 3, 4], "max_passes 2", max_passes=2)
    seeds_a, seeds_b = [11, 12], [13, 14]
    with hb.Ensemble(off, idx, 6, seeds_a) as e:
        e.run()
        e.reset(seeds_b)
        e.run()
        regs = e.registers()
        passes = e.passes()
        with pytest.raises(hb.HBError):
            hb.hb_reset(e._ctx, 5)       # ensembles restart with hb_ensemble_reset
    for k, sd in enumerate(seeds_b):
        r = oracle.run(off, idx, 6, sd)
        assert passes[k] == r["passes"] and np.array_equal(regs[:, k], r["regs"])


def test_ensemble_device_input_equals_plain_runs_at_scale():
    """R-MAT scale 18 (262k nodes, 4M arcs), 8 seeds at p = 16 from device
    memory: each run equals the plain single-seed GPU run (itself checked
    against the oracle at scale 20)."""
    import torch

    import paper_1308_2144_amd as hb

    off, idx = gg.rmat(18, 16, seed=25, transpose=True, relabel=True)
    seeds = list(range(100, 108))
    o = torch.from_numpy(off).cuda()
    i = torch.from_numpy(idx).cuda()
    with hb.Ensemble(o, i, 4, seeds) as e:
        e.run()
        passes = e.passes()
        regs = e.registers()
        S, H = e.accumulators()
        mean, sd = e.summary("harmonic")
    _log("ensemble s18 passes", passes)
    harm = []
    for k, s in enumerate(seeds):
        ref = run_hb(off, idx, 4, s)
        assert passes[k] == ref["passes"]
        assert np.array_equal(regs[:, k], ref["regs"]), k
        assert_fp(S[:, k], ref["S"], f"S seed {k}")
        assert_fp(H[:, k], ref["H"], f"H seed {k}")
        harm.append(ref["harmonic"])
    m, s = oracle.ensemble_summary(np.stack(harm, axis=1))
    assert_fp(mean, m, "mean harmonic")
    assert_fp(sd, s, "sd harmonic")
