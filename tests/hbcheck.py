"""Shared helpers of the GPU parity tests: run the HIP library and the oracle
on the same seeded input and compare them element by element."""
import numpy as np

import oracle

CENTRALITIES = ("closeness", "lin", "harmonic", "coreach")


def assert_fp(a, b, what, rtol=1e-12):
    """The FP64 bar: equal, or |a-b| <= rtol*max(|a|,|b|).  The design aims at
    bit-identical results, so the number of inexact entries is also 0 here."""
    a = np.asarray(a)
    b = np.asarray(b)
    assert a.shape == b.shape, what
    same = (a == b) | (np.isnan(a) & np.isnan(b))
    if same.all():
        return
    bad = ~same
    scale = np.maximum(np.abs(a), np.abs(b))
    close = np.abs(a - b) <= rtol * scale
    assert close[bad].all(), f"{what}: {int((~close).sum())} entries differ beyond {rtol}"
    raise AssertionError(f"{what}: {int(bad.sum())} entries within {rtol} but not bit-identical")


def run_hb(off, idx, b, seed, max_passes=0, **opt):
    import paper_1308_2144_amd as hb

    with hb.HyperBall(off, idx, b, seed, **opt) as g:
        passes = g.run(max_passes)
        out = dict(passes=passes, regs=g.registers(), stats=g.stats(),
                   pass_stats=[g.pass_stats(t) for t in range(passes)])
        out["S"], out["H"] = g.accumulators()
        out.update(g.centralities())
    return out


def run_oracle(off, idx, b, seed, max_passes=0):
    ref = oracle.run(np.asarray(off, dtype=np.int64), idx, b, seed, max_passes=max_passes)
    ref.update(oracle.finalize(ref["regs"], b, ref["S"], ref["H"]))
    return ref


def compare(got, ref, what=""):
    assert got["passes"] == ref["passes"], f"{what}: passes {got['passes']} != {ref['passes']}"
    assert np.array_equal(got["regs"], ref["regs"]), f"{what}: registers differ"
    nmod = [p["rows_changed"] for p in got["pass_stats"]]
    assert nmod == list(ref["nmod"]), f"{what}: per-pass changes {nmod} != {list(ref['nmod'])}"
    assert_fp(got["S"], ref["S"], f"{what} S")
    assert_fp(got["H"], ref["H"], f"{what} H")
    for k in CENTRALITIES:
        assert_fp(got[k], ref[k], f"{what} {k}")


def check(off, idx, b, seed, what="", max_passes=0, **opt):
    got = run_hb(off, idx, b, seed, max_passes=max_passes, **opt)
    ref = run_oracle(off, idx, b, seed, max_passes=max_passes)
    compare(got, ref, what)
    return got, ref
