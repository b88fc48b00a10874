"""Shared helpers of the GPU parity tests: run the HIP library and the oracle
on the same seeded input and compare them element by element."""
import hashlib
import os

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


GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def sha256_of(a) -> str:
    """Digest of an array's raw bytes (float64 as little-endian), the form
    tests/golden/make_fullsize.py writes."""
    a = np.ascontiguousarray(a)
    if a.dtype == np.float64:
        a = a.astype("<f8", copy=False)
    return hashlib.sha256(a.tobytes()).hexdigest()


def seq_sha256(xs) -> str:
    return hashlib.sha256(",".join(str(int(x)) for x in xs).encode()).hexdigest()


def load_golden_single(name):
    """A single-graph golden file: scalar lines, nmod, sha256 digests, and
    node lines (id lastmod S H closeness lin harmonic coreach, hex floats)."""
    out = {"sha256": {}, "nodes": {}}
    for line in open(os.path.join(GOLDEN, name)):
        if line.startswith("#") or not line.strip():
            continue
        f = line.split()
        if f[0] == "sha256":
            out["sha256"][f[1]] = f[2]
        elif f[0] == "nmod":
            out["nmod"] = [int(x) for x in f[1:]]
        elif f[0] == "node":
            vals = [float.fromhex(x) for x in f[3:]]
            out["nodes"][int(f[1])] = dict(lastmod=int(f[2]), S=vals[0], H=vals[1],
                                           **dict(zip(CENTRALITIES, vals[2:])))
        else:
            out[f[0]] = int(f[1])
    return out


def load_golden_batch(name):
    """Per-graph lines: g n m passes and 16-hex digests of registers, S, H and
    the per-pass change counts."""
    rows = {}
    for line in open(os.path.join(GOLDEN, name)):
        if line.startswith("#") or not line.strip():
            continue
        f = line.split()
        rows[int(f[0])] = dict(n=int(f[1]), m=int(f[2]), passes=int(f[3]), regs=f[4], S=f[5], H=f[6], nmod=f[7])
    return rows


def load_golden_targets(name):
    """Served targets: `target j sc ef b n m passes`, then its nmod and
    sha256 lines."""
    out, cur = [], None
    for line in open(os.path.join(GOLDEN, name)):
        if line.startswith("#") or not line.strip():
            continue
        f = line.split()
        if f[0] == "target":
            cur = dict(zip(("j", "sc", "ef", "b", "n", "m", "passes"), (int(x) for x in f[1:])), sha256={})
            out.append(cur)
        elif f[0] == "nmod":
            cur["nmod"] = [int(x) for x in f[1:]]
        elif f[0] == "sha256":
            cur["sha256"][f[1]] = f[2]
    return out
