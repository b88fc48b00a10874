"""The stored whole oracle runs under tests/golden (written by
tests/golden/make_fullsize.py from oracle/ and graphgen/ only), checked on the
CPU: internal consistency of the R-MAT scale-24 file (the outputs are the
Sec. 3 / Sec. 5 finalisation of the stored S and H, the late-changing nodes
are all there), and the batch and served-target files re-derived from fresh
oracle runs on their smallest graphs."""
import hashlib

import numpy as np

from hbcheck import load_golden_batch, load_golden_single, load_golden_targets


def _sha(a) -> str:
    return hashlib.sha256(np.ascontiguousarray(a).tobytes()).hexdigest()


def _seq_sha(xs) -> str:
    return hashlib.sha256(",".join(str(int(x)) for x in xs).encode()).hexdigest()


def test_rmat_s24_golden_is_self_consistent():
    gold = load_golden_single("fullsize_rmat-s24.txt")
    passes, nmod = gold["passes"], gold["nmod"]
    assert len(nmod) == passes and nmod[-1] == 0 and all(x > 0 for x in nmod[:-1])
    assert gold["sha256"]["harmonic"] == gold["sha256"]["H"]       # harmonic centrality is H itself
    nodes = gold["nodes"]
    assert len(nodes) >= 1024
    for v, r in nodes.items():
        assert 0 <= r["lastmod"] <= passes and 0 <= v < gold["n"]
        S, E = r["S"], r["coreach"]
        assert r["closeness"] == (0.0 if S == 0.0 else 1.0 / S)
        assert r["lin"] == (1.0 if S == 0.0 else (E * E) / S)
        assert r["harmonic"] == r["H"]
        if r["lastmod"] == 0:                                      # never changed: radius-0 ball only
            assert S == 0.0 and r["H"] == 0.0
    late = [v for v, r in nodes.items() if r["lastmod"] >= passes - 1]
    assert len(late) == nmod[-2] + nmod[-1]


def test_batch_golden_rederived_on_its_smallest_graphs(orc, gg):
    gold = load_golden_batch("fullsize_batch-4096.txt")
    assert sorted(gold) == list(range(4096))
    count = 4096
    rng = np.random.default_rng(4)                                  # the recipe of graphgen.batch_workload
    ns = np.exp(rng.uniform(np.log(1000), np.log(200_000), size=count)).astype(np.int64)
    kinds = (np.arange(count) >= count // 2).astype(np.int32)
    gseeds = rng.integers(1, 2**62, size=count, dtype=np.int64).astype(np.uint64)
    picks = []
    for k in (0, 1):
        ids = np.flatnonzero(kinds == k)
        picks += ids[np.argsort(ns[ids])[:3]].tolist()
    for g in picks:
        (off, idx), = gg.batch(kinds[g:g + 1], ns[g:g + 1], gseeds[g:g + 1])
        row = gold[g]
        assert (row["n"], row["m"]) == (len(off) - 1, len(idx)), g
        r = orc.run(off, idx, 5, 42 + g)
        assert r["passes"] == row["passes"], g
        assert _sha(r["regs"])[:16] == row["regs"] and _sha(r["S"])[:16] == row["S"] and _sha(r["H"])[:16] == row["H"], g
        assert _seq_sha(r["nmod"])[:16] == row["nmod"], g


def test_served_target_golden_rederived_on_its_smallest_target(orc, gg):
    targets = load_golden_targets("fullsize_serve-targets.txt")
    t = min(targets, key=lambda x: x["m"])
    off, idx = gg.rmat(t["sc"], t["ef"], seed=1000 + t["j"], transpose=True)
    assert (len(off) - 1, len(idx)) == (t["n"], t["m"])
    r = orc.run(off, idx, t["b"], 42 + t["j"])
    assert r["passes"] == t["passes"] and [int(x) for x in r["nmod"]] == t["nmod"]
    assert _sha(r["regs"]) == t["sha256"]["registers"]
    assert _sha(r["S"]) == t["sha256"]["S"] and _sha(r["H"]) == t["sha256"]["H"]
    fin = orc.finalize(r["regs"], t["b"], r["S"], r["H"])
    for k in ("closeness", "lin", "harmonic", "coreach"):
        assert _sha(fin[k]) == t["sha256"][k], k
