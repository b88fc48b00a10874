"""Pins for the oracle's HyperLogLog layer (Sec. 4.1, Algorithm 1).

Each check ties the oracle to something outside itself: published SplitMix64
outputs, the paper's rho+ example, Python's correctly rounded int->float
conversion, closed forms of the estimator, and the statistical behaviour the
paper states for HyperLogLog counters.
"""
import math
import os

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def golden(name):
    """Data lines of a fixture under tests/golden (each file cites its source)."""
    with open(os.path.join(GOLDEN, name)) as f:
        return [ln.split() for ln in f if ln.strip() and not ln.startswith("#")]


def test_hash_matches_published_splitmix64(orc):
    rows = golden("splitmix64.txt")
    assert len(rows) >= 2
    for state, *outs in rows:
        want = [int(x, 0) for x in outs]
        assert [orc.hash64(int(state, 0), s) for s in range(len(want))] == want


def test_hash_is_injective_on_ids(orc):
    hs = {orc.hash64(x, 42) for x in range(200_000)}
    assert len(hs) == 200_000


def test_rho_paper_example(orc):
    # Sec. 4.1 example; the bit string is put right after the leftmost b bits.
    for bits, want in golden("paper_rho.txt"):
        k = len(bits)
        for b in (4, 7, 16):
            for idx in (0, 1, (1 << b) - 1):
                h = (idx << (64 - b)) | (int(bits, 2) << (64 - b - k)) | 0x1F
                assert orc.rho(h, b) == int(want)


def test_rho_extremes(orc):
    for b in (4, 6, 16):
        top = 1 << (63 - b)  # first bit after the index is 1
        assert orc.rho(top, b) == 1
        assert orc.rho(top | ((1 << b) - 1) << (64 - b), b) == 1
        assert orc.rho(0, b) == 65 - b                      # all-zero remainder
        assert orc.rho(((1 << b) - 1) << (64 - b), b) == 65 - b
        assert orc.rho(1, b) == 64 - b                      # only the last bit set


def test_add_register_index_uniform_and_rank_geometric(orc):
    # One add per fresh counter: the touched register is uniform over p and
    # its value is geometric(1/2) (Sec. 4.1: h maps to random bit sequences).
    b, p, N = 6, 64, 60_000
    idx = np.zeros(p)
    ranks = np.zeros(70)
    for x in range(N):
        M = orc.new_counter(b)
        orc.add(M, b, x, 7)
        nz = np.flatnonzero(M)
        assert nz.size == 1
        idx[nz[0]] += 1
        ranks[M[nz[0]]] += 1
    # chi-square for uniform index (63 dof): mean 63, sd ~ 11.2
    chi = ((idx - N / p) ** 2 / (N / p)).sum()
    assert chi < 63 + 5 * 11.3
    for k in range(1, 8):
        expect = N * 2.0 ** -k
        assert abs(ranks[k] - expect) < 5 * math.sqrt(expect)


def test_add_uses_leftmost_bits(orc):
    # h(0, seed 0) = 0xE220A8397B1DCDAF = 1110 0010 0010 0000 1010 ... (first
    # published SplitMix64 output).  The register is its leftmost b bits and
    # the value is rho+ of what follows (Sec. 4.1, Algorithm 1).
    expect = {4: (0b1110, 3), 5: (0b11100, 2), 6: (0b111000, 1), 7: (0b1110001, 4),
              8: (0b11100010, 3)}
    for b, (idx, r) in expect.items():
        M = orc.new_counter(b)
        orc.add(M, b, 0, 0)
        want = np.zeros(1 << b, dtype=np.uint8)
        want[idx] = r
        assert np.array_equal(M, want), b


def test_add_is_max(orc):
    b = 4
    M = orc.new_counter(b)
    for x in range(1000):
        before = M.copy()
        orc.add(M, b, x, 3)
        assert (M >= before).all()
        assert (M != before).sum() <= 1


def _exact_sum(M, b):
    K = 65 - b
    return float(sum(1 << (K - int(r)) for r in M)) / float(1 << K)


@pytest.mark.parametrize("b", [4, 5, 6, 7, 8, 12, 16])
def test_register_sum_is_exact_sum_rounded_once(orc, b):
    rng = np.random.default_rng(b)
    p = 1 << b
    for trial in range(40):
        hi = [3, 20, 40, 65 - b][trial % 4]
        M = rng.integers(0, hi + 1, size=p).astype(np.uint8)
        if trial % 5 == 0:
            M[:] = 0
            M[rng.integers(0, p)] = 65 - b  # forces a rounding decision
        assert orc.register_sum(M, b) == _exact_sum(M, b)


def test_alpha_constants(orc):
    # Tabulated values of Flajolet et al. 2007, and 0.7213/(1+1.079/p) beyond;
    # all lie in (0.67, 0.7213).
    for m, a in golden("hll_alpha.txt"):
        assert orc.alpha(int(m).bit_length() - 1) == float(a)
    for b in range(7, 17):
        a = orc.alpha(b)
        assert 0.709 < a < 0.7213
    assert orc.alpha(16) > orc.alpha(7)


@pytest.mark.parametrize("b", [4, 5, 6, 7, 8, 16])
def test_size_constant_registers(orc, b):
    # All registers = k >= 1: sum = p 2^-k, so E = alpha_p p 2^k exactly (the
    # powers of two make every rounding exact), and no register is zero.
    p = 1 << b
    for k in range(1, 40):
        M = np.full(p, k, dtype=np.uint8)
        assert orc.size(M, b) == orc.alpha(b) * p * 2.0 ** k


@pytest.mark.parametrize("b", [4, 6, 8, 16])
def test_size_small_range(orc, b):
    p = 1 << b
    M = np.zeros(p, dtype=np.uint8)
    assert orc.size(M, b) == 0.0                      # empty counter: p ln(p/p)
    for r in (1, 5, 30, 65 - b):
        M[:] = 0
        M[p // 3] = r
        assert orc.size(M, b) == p * math.log(p / (p - 1))


def test_size_switches_to_raw_above_five_halves_p(orc):
    # V > 0 but raw estimate above 5p/2: the raw estimate is kept.
    b, p = 4, 16
    M = np.full(p, 10, dtype=np.uint8)
    M[0] = 0
    s = 1.0 + 15 * 2.0 ** -10
    assert orc.size(M, b) == (0.673 * p * p) / s


def test_size_exact_regime(orc):
    # p = 2^16 and at most 64 distinct items: with no register collision the
    # linear-counting estimate p ln(p/(p-k)) = k + k^2/2p + ... rounds to k.
    b = 16
    p = 1 << b
    M = orc.new_counter(b)
    for k in range(1, 65):
        orc.add(M, b, 1000 + k, 42)
        assert int(np.count_nonzero(M)) == k          # no collision for this seed
        E = orc.size(M, b)
        assert round(E) == k
        assert abs(E - (k + k * k / (2 * p))) < 1e-6 * k


@pytest.mark.parametrize("b,seeds", [(4, 2000), (6, 1500), (8, 600)])
def test_size_statistics(orc, b, seeds):
    # Sec. 4.1: asymptotically unbiased with relative standard deviation
    # beta_p/sqrt(p) <= 1.06/sqrt(p) (13.18% quoted at p = 64).
    p = 1 << b
    N = 20 * p
    est = np.empty(seeds)
    for s in range(seeds):
        M = orc.new_counter(b)
        for x in range(N):
            orc.add(M, b, x, 1000 + s)
        est[s] = orc.size(M, b)
    rel = est / N
    rsd = rel.std(ddof=1)
    se_mean = rsd / math.sqrt(seeds)
    assert abs(rel.mean() - 1.0) < 4 * se_mean
    assert 0.85 * 1.04 / math.sqrt(p) < rsd < 1.06 / math.sqrt(p) * 1.12
