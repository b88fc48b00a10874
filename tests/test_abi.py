"""CPU checks of the C ABI boundary: the library loads, exports every entry
point that include/hb.h declares, and rejects bad arguments on the host
before touching a device."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for fname in os.listdir(os.path.join(ROOT, "include")):
        if not fname.endswith(".h"):
            continue
        text = open(os.path.join(ROOT, "include", fname)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(hb_[a-z_]+)\s*\(", text, re.M):
            names.add(m.group(1))
    return names


def test_header_declares_the_boundary():
    names = declared_functions()
    for n in ("hb_init", "hb_iterate", "hb_centralities", "hb_free", "hb_run", "hb_reset",
              "hb_get_registers", "hb_stats", "hb_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    import paper_1308_2144_amd as hb

    raw = ctypes.CDLL(hb.LIB_PATH)
    missing = [n for n in sorted(declared_functions()) if not hasattr(raw, n)]
    assert not missing, missing
    assert hb.hb_version() == 1


def test_host_side_argument_errors():
    import paper_1308_2144_amd as hb

    off = np.array([0, 1, 2], dtype=np.int64)
    idx = np.array([1, 0], dtype=np.int32)
    for b in (3, 17, -1):
        with pytest.raises(hb.HBError) as e:
            hb.hb_init(off, idx, b, 1)
        assert e.value.status == hb.HB_EINVAL and "log2m" in str(e.value)
    with pytest.raises(hb.HBError) as e:
        hb.hb_init(np.array([0, 1, 3], dtype=np.int64), idx, 4, 1)   # offsets[n] != m
    assert e.value.status == hb.HB_EINVAL
    with pytest.raises(hb.HBError) as e:
        hb.hb_init(np.array([1, 1, 2], dtype=np.int64), idx, 4, 1)   # offsets[0] != 0
    assert e.value.status == hb.HB_EINVAL
    L = hb.lib()
    assert L.hb_init(None, None, 4, 1, None, None) == hb.HB_EINVAL
    assert b"NULL" in L.hb_last_error()
    ctx = ctypes.c_void_p()
    assert L.hb_init(ctypes.byref(ctx), None, 4, 1, None, None) == hb.HB_EINVAL
    # context-less calls fail cleanly, hb_free(NULL) is a no-op
    assert L.hb_iterate(None, None) == hb.HB_EINVAL
    assert L.hb_run(None, 0, None) == hb.HB_EINVAL
    assert L.hb_centralities(None, None, None, None, None, 0) == hb.HB_EINVAL
    assert L.hb_get_registers(None, None, 0) == hb.HB_EINVAL
    assert L.hb_reset(None, 1) == hb.HB_EINVAL
    L.hb_free(None)


def test_default_options():
    import paper_1308_2144_amd as hb

    o = hb.default_options()
    assert o.frontier == 1 and o.validate == 1 and o.timing == 0
    assert 0 < o.light_max < o.heavy_min and o.chunk > 0
    with pytest.raises(TypeError):
        hb.default_options(nonsense=1)


def test_binding_refuses_mixed_inputs():
    import paper_1308_2144_amd as hb
    import torch

    with pytest.raises(TypeError):
        hb.hb_init(torch.zeros(2, dtype=torch.int64), np.zeros(1, dtype=np.int32), 4, 1)


def test_autotune_argument_errors():
    import paper_1308_2144_amd as hb

    g = [(np.array([0, 1, 2], dtype=np.int64), np.array([1, 0], dtype=np.int32))]
    with pytest.raises(hb.HBError) as e:
        hb.hb_batch_autotune(g, 3, [1])
    assert e.value.status == hb.HB_EINVAL
    with pytest.raises(hb.HBError) as e:
        hb.hb_batch_autotune(g, 9, [1])
    assert e.value.status == hb.HB_EINVAL
    L = hb.lib()
    assert L.hb_batch_autotune(None, 0, 5, None, 0, None, None, None) == hb.HB_EINVAL


def test_ensemble_argument_errors():
    """Refused on the host before any device work."""
    import paper_1308_2144_amd as hb

    off = np.array([0, 1, 2], dtype=np.int64)
    idx = np.array([1, 0], dtype=np.int32)
    for b, seeds in ((4, [1, 2, 3]), (4, list(range(32))), (6, list(range(8))), (3, [1, 2]), (9, [1, 2]),
                     (4, [1])):
        with pytest.raises(hb.HBError) as e:
            hb.Ensemble(off, idx, b, seeds)
        assert e.value.status == hb.HB_EINVAL
    with pytest.raises(hb.HBError) as e:
        hb.Ensemble(np.array([0, 1, 3], dtype=np.int64), idx, 4, [1, 2])    # offsets[n] != m
    assert e.value.status == hb.HB_EINVAL


def test_distance_stats_equal_oracle():
    """hb_distance_stats is host arithmetic: equal to the oracle's bit for bit."""
    import oracle
    import paper_1308_2144_amd as hb

    rng = np.random.default_rng(8)
    for T in (1, 2, 5, 17, 60):
        N = np.cumsum(rng.lognormal(3.0, 1.0, size=T))
        for alpha in (0.5, 0.9, 0.99):
            got, ref = hb.hb_distance_stats(N, alpha), oracle.distance_stats(N, alpha)
            assert got == ref
    assert hb.hb_distance_stats([5.0]) == oracle.distance_stats([5.0])
    with pytest.raises(hb.HBError):
        hb.hb_distance_stats([])


def test_batch_argument_errors():
    """Malformed graphs of a batch are refused while the host arena is filled,
    before any device work, with the index of the first bad graph."""
    import paper_1308_2144_amd as hb

    good = (np.array([0, 1, 2], dtype=np.int64), np.array([1, 0], dtype=np.int32))
    bad_idx = (np.array([0, 1, 2], dtype=np.int64), np.array([1, 2], dtype=np.int32))     # id 2 >= n
    bad_off = (np.array([0, 2, 1], dtype=np.int32), np.array([1, 0], dtype=np.int32))     # decreasing
    for graphs, msg in (([good, bad_idx], "graph 1: index outside"), ([bad_off, good], "graph 0: malformed offsets"),
                        ([good] * 40 + [bad_idx], "graph 40: index outside")):
        with pytest.raises(hb.HBError) as e:
            hb.hb_batch_init(graphs, 5, np.arange(len(graphs), dtype=np.uint64))
        assert e.value.status == hb.HB_EINVAL and msg in str(e.value), str(e.value)
    for b in (3, 9):
        with pytest.raises(hb.HBError) as e:
            hb.hb_batch_init([good], b, [1])
        assert e.value.status == hb.HB_EINVAL
    with pytest.raises(ValueError):
        hb.hb_batch_init([good, good], 5, [1])       # one seed per graph (checked by the binding)
    empty = (np.zeros(1, dtype=np.int64), np.zeros(0, dtype=np.int32))
    with pytest.raises(hb.HBError) as e:
        hb.hb_batch_init([empty, empty], 5, [1, 2])  # nothing to compute
    assert e.value.status == hb.HB_EINVAL and "at least one graph with nodes" in str(e.value)


def test_discount_table_is_host_only_and_matches_the_oracle():
    """hb_discount_table needs no device; its values equal the oracle's own
    Sec. 7 tables bit for bit (both evaluate the definitions with the host
    libm), and unknown kinds are refused."""
    import oracle
    import paper_1308_2144_amd as hb

    for kind in ("harmonic", "quadratic", "logarithmic", "constant"):
        assert np.array_equal(hb.discount_table(kind, 100), oracle.discount_table(kind, 100)), kind
    L = hb.lib()
    f = np.zeros(4)
    assert L.hb_discount_table(9, 4, f.ctypes.data) == hb.HB_EINVAL
    assert L.hb_discount_table(0, 0, f.ctypes.data) == hb.HB_EINVAL
    assert L.hb_discount_table(0, 4, None) == hb.HB_EINVAL
