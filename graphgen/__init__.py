"""Seeded synthetic graphs in compressed-sparse-row form.

This package is the single source of inputs for both sides of the HyperBall
checks: the HIP library under test and the CPU oracle.  It draws arcs and
builds CSR arrays; it contains none of the HyperBall method's arithmetic.

Graph families (recipes in ``graphgen.cpp``):

* ``rmat``  - R-MAT with (a, b, c, d) = (0.57, 0.19, 0.19, 0.05) by default,
  ``edge_factor * 2**scale`` drawn arcs, self-loops and duplicates removed,
  optionally symmetrised (undirected), transposed and relabelled by a seeded
  random permutation.
* ``ba``    - Barabasi-Albert, m edges per new node from an m-clique seed.
* ``ws``    - Watts-Strogatz ring lattice, k neighbours, rewiring beta.
* small deterministic shapes (path, cycle, star, complete, grid) used by the
  closed-form checks.

Every function returns ``(offsets, indices)``: int64 ``offsets`` of length
n+1 and int32 ``indices`` of length m; row v lists the successors of v.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "graphgen.cpp")
_LIB = os.path.join(_HERE, "libgraphgen.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile ``libgraphgen.so`` next to its source (host code, g++ + OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["g++", "-O3", "-std=c++17", "-fopenmp", "-fPIC", "-shared", _SRC, "-o", tmp]
        )
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        lib = ctypes.CDLL(_LIB)
        i64, i32p, i64p, u64 = ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_uint64
        lib.gg_rmat_arcs.argtypes = [ctypes.c_int, i64, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_double, u64, i32p, i32p]
        lib.gg_rmat_arcs.restype = None
        lib.gg_permutation.argtypes = [i64, u64, i32p]
        lib.gg_permutation.restype = None
        lib.gg_relabel.argtypes = [i64, i32p, i32p]
        lib.gg_relabel.restype = None
        lib.gg_csr.argtypes = [i64, i64, i32p, i32p, ctypes.c_int, ctypes.c_int, i64p, i32p]
        lib.gg_csr.restype = i64
        lib.gg_ba_edges.argtypes = [i64, ctypes.c_int, u64, i32p, i32p]
        lib.gg_ba_edges.restype = i64
        lib.gg_ws_edges.argtypes = [i64, ctypes.c_int, ctypes.c_double, u64, i32p, i32p]
        lib.gg_ws_edges.restype = i64
        lib.gg_batch_arcs.argtypes = [ctypes.c_int32, i64, ctypes.c_int]
        lib.gg_batch_arcs.restype = i64
        lib.gg_batch_build.argtypes = [ctypes.c_int32, i32p, i64p, i64p, ctypes.c_int, ctypes.c_int,
                                       ctypes.c_double, i64p, i64p, i64p, i32p]
        lib.gg_batch_build.restype = ctypes.c_int32
        lib.gg_num_threads.argtypes = []
        lib.gg_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def csr_from_pairs(n: int, rows: np.ndarray, cols: np.ndarray, drop_self: bool = True,
                   dedup: bool = True):
    """CSR whose row r lists, sorted, every c with (r, c) among the pairs."""
    lib = _load()
    rows = np.ascontiguousarray(rows, dtype=np.int32)
    cols = np.ascontiguousarray(cols, dtype=np.int32)
    m = rows.shape[0]
    offsets = np.empty(n + 1, dtype=np.int64)
    out = np.empty(max(m, 1), dtype=np.int32)
    got = lib.gg_csr(n, m, _ptr(rows), _ptr(cols), int(drop_self), int(dedup), _ptr(offsets), _ptr(out))
    if got < 0:
        raise ValueError("pair names a node outside [0, n)")
    return offsets, out[:got].copy()


def symmetric_pairs(src: np.ndarray, dst: np.ndarray):
    return np.concatenate([src, dst]), np.concatenate([dst, src])


def permutation(n: int, seed: int) -> np.ndarray:
    perm = np.empty(n, dtype=np.int32)
    _load().gg_permutation(n, seed, _ptr(perm))
    return perm


def rmat_arcs(scale: int, n_arcs: int, seed: int, a=0.57, b=0.19, c=0.19):
    src = np.empty(n_arcs, dtype=np.int32)
    dst = np.empty(n_arcs, dtype=np.int32)
    _load().gg_rmat_arcs(scale, n_arcs, a, b, c, seed, _ptr(src), _ptr(dst))
    return src, dst


def rmat(scale: int, edge_factor: int, seed: int, *, directed: bool = True,
         transpose: bool = False, relabel: bool = False, relabel_seed: int | None = None,
         a=0.57, b=0.19, c=0.19):
    """R-MAT CSR.

    directed=False symmetrises the arcs.  transpose=True returns the CSR of the
    transposed graph (row v lists the predecessors of v).  relabel=True maps
    node ids through a seeded random permutation before building rows.
    """
    n = 1 << scale
    src, dst = rmat_arcs(scale, edge_factor * n, seed, a, b, c)
    if relabel:
        perm = permutation(n, seed if relabel_seed is None else relabel_seed)
        lib = _load()
        lib.gg_relabel(src.shape[0], _ptr(perm), _ptr(src))
        lib.gg_relabel(dst.shape[0], _ptr(perm), _ptr(dst))
    if not directed:
        rows, cols = symmetric_pairs(src, dst)
    elif transpose:
        rows, cols = dst, src
    else:
        rows, cols = src, dst
    del src, dst
    return csr_from_pairs(n, rows, cols)


def ba(n: int, m: int, seed: int):
    """Undirected Barabasi-Albert graph as a symmetric CSR."""
    lib = _load()
    mm = min(m, n)
    cap = mm * (mm - 1) // 2 + mm * max(n - mm, 0)
    src = np.empty(max(cap, 1), dtype=np.int32)
    dst = np.empty(max(cap, 1), dtype=np.int32)
    e = lib.gg_ba_edges(n, m, seed, _ptr(src), _ptr(dst))
    rows, cols = symmetric_pairs(src[:e], dst[:e])
    return csr_from_pairs(n, rows, cols)


def ws(n: int, k: int, beta: float, seed: int):
    """Undirected Watts-Strogatz graph as a symmetric CSR."""
    lib = _load()
    cap = n * (k // 2)
    src = np.empty(max(cap, 1), dtype=np.int32)
    dst = np.empty(max(cap, 1), dtype=np.int32)
    e = lib.gg_ws_edges(n, k, beta, seed, _ptr(src), _ptr(dst))
    rows, cols = symmetric_pairs(src[:e], dst[:e])
    return csr_from_pairs(n, rows, cols)


def random_digraph(n: int, m: int, seed: int, self_loops: bool = False, dedup: bool = True):
    """Uniform random directed graph: m arcs with uniform endpoints (numpy PCG64)."""
    rng = np.random.default_rng(seed)
    src = rng.integers(0, max(n, 1), size=m, dtype=np.int64).astype(np.int32)
    dst = rng.integers(0, max(n, 1), size=m, dtype=np.int64).astype(np.int32)
    return csr_from_pairs(n, src, dst, drop_self=not self_loops, dedup=dedup)


# --- small deterministic shapes -------------------------------------------------

def from_edges(n: int, edges, undirected: bool = False):
    e = np.asarray(list(edges), dtype=np.int32).reshape(-1, 2)
    src, dst = e[:, 0], e[:, 1]
    if undirected:
        src, dst = symmetric_pairs(src, dst)
    return csr_from_pairs(n, src, dst)


def directed_cycle(n: int):
    return from_edges(n, [(i, (i + 1) % n) for i in range(n)])


def directed_path(n: int):
    return from_edges(n, [(i, i + 1) for i in range(n - 1)])


def undirected_path(n: int):
    return from_edges(n, [(i, i + 1) for i in range(n - 1)], undirected=True)


def star(n: int):
    """Undirected star: node 0 is the centre, nodes 1..n-1 are leaves."""
    return from_edges(n, [(0, i) for i in range(1, n)], undirected=True)


def complete(n: int):
    return from_edges(n, [(i, j) for i in range(n) for j in range(n) if i != j])


def grid(rows: int, cols: int):
    """Undirected rows x cols grid."""
    e = []
    for r in range(rows):
        for c in range(cols):
            v = r * cols + c
            if c + 1 < cols:
                e.append((v, v + 1))
            if r + 1 < rows:
                e.append((v, v + cols))
    return from_edges(rows * cols, e, undirected=True)


def empty(n: int):
    return np.zeros(n + 1, dtype=np.int64), np.zeros(0, dtype=np.int32)


def transpose(offsets: np.ndarray, indices: np.ndarray):
    n = offsets.shape[0] - 1
    rows = np.repeat(np.arange(n, dtype=np.int32), np.diff(offsets))
    return csr_from_pairs(n, indices, rows, drop_self=False, dedup=False)


def batch(kinds, ns, seeds, ba_m: int = 4, ws_k: int = 10, ws_beta: float = 0.1):
    """Many undirected graphs at once (C, parallel over graphs): kinds[i] 0 =
    Barabasi-Albert (ba_m edges per node), 1 = Watts-Strogatz (ws_k, ws_beta).
    Returns a list of (offsets, indices) views into two shared arrays."""
    lib = _load()
    kinds = np.ascontiguousarray(kinds, dtype=np.int32)
    ns = np.ascontiguousarray(ns, dtype=np.int64)
    seeds = np.ascontiguousarray(seeds, dtype=np.uint64)
    k = kinds.shape[0]
    arcs = np.array([lib.gg_batch_arcs(int(kinds[i]), int(ns[i]), ba_m if kinds[i] == 0 else ws_k)
                     for i in range(k)], dtype=np.int64)
    off_start = np.concatenate([[0], np.cumsum(ns + 1)[:-1]]).astype(np.int64)
    idx_start = np.concatenate([[0], np.cumsum(arcs)[:-1]]).astype(np.int64)
    offsets_all = np.empty(int((ns + 1).sum()), dtype=np.int64)
    indices_all = np.empty(max(int(arcs.sum()), 1), dtype=np.int32)
    bad = lib.gg_batch_build(k, _ptr(kinds), _ptr(ns), _ptr(seeds), ba_m, ws_k, ws_beta, _ptr(off_start),
                             _ptr(idx_start), _ptr(offsets_all), _ptr(indices_all))
    if bad:
        raise RuntimeError(f"graph {bad - 1}: unexpected edge count")
    return [(offsets_all[off_start[i]:off_start[i] + ns[i] + 1],
             indices_all[idx_start[i]:idx_start[i] + arcs[i]]) for i in range(k)]


def batch_workload(count: int = 4096, n_min: int = 1000, n_max: int = 200_000, seed: int = 4):
    """The batched workload: `count` graphs, first half Barabasi-Albert (m = 4),
    second half Watts-Strogatz (k = 10, beta = 0.1), sizes log-uniform in
    [n_min, n_max] drawn with numpy's PCG64 from `seed`."""
    rng = np.random.default_rng(seed)
    ns = np.exp(rng.uniform(np.log(n_min), np.log(n_max), size=count)).astype(np.int64)
    kinds = (np.arange(count) >= count // 2).astype(np.int32)
    gseeds = rng.integers(1, 2**62, size=count, dtype=np.int64).astype(np.uint64)
    return batch(kinds, ns, gseeds)
