"""CPU oracle for HyperBall (test infrastructure).

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The HIP library never loads it, and the
two share no code: the oracle is a plain single-threaded C implementation of
Algorithms 1 and 2 of the paper (``hb_oracle.c``), wrapped here with ctypes.

Parity status of every function (pins live in ``tests/test_oracle_*.py``):

* ``hash64``/``rho``/``add``  - pinned: published SplitMix64 outputs, the
  paper's rho+ example, uniformity of index and rank.
* ``register_sum``           - pinned: Python's correctly rounded int->float.
* ``size``                   - pinned: closed forms (constant registers,
  single register), exact small-set regime, statistical bias/RSD vs Sec. 4.1.
* ``run``                    - pinned: registers equal the HyperLogLog state of
  breadth-first balls (computed with scipy), termination count, closed-form
  accumulators on cycles, paths, stars, complete graphs in the exact regime.
* ``node``                   - pinned: agrees with ``run`` and with closed forms;
  with weights and a discount table it agrees with ``run_ext`` bit for bit.
* ``finalize``               - pinned: closed forms on the same graphs.
* ``run_ext``                - ``run`` with Sec. 6 node weights (replicas),
  a Sec. 7 discount accumulator and the per-pass estimate trace; pinned:
  unit weights and no discount reproduce ``run`` bit for bit, f(d) = d
  reproduces S bit for bit, weighted distance sums and discounted sums
  against breadth-first distances in the exact regime, the replica counter
  against ``counter_of``.
* ``neighbourhood``          - N(t) = correctly rounded sum over nodes of the
  estimates after t passes (``math.fsum`` of the trace); pinned: exact-regime
  ball sizes from breadth-first search.
* ``discount_table``         - the Sec. 7 discounts; pinned: exact values
  (1/d, 1/d^2, log2(d+1) at d = 2^k - 1, constant 1).
* ``distance_stats``         - average distance and interpolated effective
  diameter from N(t); pinned: closed forms on paths and cycles.
* ``ensemble``               - K independent runs (Sec. 5: several runs of
  HyperBall), one ``run`` + ``finalize`` per seed; pinned through ``run``.
* ``ensemble_summary``       - pinned: numpy's mean and std (ddof=1), and
  closed forms (equal values, two values, arithmetic progressions).
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hb_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


_LIB_OMP = os.path.join(_HERE, "liboracle_omp.so")
_lib_omp = None


def build(force: bool = True) -> str:
    """Compile the oracle (gcc -O3, no FMA contraction, no fast-math), and the
    OpenMP build of the same file that only the all-core CPU baseline uses."""
    from oracle.build import build as _build

    return _build(force)


def _declare(L):
    vp, i64, u64, ci = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_int
    L.hbo_hash.argtypes = [u64, u64]
    L.hbo_hash.restype = u64
    L.hbo_rho.argtypes = [u64, ci]
    L.hbo_rho.restype = ci
    L.hbo_add.argtypes = [vp, ci, u64, u64]
    L.hbo_add.restype = None
    L.hbo_alpha.argtypes = [ci]
    L.hbo_alpha.restype = ctypes.c_double
    L.hbo_register_sum.argtypes = [vp, ci]
    L.hbo_register_sum.restype = ctypes.c_double
    L.hbo_size.argtypes = [vp, ci]
    L.hbo_size.restype = ctypes.c_double
    L.hbo_run.argtypes = [i64, vp, vp, ci, u64, ci, vp, vp, vp, vp, vp]
    L.hbo_run.restype = ci
    L.hbo_run_ext.argtypes = [i64, vp, vp, ci, u64, ci, vp, vp, ci, vp, vp, vp, vp, vp, i64, vp, vp]
    L.hbo_run_ext.restype = ci
    L.hbo_finalize.argtypes = [i64, vp, ci, vp, vp, vp, vp, vp, vp]
    L.hbo_finalize.restype = None
    L.hbo_node.argtypes = [i64, vp, vp, ci, u64, i64, ci, vp, vp, vp, vp, vp]
    L.hbo_node.restype = ci
    L.hbo_node_ext.argtypes = [i64, vp, vp, ci, u64, i64, ci, vp, vp, ci, vp, vp, vp, vp, vp, vp]
    L.hbo_node_ext.restype = ci
    L.hbo_run_full.argtypes = [i64, vp, vp, ci, u64, ci, vp, vp, ci, vp, vp, vp, vp, vp, i64, vp, vp, vp]
    L.hbo_run_full.restype = ci
    L.hbo_init_counters.argtypes = [i64, ci, u64, vp, vp]
    L.hbo_init_counters.restype = None
    L.hbo_pass.argtypes = [vp, vp, ci, ci, vp, vp, vp, vp, ctypes.c_double, vp, vp, i64, i64]
    L.hbo_pass.restype = i64
    L.hbo_discount.argtypes = [ci, ci]
    L.hbo_discount.restype = ctypes.c_double
    L.hbo_threads.argtypes = []
    L.hbo_threads.restype = ci
    return L


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=False)
        _lib = _declare(ctypes.CDLL(_LIB))
    return _lib


def _load_omp():
    global _lib_omp
    if _lib_omp is None:
        if not os.path.exists(_LIB_OMP):
            build(force=False)
        _lib_omp = _declare(ctypes.CDLL(_LIB_OMP))
    return _lib_omp


def _p(a):
    return None if a is None else a.ctypes.data


def hash64(x: int, seed: int) -> int:
    return _load().hbo_hash(x, seed)


def rho(h: int, b: int) -> int:
    return _load().hbo_rho(h, b)


def alpha(b: int) -> float:
    return _load().hbo_alpha(b)


def new_counter(b: int) -> np.ndarray:
    return np.zeros(1 << b, dtype=np.uint8)


def add(M: np.ndarray, b: int, item: int, seed: int) -> None:
    assert M.dtype == np.uint8 and M.flags.c_contiguous and M.shape == (1 << b,)
    _load().hbo_add(_p(M), b, item, seed)


def counter_of(items, b: int, seed: int) -> np.ndarray:
    M = new_counter(b)
    for x in items:
        add(M, b, int(x), seed)
    return M


def register_sum(M: np.ndarray, b: int) -> float:
    M = np.ascontiguousarray(M, dtype=np.uint8)
    return _load().hbo_register_sum(_p(M), b)


def size(M: np.ndarray, b: int) -> float:
    M = np.ascontiguousarray(M, dtype=np.uint8)
    return _load().hbo_size(_p(M), b)


def _csr(offsets, indices):
    o = np.ascontiguousarray(offsets, dtype=np.int64)
    i = np.ascontiguousarray(indices, dtype=np.int32)
    if i.size == 0:
        i = np.zeros(1, dtype=np.int32)
    return o, i


def run(offsets, indices, b: int, seed: int, max_passes: int = 0, lastmod: bool = False):
    """Algorithm 2 to stabilisation (or max_passes passes).

    Returns dict(regs (n, p) uint8, S, H float64, nmod int64 per pass, passes),
    and with lastmod=True also lastmod (n int32: 1 + the last pass that
    changed the node's counter, 0 if none did).
    """
    o, i = _csr(offsets, indices)
    n = o.shape[0] - 1
    p = 1 << b
    regs = np.zeros((max(n, 1), p), dtype=np.uint8)
    S = np.zeros(max(n, 1))
    H = np.zeros(max(n, 1))
    lm = np.zeros(max(n, 1), dtype=np.int32) if lastmod else None
    cap = max_passes if max_passes > 0 else n + 2
    nmod = np.zeros(cap + 1, dtype=np.int64)
    passes = ctypes.c_int(0)
    rc = _load().hbo_run_full(n, _p(o), _p(i), b, seed, max_passes, None, None, 0, _p(regs), _p(S), _p(H),
                              None, None, 0, _p(nmod), _p(lm), ctypes.byref(passes))
    if rc != 0:
        raise RuntimeError("oracle run failed")
    t = passes.value
    out = dict(regs=regs[:n], S=S[:n], H=H[:n], nmod=nmod[:t].copy(), passes=t)
    if lastmod:
        out["lastmod"] = lm[:n]
    return out


def threads(all_cores: bool = False) -> int:
    """Threads a pass uses: 1 for the oracle proper; with all_cores, those of
    the OpenMP build of the same source (OMP_NUM_THREADS, else every core)."""
    return (_load_omp() if all_cores else _load()).hbo_threads()


def first_pass_rows(offsets, indices, b: int, seed: int, v_begin: int, v_end: int, all_cores: bool = False):
    """Pass 0 of ``run`` over the rows [v_begin, v_end) only, timed: the
    counters of every node are set to radius 0 first (not timed), then the
    pass's node loop runs over the range (the same function ``run`` calls,
    from the plain or, with all_cores, the OpenMP build).  Used for the CPU
    baseline on a bounded sample of a large graph.

    Returns dict(seconds, changed, next (rows of the range, radius-1
    counters), S, H over the range, threads)."""
    import time

    L = _load_omp() if all_cores else _load()
    o, i = _csr(offsets, indices)
    n = o.shape[0] - 1
    p = 1 << b
    if not (0 <= v_begin <= v_end <= n):
        raise ValueError("row range outside the graph")
    c = np.empty(max(n, 1) * p, dtype=np.uint8)
    L.hbo_init_counters(n, b, seed, None, _p(c))
    nxt = np.zeros(max(n, 1) * p, dtype=np.uint8)
    S = np.zeros(max(n, 1))
    H = np.zeros(max(n, 1))
    t0 = time.perf_counter()
    changed = L.hbo_pass(_p(o), _p(i), b, 0, _p(c), _p(nxt), _p(S), _p(H), 0.0, None, None, v_begin, v_end)
    dt = time.perf_counter() - t0
    return dict(seconds=dt, changed=int(changed), next=nxt[v_begin * p:v_end * p].reshape(-1, p).copy(),
                S=S[v_begin:v_end].copy(), H=H[v_begin:v_end].copy(), threads=L.hbo_threads())


def replica_item(x: int, j: int) -> int:
    """Item of replica j of node x (Sec. 6): x for j = 0, x + j * 2^32 after."""
    return x + (j << 32)


def run_ext(offsets, indices, b: int, seed: int, max_passes: int = 0, weights=None, discount=None,
            trace: bool = False):
    """``run`` with node weights w(x) >= 1 (counter x starts as the
    HyperLogLog of the w(x) replicas of x, Sec. 6), a discount table
    f(1..L) (D[v] += f(t+1) * delta in pass t, f(d) = f(L) for d > L,
    Sec. 7), and the trace of every counter's estimate after each pass.

    Returns run()'s dict plus D (if discount) and etrace ((passes+1, n), if
    trace)."""
    o, i = _csr(offsets, indices)
    n = o.shape[0] - 1
    p = 1 << b
    regs = np.zeros((max(n, 1), p), dtype=np.uint8)
    S = np.zeros(max(n, 1))
    H = np.zeros(max(n, 1))
    D = np.zeros(max(n, 1))
    cap = max_passes if max_passes > 0 else n + 2
    nmod = np.zeros(cap + 1, dtype=np.int64)
    w = None if weights is None else np.ascontiguousarray(weights, dtype=np.int32)
    if w is not None and (w.shape[0] != n or (n and w.min() < 1)):
        raise ValueError("need one weight >= 1 per node")
    f = None if discount is None else np.ascontiguousarray(discount, dtype=np.float64)
    rows = cap + 1 if trace else 0
    if trace and rows * max(n, 1) > (1 << 25):
        # large graph: learn the pass count first, then trace exactly that many rows
        rows = run_ext(offsets, indices, b, seed, max_passes=max_passes, weights=weights)["passes"] + 1
    et = np.zeros((max(rows, 1), max(n, 1))) if trace else None
    passes = ctypes.c_int(0)
    rc = _load().hbo_run_ext(n, _p(o), _p(i), b, seed, max_passes, None if w is None else _p(w),
                             None if f is None else _p(f), 0 if f is None else f.shape[0], _p(regs), _p(S), _p(H),
                             _p(D), None if et is None else _p(et), rows, _p(nmod), ctypes.byref(passes))
    if rc != 0:
        raise RuntimeError("oracle run failed")
    t = passes.value
    out = dict(regs=regs[:n], S=S[:n], H=H[:n], nmod=nmod[:t].copy(), passes=t)
    if f is not None:
        out["D"] = D[:n]
    if trace:
        out["etrace"] = et[: t + 1, :n].copy()
    return out


DISCOUNTS = {"harmonic": 0, "quadratic": 1, "logarithmic": 2, "constant": 3}


def discount_table(kind: str, length: int = 64) -> np.ndarray:
    """f(1..length) of the discounts Sec. 7 names: harmonic 1/d, quadratic
    1/d^2, logarithmic 1/log2(d+1), constant 1."""
    L = _load()
    return np.array([L.hbo_discount(DISCOUNTS[kind], d) for d in range(1, length + 1)], dtype=np.float64)


def neighbourhood(etrace) -> np.ndarray:
    """N(t) for t = 0..passes: the sum over nodes of the size estimates after
    t passes (an estimate of the number of pairs (x, y) with y in B(x, t)),
    correctly rounded (math.fsum)."""
    import math

    return np.array([math.fsum(row.tolist()) for row in np.asarray(etrace)])


def distance_stats(N, alpha: float = 0.9):
    """From the neighbourhood function N(0..T): reachable pairs at distance
    >= 1 (N(T) - N(0)), the average distance sum_{t>=1} t (N(t) - N(t-1)) /
    (N(T) - N(0)), and the effective diameter: the smallest t with N(t) >=
    alpha N(T), interpolated linearly between t-1 and t.  Sums in t order."""
    N = [float(x) for x in N]
    T = len(N) - 1
    pairs = N[T] - N[0]
    num = 0.0
    for t in range(1, T + 1):
        num = num + float(t) * (N[t] - N[t - 1])
    avg = num / pairs if pairs > 0 else 0.0
    target = alpha * N[T]
    eff = 0.0
    for t in range(0, T + 1):
        if N[t] >= target:
            eff = float(t) if t == 0 else float(t - 1) + (target - N[t - 1]) / (N[t] - N[t - 1])
            break
    return dict(pairs=pairs, average_distance=avg, effective_diameter=eff)


def finalize(regs: np.ndarray, b: int, S: np.ndarray, H: np.ndarray):
    """Closeness, Lin, harmonic and coreachable-set size per node."""
    n = regs.shape[0]
    regs = np.ascontiguousarray(regs, dtype=np.uint8)
    S = np.ascontiguousarray(S, dtype=np.float64)
    H = np.ascontiguousarray(H, dtype=np.float64)
    out = [np.zeros(max(n, 1)) for _ in range(4)]
    _load().hbo_finalize(n, _p(regs), b, _p(S), _p(H), *(_p(a) for a in out))
    clo, lin, harm, core = (a[:n] for a in out)
    return dict(closeness=clo, lin=lin, harmonic=harm, coreach=core)


def node(offsets, indices, b: int, seed: int, x: int, radius: int = -1, weights=None, discount=None):
    """Per-node evaluation from breadth-first balls (with optional node
    weights and discount table, as in run_ext).

    Returns dict(regs (registers of B(x, radius), or of the reachable set when
    radius < 0), S, H, D (with a discount), last_change, ecc).
    """
    o, i = _csr(offsets, indices)
    n = o.shape[0] - 1
    regs = new_counter(b)
    S = ctypes.c_double(0.0)
    H = ctypes.c_double(0.0)
    D = ctypes.c_double(0.0)
    last = ctypes.c_int(0)
    ecc = ctypes.c_int(0)
    w = None if weights is None else np.ascontiguousarray(weights, dtype=np.int32)
    f = None if discount is None else np.ascontiguousarray(discount, dtype=np.float64)
    rc = _load().hbo_node_ext(n, _p(o), _p(i), b, seed, x, radius, None if w is None else _p(w),
                              None if f is None else _p(f), 0 if f is None else f.shape[0], _p(regs),
                              ctypes.byref(S), ctypes.byref(H), ctypes.byref(D), ctypes.byref(last),
                              ctypes.byref(ecc))
    if rc != 0:
        raise RuntimeError("oracle node evaluation failed")
    out = dict(regs=regs, S=S.value, H=H.value, last_change=last.value, ecc=ecc.value)
    if f is not None:
        out["D"] = D.value
    return out


def ensemble(offsets, indices, b: int, seeds, max_passes: int = 0):
    """K independent runs, one per hash seed (Sec. 5 suggests repeating the
    computation and reporting the spread).  Returns a list of run dicts with
    the finalize() outputs merged in."""
    out = []
    for sd in seeds:
        r = run(offsets, indices, b, int(sd), max_passes=max_passes)
        r.update(finalize(r["regs"], b, r["S"], r["H"]))
        out.append(r)
    return out


def ensemble_summary(values):
    """Mean and empirical standard deviation over runs of per-node values
    (array (n, K)): mean = (x_0 + x_1 + ... + x_{K-1}) / K summed in run
    order, sd = sqrt(sum_k (x_k - mean)^2 / (K - 1)), the squares also summed
    in run order."""
    x = np.asarray(values, dtype=np.float64)
    K = x.shape[1]
    m = x[:, 0].copy()
    for k in range(1, K):
        m = m + x[:, k]
    m = m / float(K)
    q = np.zeros_like(m)
    for k in range(K):
        d = x[:, k] - m
        q = q + d * d
    sd = np.sqrt(q / float(K - 1)) if K > 1 else np.zeros_like(m)
    return m, sd
