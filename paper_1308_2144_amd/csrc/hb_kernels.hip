// HIP kernels of the HyperBall pass for gfx950 (MI355X).
//
// Data layout in HBM:
//   counters  two buffers of n * p bytes, node-major (register j of node v at
//             v*p + j); pass t reads `cur` and writes `nxt`, then they swap.
//   bitmaps   two arrays of ceil(n/64) words; bit v of mod_prev says the
//             counter of v changed in the previous pass.
//   S, H, E   doubles per node: the two accumulators of Sec. 5 and the size
//             estimate of the current counter (cached so that a pass only
//             evaluates the estimator once per changed node).
//
// One pass (Algorithm 2, one iteration of the do-loop):
//   a = c[v] U (U over arcs v->w of c[w])       (register-wise max, Sec. 4.2)
// with two exact shortcuts:
//   * edge skipping: a successor whose counter did not change in the previous
//     pass is already contained in c[v] (c_t(v) contains c_{t-1}(w) for every
//     arc v->w), so only changed successors are gathered;
//   * write skipping: the next buffer still holds c_{t-1}(v), which equals
//     c_t(v) unless v changed in the previous pass; so a counter is written
//     only if it changes now or changed in the previous pass.
// A changed counter's estimate E(a) is computed in the same kernel and the
// increments delta*(t+1) and delta/(t+1) are added to S and H (Sec. 5).
//
// Work decomposition (degree-aware): a 64-row block per wavefront.  Each
// counter is handled by a group of G = p/16 lanes, every lane owning 16
// bytes; a wavefront holds W = 64/G groups.  Rows with <= light_max arcs are
// dealt to the groups round-robin; rows up to heavy_min arcs are processed by
// the whole wavefront (groups stride over the arcs, then reduce by shuffles);
// heavier rows are cut into chunks reduced by separate workgroups into
// partial counters that a second kernel merges.  Counters wider than 256
// bytes use a one-workgroup-per-block kernel.
//
// There is no dense contraction here: the pass is a gather of p-byte rows and
// byte-wise maxima, bound by HBM bandwidth, so no MFMA is involved.
#include <algorithm>

#include <hipcub/hipcub.hpp>

#include "hb_internal.h"

namespace hb {
namespace {

// Compile-time tuning: successor counters in flight per lane group, a cap on
// waves per SIMD for the expand kernels (0: compiler's choice), and
// non-temporal hints for data that is streamed once per pass.
#ifndef HB_U
#define HB_U 8
#endif
#ifndef HB_WAVES
#define HB_WAVES 5
#endif
#ifndef HB_NT
#define HB_NT 0
#endif
constexpr int U = HB_U;

// Kernel flavours of the fused estimator/accumulator step: one counter per
// row; an ensemble row of several seeds' counters; one counter per row plus
// the discounted-gain accumulator.
constexpr int FL_PLAIN = 0;
constexpr int FL_ENS = 1;
constexpr int FL_DISC = 2;

template <class T>
__device__ __forceinline__ T ld_stream(const T* p) {
#if HB_NT
  return __builtin_nontemporal_load(p);
#else
  return *p;
#endif
}

template <class T>
__device__ __forceinline__ void st_stream(T* p, T v) {
#if HB_NT
  __builtin_nontemporal_store(v, p);
#else
  *p = v;
#endif
}

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ uint4 ld_stream(const uint4* p) {
#if HB_NT
  const u32x4 v = __builtin_nontemporal_load(reinterpret_cast<const u32x4*>(p));
  return make_uint4(v.x, v.y, v.z, v.w);
#else
  return *p;
#endif
}

__device__ __forceinline__ void st_stream(uint4* p, uint4 v) {
#if HB_NT
  u32x4 x;
  x.x = v.x;
  x.y = v.y;
  x.z = v.z;
  x.w = v.w;
  __builtin_nontemporal_store(x, reinterpret_cast<u32x4*>(p));
#else
  *p = v;
#endif
}

// Node hash: SplitMix64 finalizer (Steele, Lea, Flood 2014) of
// v + (seed+1) * golden-ratio increment.  The paper asks only for a fixed
// hash (Sec. 4.1); this is the library's convention.
__device__ __forceinline__ uint64_t node_hash(uint64_t v, uint64_t seed) {
  uint64_t z = v + (seed + 1ull) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Byte-wise maximum of four packed registers.  Even and odd bytes are
// maximised separately in 16-bit lanes (packed u16 max), where no byte can
// carry into its neighbour, then recombined.
typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));

__device__ __forceinline__ uint32_t bmax4(uint32_t a, uint32_t b) {
  const u16x2 ae = __builtin_bit_cast(u16x2, a & 0x00FF00FFu);
  const u16x2 be = __builtin_bit_cast(u16x2, b & 0x00FF00FFu);
  const u16x2 ao = __builtin_bit_cast(u16x2, a & 0xFF00FF00u);
  const u16x2 bo = __builtin_bit_cast(u16x2, b & 0xFF00FF00u);
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(ae, be)) |
         __builtin_bit_cast(uint32_t, __builtin_elementwise_max(ao, bo));
}

__device__ __forceinline__ uint4 bmax(uint4 a, uint4 b) {
  a.x = bmax4(a.x, b.x);
  a.y = bmax4(a.y, b.y);
  a.z = bmax4(a.z, b.z);
  a.w = bmax4(a.w, b.w);
  return a;
}

// Gather accumulator in two sets of 16-bit lanes: e holds the even bytes
// (masked into the low half of each lane), o the raw dwords.  A 16-bit
// maximum orders lanes by their high byte first, so the high bytes of o are
// the maxima of the odd bytes whatever the low bytes were; folding in one
// dword costs one mask and two packed maxima.
struct SplitAcc {
  uint4 e;
  uint4 o;
};

__device__ __forceinline__ uint32_t pkmax(uint32_t a, uint32_t b) {
  return __builtin_bit_cast(uint32_t, __builtin_elementwise_max(__builtin_bit_cast(u16x2, a),
                                                                __builtin_bit_cast(u16x2, b)));
}

__device__ __forceinline__ void fold(SplitAcc& acc, uint4 x) {
  acc.e.x = pkmax(acc.e.x, x.x & 0x00FF00FFu);
  acc.o.x = pkmax(acc.o.x, x.x);
  acc.e.y = pkmax(acc.e.y, x.y & 0x00FF00FFu);
  acc.o.y = pkmax(acc.o.y, x.y);
  acc.e.z = pkmax(acc.e.z, x.z & 0x00FF00FFu);
  acc.o.z = pkmax(acc.o.z, x.z);
  acc.e.w = pkmax(acc.e.w, x.w & 0x00FF00FFu);
  acc.o.w = pkmax(acc.o.w, x.w);
}

__device__ __forceinline__ uint4 unsplit(const SplitAcc& acc) {
  constexpr uint32_t ODD = 0xFF00FF00u;
  return make_uint4(acc.e.x | (acc.o.x & ODD), acc.e.y | (acc.o.y & ODD), acc.e.z | (acc.o.z & ODD),
                    acc.e.w | (acc.o.w & ODD));
}

__device__ __forceinline__ bool differs(uint4 a, uint4 b) {
  return ((a.x ^ b.x) | (a.y ^ b.y) | (a.z ^ b.z) | (a.w ^ b.w)) != 0u;
}

__device__ __forceinline__ uint4 shfl_xor4(uint4 v, int m) {
  v.x = __shfl_xor(v.x, m);
  v.y = __shfl_xor(v.y, m);
  v.z = __shfl_xor(v.z, m);
  v.w = __shfl_xor(v.w, m);
  return v;
}

__device__ __forceinline__ uint4 zero4() { return make_uint4(0u, 0u, 0u, 0u); }

// 2^-r as a double, built from its exponent field (r <= 61 here).
__device__ __forceinline__ double pow2neg(uint32_t r) {
  return __hiloint2double((int)(0x3FF00000u - (r << 20)), 0);
}

// Exact pieces of sum_j 2^-M[j] over the 16 registers in v.  Terms with
// M[j] <= 26 go to `big`, the others to `small`: any sum of up to 2^16 terms
// of either kind is a multiple of a fixed power of two below 2^53 ulps, so
// both partial sums (and sums of them across lanes) are exact in double, and
// big + small rounds the exact total once.  `zeros` counts empty registers.
struct Parts {
  double big;
  double small;
  int zeros;
};

__device__ __forceinline__ Parts reg_parts(uint4 v) {
  const uint32_t w[4] = {v.x, v.y, v.z, v.w};
  uint32_t high = 0;
  int zeros = 0;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    high |= (w[i] + 0x65656565u) & 0x80808080u;  // some byte >= 27 (bytes are <= 61)
    const uint32_t t = ((w[i] & 0x7F7F7F7Fu) + 0x7F7F7F7Fu) | w[i];
    zeros += __popc(~t & 0x80808080u);          // bytes equal to 0
  }
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0, sm = 0.0;
  if (high == 0u) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      a0 += pow2neg(w[i] & 0xFFu);
      a1 += pow2neg((w[i] >> 8) & 0xFFu);
      a2 += pow2neg((w[i] >> 16) & 0xFFu);
      a3 += pow2neg(w[i] >> 24);
    }
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int k = 0; k < 4; ++k) {
        const uint32_t r = (w[i] >> (8 * k)) & 0xFFu;
        const double t = pow2neg(r);
        const bool lo = r <= 26u;
        a0 += lo ? t : 0.0;
        sm += lo ? 0.0 : t;
      }
  }
  Parts out;
  out.big = (a0 + a1) + (a2 + a3);
  out.small = sm;
  out.zeros = zeros;
  return out;
}

// Algorithm 1 `size` with the small-range (linear counting) estimator:
// alpha_p p^2 / Z, or p ln(p/V) (tabulated in lc) when that is <= 5p/2 and
// V > 0 registers are empty.
__device__ __forceinline__ double estimate(double big, double small, int V, double alpha_pp,
                                           double p, const double* lc) {
  const double z = big + small;
  double E = alpha_pp / z;
  if (E <= 2.5 * p && V > 0) E = lc[V];
  return E;
}

__device__ __forceinline__ bool bit_of(const uint64_t* bm, int64_t v) {
  return ((bm[v >> 6] >> (v & 63)) & 1ull) != 0ull;
}

// Per-wavefront work counters (summed over lanes before the atomics).
struct Counts {
  uint32_t gath, load, write, chg, arcs, slices, sch, pairs;
  uint32_t seeds;  // ensembles: OR of the seeds whose counter changed
};

// own_mod: the row's counter changed in the previous pass (so the next buffer
// holds a stale copy).  need: the row takes part in this pass.  In a sparse
// pass a row without a changed successor cannot change; it only runs to
// refresh a stale copy.  Rows of converged graphs never run.
template <bool MG>
__device__ __forceinline__ void row_flags(const PassArgs& A, int64_t row, bool& own_mod, bool& need) {
  own_mod = A.mode != MODE_FIRST && bit_of(A.mod_prev, row);
  need = A.mode != MODE_SPARSE || own_mod || A.act == nullptr || A.act[row] == A.epoch;
  if constexpr (MG) {
    if (A.graphs[A.blk_graph[row >> 6]].done) need = false;
  }
}

// Distance weight of this pass for a row: t+1, counted from the pass at which
// the row's graph started.
template <bool MG>
__device__ __forceinline__ double row_d(const PassArgs& A, int64_t row) {
  if constexpr (MG) return (double)(A.epoch - A.graphs[A.blk_graph[row >> 6]].t0);
  return A.d;
}

// With device pass control, the pass's buffers and mode come from ctl.
__device__ __forceinline__ PassArgs resolve(const PassArgs& A) {
  if (!A.ctl) return A;
  PassArgs L = A;
  const int par = A.ctl->parity;
  const int t = A.ctl->t;
  L.cur = A.cntb[par];
  L.nxt = A.cntb[par ^ 1];
  L.mod_prev = A.modb[par];
  L.mod_cur = A.modb[par ^ 1];
  L.mode = A.ctl->mode;
  L.epoch = t + 1;
  L.d = (double)(t + 1);
  L.act = (L.mode == MODE_SPARSE) ? A.act : nullptr;
  L.stats = A.stats_base + (size_t)(t & 1) * STAT_SLOTS * STAT_K;
  L.stats_next = A.stats_base + (size_t)((t + 1) & 1) * STAT_SLOTS * STAT_K;
  return L;
}

// Direct gather-max (dense passes) over the arcs k, k+st, k+2st, ... < e of
// a row: every lane of the group loads its 16-byte slice of each successor
// counter, U successors in flight.
//
// For p >= 64, slots past the end (and, with NEG, negative ids, which mark
// no successor) load the row's own counter instead: the row's result is the
// maximum with its own counter anyway, so the extra operand changes nothing;
// every load is unconditional (no zeroing, no exec masking), offsets are 32
// bits, and without NEG the number of gathered successors is known from the
// range, so the loop keeps no tally (R-MAT s24 dense pass 5.83 -> 5.45 ms).
// For p <= 32 rows are short relative to a round of U slots and the padding
// loads cost more than they save (4096-graph batch: 2 % slower), so slots
// past the end are zeroed and their loads skipped.
template <int B, bool NEG = false>
__device__ __forceinline__ uint4 gather(const PassArgs& A, int64_t k, int64_t e, int64_t st, int gl, int64_t own,
                                        bool& got, Counts& c) {
  constexpr int P = 1 << B;
  SplitAcc acc{zero4(), zero4()};
  const uint8_t* base = A.cur + gl * 16;
  if constexpr (B <= 5) {
    (void)own;
    for (; k < e; k += st * U) {
      int32_t w[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t kk = k + u * st;
        w[u] = kk < e ? ld_stream(A.idx + kk) : -1;
      }
      uint4 v[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        v[u] = zero4();
        if (w[u] >= 0) v[u] = *reinterpret_cast<const uint4*>(base + (size_t)w[u] * P);
      }
#pragma unroll
      for (int u = 0; u < U; ++u) {
        fold(acc, v[u]);
        const uint32_t hit = w[u] >= 0 ? 1u : 0u;
        got |= hit != 0u;
        c.slices += hit;
        if (gl == 0) c.gath += hit;
      }
    }
    return unsplit(acc);
  }
  const uint32_t own32 = (uint32_t)own;  // node ids fit 31 bits
  const int32_t st32 = (int32_t)st;
  if constexpr (!NEG) {
    const uint32_t n = k < e ? (uint32_t)((e - k + st - 1) / st) : 0u;
    got |= n > 0u;
    c.slices += n;
    if (gl == 0) c.gath += n;
  }
  for (; k < e; k += st * U) {
    // offsets from k in 32 bits: a row's or a chunk's arcs number < 2^31
    const int32_t rem = (int32_t)(e - 1 - k);
    int32_t w[U];
    bool ok[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int32_t d = u * st32;
      ok[u] = d <= rem;
      w[u] = ld_stream(A.idx + k + (d < rem ? d : rem));
    }
    uint4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      if constexpr (NEG) ok[u] = ok[u] && w[u] >= 0;
      const uint32_t src = ok[u] ? (uint32_t)w[u] : own32;
      v[u] = *reinterpret_cast<const uint4*>(base + (size_t)src * P);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      fold(acc, v[u]);
      if constexpr (NEG) {
        const uint32_t hit = ok[u] ? 1u : 0u;
        got |= hit != 0u;
        c.slices += hit;
        if (gl == 0) c.gath += hit;
      }
    }
  }
  return unsplit(acc);
}

// Queued gather (slice, sparse and optionally dense passes), in two phases:
// (1) a team of lanes reads successor ids and their change masks with
// consecutive lanes on consecutive arcs, and appends every successor with a
// nonzero mask to a queue in LDS; (2) lane groups drain the queue, each lane
// loading its 16-byte slice of a queued counter only if that slice changed.
struct QEnt {
  int32_t w;
  uint32_t msk;
};

constexpr int QCAP = 64 * U;  // queue entries per wavefront

template <int B>
__device__ __forceinline__ uint32_t change_mask(const PassArgs& A, int32_t w) {
  constexpr uint32_t FULL = (1u << ((1 << B) / 16)) - 1u;
  if (w < 0) return 0u;
  if (A.mode == MODE_FIRST || A.mode == MODE_DENSE) return FULL;
  // The change bitmap (n/8 bytes) stays in L2; the slice masks (2n bytes) are
  // read only for successors that changed.
  if (!bit_of(A.mod_prev, w)) return 0u;
  return A.mode == MODE_SLICE ? (uint32_t)A.dmask_prev[w] : FULL;
}

// Phase 1 for a team of TL lanes (a lane group or the wavefront): arcs
// k + tid + u*TL for u < U.  Returns the number of queued successors.
template <int B, int TL>
__device__ __forceinline__ int scan_chunk(const PassArgs& A, QEnt* q, int64_t k, int64_t e, int tid,
                                          uint64_t team, uint64_t below) {
  int32_t w[U];
  uint32_t m[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t kk = k + tid + (int64_t)u * TL;
    w[u] = kk < e ? ld_stream(A.idx + kk) : -1;
  }
#pragma unroll
  for (int u = 0; u < U; ++u) m[u] = change_mask<B>(A, w[u]);
  int nh = 0;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const bool hit = m[u] != 0u;
    const uint64_t hb = __ballot(hit) & team;
    if (hit) {
      QEnt ent;
      ent.w = w[u];
      ent.msk = m[u];
      q[nh + __popcll(hb & below)] = ent;
    }
    nh += __popcll(hb);
  }
  return nh;
}

// Phase 2: entries first, first+step, ... < nh of the queue, U in flight.
// As in the direct gather, slots past the queue's end and slices the entry
// does not need load the row's own counter (own) instead, unconditionally.
template <int B>
__device__ __forceinline__ void drain(const PassArgs& A, const QEnt* q, int first, int nh, int step, int gl,
                                      uint32_t own, SplitAcc& acc, Counts& c) {
  constexpr int P = 1 << B;
  const uint8_t* base = A.cur + gl * 16;
  for (int i = first; i < nh; i += step * U) {
    uint4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int j = i + u * step;
      const bool in = j < nh;
      const QEnt ent = q[in ? j : i];
      const bool hit = in && ((ent.msk >> gl) & 1u) != 0u;
      c.slices += hit ? 1u : 0u;
      v[u] = *reinterpret_cast<const uint4*>(base + (size_t)(hit ? (uint32_t)ent.w : own) * P);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) fold(acc, v[u]);
  }
}

// Queued gather of one row's arcs [s, e) by one lane group (light rows).
template <int B>
__device__ __forceinline__ uint4 gather_group_q(const PassArgs& A, QEnt* q, int64_t s, int64_t e, int gl,
                                                uint64_t gmask, uint64_t below, int64_t own, bool& got, Counts& c) {
  constexpr int G = (1 << B) / 16;
  SplitAcc acc{zero4(), zero4()};
  for (int64_t k = s; k < e; k += (int64_t)G * U) {
    const int nh = scan_chunk<B, G>(A, q, k, e, gl, gmask, below);
    __builtin_amdgcn_wave_barrier();
    if (gl == 0) c.gath += (uint32_t)nh;
    got |= nh > 0;
    drain<B>(A, q, 0, nh, 1, gl, (uint32_t)own, acc, c);
    __builtin_amdgcn_wave_barrier();
  }
  return unsplit(acc);
}

// Queued gather of arcs [s, e) by a whole wavefront; group grp drains
// entries grp, grp+W, ...  Returns the group's partial maximum.
template <int B>
__device__ __forceinline__ uint4 gather_wave_q(const PassArgs& A, QEnt* q, int64_t s, int64_t e, int lane,
                                               int gl, int grp, uint64_t below, int64_t own, bool& got, Counts& c) {
  constexpr int G = (1 << B) / 16;
  constexpr int W = 64 / G;
  SplitAcc acc{zero4(), zero4()};
  for (int64_t k = s; k < e; k += 64 * U) {
    const int nh = scan_chunk<B, 64>(A, q, k, e, lane, ~0ull, below);
    __builtin_amdgcn_wave_barrier();
    if (lane == 0) c.gath += (uint32_t)nh;
    got |= nh > 0;
    drain<B>(A, q, grp, nh, W, gl, (uint32_t)own, acc, c);
    __builtin_amdgcn_wave_barrier();
  }
  return unsplit(acc);
}

// What a row needs besides its successors, loaded before the gather so the
// loads overlap: the lane's slice of the own counter and, in the group's
// first lane, the cached estimate and the two accumulators.
struct RowPre {
  uint4 own;
  double e, s, h;
  double dd;  // discounted sum (FL_DISC)
};

template <int B, int FL = FL_PLAIN>
__device__ __forceinline__ RowPre preload(const PassArgs& A, int64_t row, int gl) {
  constexpr int P = 1 << B;
  constexpr int G = P / 16;
  RowPre r;
  r.own = ld_stream(reinterpret_cast<const uint4*>(A.cur + (size_t)row * P + (size_t)gl * 16));
  r.e = r.s = r.h = r.dd = 0.0;
  if constexpr (FL == FL_ENS) {
    // first lane of each seed's counter: its cached estimate and accumulators
    const int gs = A.seg_lanes;
    if ((gl & (gs - 1)) == 0) {
      const int64_t i = row * (G / gs) + gl / gs;
      r.e = ld_stream(A.E + i);
      r.s = ld_stream(A.S + i);
      r.h = ld_stream(A.H + i);
    }
  } else if (gl == 0) {
    r.e = ld_stream(A.E + row);
    r.s = ld_stream(A.S + row);
    r.h = ld_stream(A.H + row);
    if constexpr (FL == FL_DISC) r.dd = ld_stream(A.D + row);
  }
  return r;
}

// Completes row `row` for a group of G lanes: a = own U gathered, write-back
// rule, change detection, the fused estimator/accumulator, the change bit
// and the mask of changed slices (with DEFER the caller sets the change bit,
// see set_change_bits).  In an ensemble row (FL_ENS) every seed's
// counter gets its own estimator and accumulators, and the row's change bit
// is set if any of them changed; FL_DISC also accumulates the discounted sum
// D += f(t+1) * delta.  Returns whether the row changed.
template <int B, bool MG, int FL = FL_PLAIN, bool DEFER = false>
__device__ __forceinline__ bool finish_row(const PassArgs& A, int64_t row, uint4 acc, bool got,
                                           const RowPre& pre, bool own_mod, int gl, int grp,
                                           Counts& c) {
  constexpr int P = 1 << B;
  constexpr int G = P / 16;
  const size_t off = (size_t)row * P + (size_t)gl * 16;
  const uint4 a = got ? bmax(acc, pre.own) : pre.own;
  const bool diff = got && differs(a, pre.own);
  const uint64_t bal = __ballot(diff);
  const uint32_t msk = (uint32_t)((bal >> (grp * G)) & ((1ull << G) - 1ull));
  const bool changed = msk != 0u;
  if (changed || own_mod) st_stream(reinterpret_cast<uint4*>(A.nxt + off), a);
  if (gl == 0) {
    c.load += 1u;
    c.write += (changed || own_mod) ? 1u : 0u;
    c.chg += changed ? 1u : 0u;
    c.sch += (uint32_t)__popc(msk);
    if (changed && A.roff) c.pairs += (uint32_t)(A.roff[row + 1] - A.roff[row]);
  }
  if constexpr (FL == FL_ENS) {
    const int gs = A.seg_lanes;  // lanes per seed's counter
    const int seg = gl / gs;
    if (gl == 0 && changed)
      for (int k = 0; k < G / gs; ++k)
        if ((msk >> (k * gs)) & ((1u << gs) - 1u)) c.seeds |= 1u << k;
    if ((msk >> (seg * gs)) & ((1u << gs) - 1u)) {  // uniform over the lanes of one counter
      const Parts pr = reg_parts(a);
      double big = pr.big, small = pr.small;
      int V = pr.zeros;
#pragma unroll
      for (int o = 1; o < G; o <<= 1) {
        if (o < gs) {
          big += __shfl_xor(big, o);
          small += __shfl_xor(small, o);
          V += __shfl_xor(V, o);
        }
      }
      if ((gl & (gs - 1)) == 0) {
        const double En = estimate(big, small, V, A.alpha_pp, (double)(16 * gs), A.lc);
        const double delta = En - pre.e;
        const double d = row_d<MG>(A, row);
        const int64_t i = row * (G / gs) + seg;
        st_stream(A.S + i, pre.s + d * delta);
        st_stream(A.H + i, pre.h + delta / d);
        st_stream(A.E + i, En);
      }
    }
    if (changed && gl == 0) {
      if (A.dmask_cur) A.dmask_cur[row] = (uint16_t)msk;
      if (!DEFER) atomicOr(A.mod_cur + (row >> 6), 1ull << (row & 63));
    }
  } else if (changed) {
    const Parts pr = reg_parts(a);
    double big = pr.big, small = pr.small;
    int V = pr.zeros;
#pragma unroll
    for (int o = 1; o < G; o <<= 1) {
      big += __shfl_xor(big, o);
      small += __shfl_xor(small, o);
      V += __shfl_xor(V, o);
    }
    if (gl == 0) {
      const double En = estimate(big, small, V, A.alpha_pp, (double)P, A.lc);
      const double delta = En - pre.e;
      const double d = row_d<MG>(A, row);
      st_stream(A.S + row, pre.s + d * delta);
      st_stream(A.H + row, pre.h + delta / d);
      if constexpr (FL == FL_DISC) st_stream(A.D + row, pre.dd + A.disc_f * delta);
      st_stream(A.E + row, En);
      if (A.dmask_cur) A.dmask_cur[row] = (uint16_t)msk;
      if (!DEFER) atomicOr(A.mod_cur + (row >> 6), 1ull << (row & 63));
    }
  }
  return changed;
}

template <int FL = FL_PLAIN>
__device__ __forceinline__ void add_stats(unsigned long long* st, const Counts& c) {
  const unsigned long long v[STAT_SEEDS] = {c.gath, c.load, c.write, c.chg, c.arcs, c.slices, c.sch, c.pairs};
#pragma unroll
  for (int k = 0; k < STAT_SEEDS; ++k)
    if (v[k]) atomicAdd(st + k, v[k]);
  if (FL == FL_ENS && c.seeds) atomicOr(st + STAT_SEEDS, (unsigned long long)c.seeds);
}

template <int FL = FL_PLAIN>
__device__ __forceinline__ void flush_counts(const PassArgs& A, Counts c, int64_t slot, int lane) {
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    c.gath += __shfl_xor(c.gath, o);
    c.load += __shfl_xor(c.load, o);
    c.write += __shfl_xor(c.write, o);
    c.chg += __shfl_xor(c.chg, o);
    c.arcs += __shfl_xor(c.arcs, o);
    c.slices += __shfl_xor(c.slices, o);
    c.sch += __shfl_xor(c.sch, o);
    c.pairs += __shfl_xor(c.pairs, o);
    if (FL == FL_ENS) c.seeds |= __shfl_xor(c.seeds, o);
  }
  if (lane == 0) add_stats<FL>(A.stats + (slot & (STAT_SLOTS - 1)) * STAT_K, c);
}

__device__ __forceinline__ uint64_t lanes_below(int lane) { return (1ull << lane) - 1ull; }

// Makes a wavefront's LDS writes visible to its other lanes.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Whether a row reads its own counter only after its gather found a changed
// successor: in the queued passes that gather changed successors only, for
// rows whose counter did not change in the previous pass (such a row with no
// changed successor cannot change and needs no write).
template <bool Q>
__device__ __forceinline__ bool lazy_row(const PassArgs& A, bool own_mod) {
  return Q && !own_mod && A.mode != MODE_FIRST && A.mode != MODE_DENSE;
}

// Sets the change bits of the rows whose leader lanes have `has` set, one
// device-scope atomic per distinct bitmap word instead of one per row (the
// rows of a light-row round are consecutive list entries, mostly in one or
// two words).  Must be called by the whole wavefront.
__device__ __forceinline__ void set_change_bits(uint64_t* mod_cur, int64_t row, bool has, int lane) {
  uint64_t pending = __ballot(has);
  const int64_t word = row >> 6;
  const uint64_t bit = 1ull << (row & 63);
  while (pending) {
    const int first = __ffsll((long long)pending) - 1;
    const int64_t w0 = __shfl(word, first);
    const bool mine = has && word == w0;
    uint32_t lo = mine ? (uint32_t)bit : 0u;
    uint32_t hi = mine ? (uint32_t)(bit >> 32) : 0u;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
      lo |= __shfl_xor(lo, o);
      hi |= __shfl_xor(hi, o);
    }
    if (lane == first) atomicOr(mod_cur + w0, ((uint64_t)hi << 32) | lo);
    pending &= ~__ballot(mine);
  }
}

// Light rows taken 64 to a wavefront (first and dense passes of every context,
// edge passes of single graphs) finish in two steps.  Per round, the row's
// lane group does what is per register: the write-back rule, change
// detection and the register sum (finish_group), and leaves a RowSum in LDS;
// after the rounds every lane finishes its own row, all 64 at once: the
// estimator, the accumulators, the slice mask, the change bit and the counts
// (finish_lane).  Same values in the same order as finish_row, with the
// per-row work run once per wavefront instead of once per round by the
// groups' leader lanes.
struct RowSum {
  double big, small;
  int32_t zeros;
  uint32_t msk;  // changed slices; 0: the row did not change
};

template <int B>
__device__ __forceinline__ void finish_group(const PassArgs& A, int64_t row, uint4 acc, bool got, uint4 own,
                                             bool own_mod, int gl, int grp, RowSum* slot) {
  constexpr int P = 1 << B;
  constexpr int G = P / 16;
  const uint4 a = got ? bmax(acc, own) : own;
  const bool diff = got && differs(a, own);
  const uint64_t bal = __ballot(diff);
  const uint32_t msk = (uint32_t)((bal >> (grp * G)) & ((1ull << G) - 1ull));
  if (msk != 0u || own_mod) st_stream(reinterpret_cast<uint4*>(A.nxt + (size_t)row * P + (size_t)gl * 16), a);
  RowSum out{0.0, 0.0, 0, msk};
  if (msk != 0u) {  // uniform over the group
    const Parts pr = reg_parts(a);
    double big = pr.big, small = pr.small;
    int V = pr.zeros;
#pragma unroll
    for (int o = 1; o < G; o <<= 1) {
      big += __shfl_xor(big, o);
      small += __shfl_xor(small, o);
      V += __shfl_xor(V, o);
    }
    out.big = big;
    out.small = small;
    out.zeros = V;
  }
  if (gl == 0) *slot = out;
}

// The row's own lane, after the rounds: `done` if its group finished the row
// (e0, s0, h0 = its E, S, H as before the pass).  Must be called by the whole
// wavefront (the change bits are combined per bitmap word).
template <int B, bool MG = false>
__device__ __forceinline__ void finish_lane(const PassArgs& A, int64_t row, bool done, bool own_mod,
                                            const RowSum* sums, int lane, double e0, double s0, double h0,
                                            Counts& c) {
  constexpr int P = 1 << B;
  bool chg = false;
  if (done) {
    const RowSum rs = sums[lane];
    chg = rs.msk != 0u;
    c.load += 1u;
    c.write += (chg || own_mod) ? 1u : 0u;
    if (chg) {
      c.chg += 1u;
      c.sch += (uint32_t)__popc(rs.msk);
      if (A.roff) c.pairs += (uint32_t)(A.roff[row + 1] - A.roff[row]);
      const double En = estimate(rs.big, rs.small, rs.zeros, A.alpha_pp, (double)P, A.lc);
      const double delta = En - e0;
      const double d = row_d<MG>(A, row);
      st_stream(A.S + row, s0 + d * delta);
      st_stream(A.H + row, h0 + delta / d);
      st_stream(A.E + row, En);
      if (A.dmask_cur) A.dmask_cur[row] = (uint16_t)rs.msk;
    }
  }
  set_change_bits(A.mod_cur, row, chg, lane);
}

// Light rows of a single-graph pass that gathers only changed successors,
// scanned wave-wide before any gather: the wavefront's lanes take the
// successor ids of all its 64 rows as one run of consecutive arcs (lane j of
// a round takes arc j; its row is found by a binary search over the rows'
// arc offsets held in the lanes), look up the change bits, and queue every
// changed successor with its row's slot, in arc order, so that each row's
// entries are contiguous.  Then each lane group finishes its rows in turn as
// in light_wave, issuing the row's own counter and accumulators together with
// its queued successors: one memory round trip per row instead of three
// (ids, then change bits, then counters).  Returns false, having written
// nothing but the queue, when the queue cannot hold all changed successors;
// the caller then runs the rows one by one.
template <int B>
__device__ __forceinline__ bool light_wave_scanned(const PassArgs& A, QEnt* qw, RowSum* sums, int64_t lw, int lane) {
  constexpr int P = 1 << B;
  constexpr int G = P / 16;
  constexpr int W = 64 / G;
  const int gl = lane % G;
  const int grp = lane / G;
  const int64_t i = lw * 64 + lane;
  int64_t row = 0, s = 0;
  int32_t deg = 0;
  bool own_mod = false, need = false;
  if (i < A.n_light) {
    row = A.light[i];
    s = A.off[row];
    deg = (int32_t)(A.off[row + 1] - s);
    row_flags<false>(A, row, own_mod, need);
  }
  const uint64_t needs = __ballot(need);
  const uint64_t mods = __ballot(own_mod);
  const int32_t dn = need ? deg : 0;
  int32_t incl = dn;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int32_t t = __shfl_up(incl, o);
    if (lane >= o) incl += t;
  }
  const int32_t base = incl - dn;  // first arc of this lane's row in the wave's run
  const int32_t total = __shfl(incl, 63);
  const uint64_t below = lanes_below(lane);
  int nq = 0;
  for (int32_t k0 = 0; k0 < total; k0 += 64 * U) {
    int32_t w[U];
    uint32_t m[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int32_t j = k0 + u * 64 + lane;
      // row slot of arc j: the last lane whose base is <= j
      int lo = 0, hi = 63;
#pragma unroll
      for (int step = 0; step < 6; ++step) {
        const int mid = (lo + hi + 1) >> 1;
        if (__shfl(base, mid) <= j) lo = mid; else hi = mid - 1;
      }
      const int64_t rs = __shfl(s, lo);
      const int32_t rb = __shfl(base, lo);
      w[u] = j < total ? ld_stream(A.idx + rs + (j - rb)) : -1;
      m[u] = (uint32_t)lo << 16;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t cm = change_mask<B>(A, w[u]);
      const bool hit = cm != 0u;
      const uint64_t hb = __ballot(hit);
      const int cnt = __popcll(hb);
      if (nq + cnt > QCAP) return false;  // uniform over the wavefront
      if (hit) {
        QEnt ent;
        ent.w = w[u];
        ent.msk = cm | m[u];
        qw[nq + __popcll(hb & below)] = ent;
      }
      nq += cnt;
    }
  }
  __builtin_amdgcn_wave_barrier();
  // Each lane's row: its entries are [qs, qe) (binary search over the
  // queue's row slots, which are nondecreasing).
  int qs = 0;
  {
    int lo = 0, hi = nq;
    while (lo < hi) {
      const int mid = (lo + hi) >> 1;
      if ((int)(qw[mid].msk >> 16) < lane) lo = mid + 1; else hi = mid;
    }
    qs = lo;
  }
  int qe = __shfl_down(qs, 1);
  if (lane == 63) qe = nq;
  // the lane's own row: finished by its group unless it keeps its counter
  const bool done = need && (qe > qs || own_mod);
  double e0 = 0.0, s0 = 0.0, h0 = 0.0;
  if (done) {
    e0 = ld_stream(A.E + row);
    s0 = ld_stream(A.S + row);
    h0 = ld_stream(A.H + row);
  }
  Counts c{};
  for (int r = 0; r < G; ++r) {
    const int rl = r * W + grp;
    // shuffles first, with every lane active (a lane of a group that skips
    // its row must still supply its values to the group that reads them)
    const int64_t rrow = __shfl(row, rl);
    const int32_t rd = __shfl(deg, rl);
    const int rqs = __shfl(qs, rl);
    const int rqe = __shfl(qe, rl);
    if (!((needs >> rl) & 1ull)) continue;  // uniform over the group
    const bool rmod = ((mods >> rl) & 1ull) != 0ull;
    const bool got = rqe > rqs;
    if (gl == 0) {
      c.arcs += (uint32_t)rd;
      c.gath += (uint32_t)(rqe - rqs);
    }
    // A row without a changed successor that did not change before keeps
    // its counter (lazy_row): nothing to read or write.
    if (!got && !rmod) continue;
    const uint4 own = ld_stream(reinterpret_cast<const uint4*>(A.cur + (size_t)rrow * P + (size_t)gl * 16));
    SplitAcc acc{zero4(), zero4()};
    drain<B>(A, qw, rqs, rqe, 1, gl, (uint32_t)rrow, acc, c);
    finish_group<B>(A, rrow, unsplit(acc), got, own, rmod, gl, grp, sums + rl);
  }
  wave_sync();
  finish_lane<B>(A, row, done, own_mod, sums, lane, e0, s0, h0, c);
  flush_counts(A, c, lw, lane);
  return true;
}

// Row slot (lane) of arc j of a wavefront's run of consecutive arcs, given
// each lane's first arc `base` (nondecreasing over the lanes): the last lane
// whose base is <= j.  Needs every lane active.
__device__ __forceinline__ int arc_slot(int32_t base, int32_t j) {
  int lo = 0, hi = 63;
#pragma unroll
  for (int step = 0; step < 6; ++step) {
    const int mid = (lo + hi + 1) >> 1;
    if (__shfl(base, mid) <= j) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// Direct gather of one row whose successor ids were staged in LDS
// (ids[k .. e)), p >= 64: as gather, slots past the end load the row's own
// counter.
template <int B>
__device__ __forceinline__ uint4 gather_staged(const PassArgs& A, const int32_t* ids, int k, int e, int gl,
                                               uint32_t own, bool& got, Counts& c) {
  constexpr int P = 1 << B;
  SplitAcc acc{zero4(), zero4()};
  const uint8_t* base = A.cur + gl * 16;
  const uint32_t n = k < e ? (uint32_t)(e - k) : 0u;
  got |= n > 0u;
  c.slices += n;
  if (gl == 0) c.gath += n;
  for (; k < e; k += U) {
    const int rem = e - 1 - k;
    int32_t w[U];
    bool ok[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      ok[u] = u <= rem;
      w[u] = ids[k + (u < rem ? u : rem)];
    }
    uint4 v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint32_t src = ok[u] ? (uint32_t)w[u] : own;
      v[u] = *reinterpret_cast<const uint4*>(base + (size_t)src * P);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) fold(acc, v[u]);
  }
  return unsplit(acc);
}

// Successor ids a wavefront stages in LDS in dense passes (the queue's bytes).
constexpr int ID_CAP = 2 * QCAP;

// Light rows of a single-graph pass that gathers every successor (p >= 64):
// the successor ids of all 64 rows are loaded wave-wide first (consecutive
// arcs on consecutive lanes, rows found by arc_slot) into LDS, then each lane
// group gathers its rows' successor counters with the ids taken from LDS,
// the row's own counter and accumulators issued with them: one memory round
// trip per row instead of two (ids, then counters).  Returns false, having
// written nothing but LDS, when the rows have more arcs than the buffer
// holds; the caller then runs the rows one by one.
template <int B>
__device__ __forceinline__ bool light_wave_staged(const PassArgs& A, int32_t* ids, RowSum* sums, int64_t lw,
                                                  int lane) {
  constexpr int P = 1 << B;
  constexpr int G = P / 16;
  constexpr int W = 64 / G;
  const int gl = lane % G;
  const int grp = lane / G;
  const int64_t i = lw * 64 + lane;
  int64_t row = 0, s = 0;
  int32_t deg = 0;
  bool own_mod = false, need = false;
  if (i < A.n_light) {
    row = A.light[i];
    s = A.off[row];
    deg = (int32_t)(A.off[row + 1] - s);
    row_flags<false>(A, row, own_mod, need);
  }
  const uint64_t needs = __ballot(need);
  const uint64_t mods = __ballot(own_mod);
  const int32_t dn = need ? deg : 0;
  int32_t incl = dn;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const int32_t t = __shfl_up(incl, o);
    if (lane >= o) incl += t;
  }
  const int32_t base = incl - dn;
  const int32_t total = __shfl(incl, 63);
  if (total > ID_CAP) return false;  // uniform over the wavefront
  double e0 = 0.0, s0 = 0.0, h0 = 0.0;
  if (need) {
    e0 = ld_stream(A.E + row);
    s0 = ld_stream(A.S + row);
    h0 = ld_stream(A.H + row);
  }
  for (int32_t k0 = 0; k0 < total; k0 += 64 * U) {
    int32_t w[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int32_t j = k0 + u * 64 + lane;
      const int lo = arc_slot(base, j);
      const int64_t rs = __shfl(s, lo);
      const int32_t rb = __shfl(base, lo);
      w[u] = j < total ? ld_stream(A.idx + rs + (j - rb)) : 0;
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int32_t j = k0 + u * 64 + lane;
      if (j < total) ids[j] = w[u];
    }
  }
  __builtin_amdgcn_wave_barrier();
  Counts c{};
  for (int r = 0; r < G; ++r) {
    const int rl = r * W + grp;
    const int64_t rrow = __shfl(row, rl);
    const int32_t rb = __shfl(base, rl);
    const int32_t rd = __shfl(deg, rl);
    if (((needs >> rl) & 1ull) != 0ull) {  // uniform over the group
      const bool rmod = ((mods >> rl) & 1ull) != 0ull;
      const uint4 own = ld_stream(reinterpret_cast<const uint4*>(A.cur + (size_t)rrow * P + (size_t)gl * 16));
      bool got = false;
      const uint4 acc = gather_staged<B>(A, ids, rb, rb + rd, gl, (uint32_t)rrow, got, c);
      if (gl == 0) c.arcs += (uint32_t)rd;
      finish_group<B>(A, rrow, acc, got, own, rmod, gl, grp, sums + rl);
    }
  }
  wave_sync();
  finish_lane<B>(A, row, need, own_mod, sums, lane, e0, s0, h0, c);
  flush_counts(A, c, lw, lane);
  return true;
}

// Light rows of a pass that gathers every successor (dense and first passes
// that read counters), single- or multi-graph: rows as in light_wave, the
// successor ids read by the groups, finished in two steps (finish_group,
// finish_lane) with each row's E, S, H loaded up front by its own lane.
template <int B, bool MG>
__device__ __forceinline__ void light_wave_direct(const PassArgs& A, RowSum* sums, int64_t lw, int lane) {
  constexpr int P = 1 << B;
  constexpr int G = P / 16;
  constexpr int W = 64 / G;
  const int gl = lane % G;
  const int grp = lane / G;
  const int64_t i = lw * 64 + lane;
  int64_t row = 0, s = 0, deg = 0;
  bool own_mod = false, need = false;
  double e0 = 0.0, s0 = 0.0, h0 = 0.0;
  if (i < A.n_light) {
    row = A.light[i];
    s = A.off[row];
    deg = A.off[row + 1] - s;
    row_flags<MG>(A, row, own_mod, need);
    if (need) {
      e0 = ld_stream(A.E + row);
      s0 = ld_stream(A.S + row);
      h0 = ld_stream(A.H + row);
    }
  }
  const uint64_t needs = __ballot(need);
  const uint64_t mods = __ballot(own_mod);
  Counts c{};
  if (!needs) return;  // uniform: nothing to count either
  for (int r = 0; r < G; ++r) {
    const int rl = r * W + grp;
    const int64_t rrow = __shfl(row, rl);
    const int64_t rs = __shfl(s, rl);
    const int64_t rd = __shfl(deg, rl);
    if ((needs >> rl) & 1ull) {  // uniform over the group
      const bool rmod = ((mods >> rl) & 1ull) != 0ull;
      const uint4 own = ld_stream(reinterpret_cast<const uint4*>(A.cur + (size_t)rrow * P + (size_t)gl * 16));
      bool got = false;
      const uint4 acc = gather<B>(A, rs, rs + rd, 1, gl, rrow, got, c);
      if (gl == 0) c.arcs += (uint32_t)rd;
      finish_group<B>(A, rrow, acc, got, own, rmod, gl, grp, sums + rl);
    }
  }
  wave_sync();
  finish_lane<B, MG>(A, row, need, own_mod, sums, lane, e0, s0, h0, c);
  flush_counts(A, c, lw, lane);
}

// 64 consecutive entries of the light-row list per wavefront; entry
// q*W + grp goes to lane group grp in round q.
template <int B, bool Q, bool MG, int FL = FL_PLAIN>
__device__ __forceinline__ void light_wave(const PassArgs& A, QEnt* qw, RowSum* sums, int64_t lw, int lane) {
  constexpr int P = 1 << B;
  constexpr int G = P / 16;
  constexpr int W = 64 / G;
  const int gl = lane % G;
  const int grp = lane / G;
  if constexpr (MG) {
    if (A.chunk_graph) {  // a chunk of one converged graph has nothing to do
      const int32_t g = A.chunk_graph[lw];
      if (g >= 0 && A.graphs[g].done) return;
    }
  }
  if constexpr (Q && !MG && FL == FL_PLAIN) {
    if (A.mode != MODE_FIRST && A.mode != MODE_DENSE && light_wave_scanned<B>(A, qw, sums, lw, lane)) return;
    __builtin_amdgcn_wave_barrier();
  }
  if constexpr (!Q && !MG && FL == FL_PLAIN && B >= 6) {
    if (qw && light_wave_staged<B>(A, reinterpret_cast<int32_t*>(qw), sums, lw, lane)) return;
    __builtin_amdgcn_wave_barrier();
  }
  if constexpr (!Q && FL == FL_PLAIN) {
    if (sums) {
      light_wave_direct<B, MG>(A, sums, lw, lane);
      return;
    }
  }
  const int64_t i = lw * 64 + lane;
  int64_t row = 0, s = 0, deg = 0;
  bool own_mod = false, need = false;
  if (i < A.n_light) {
    row = A.light[i];
    s = A.off[row];
    deg = A.off[row + 1] - s;
    row_flags<MG>(A, row, own_mod, need);
  }
  const uint64_t needs = __ballot(need);
  const uint64_t mods = __ballot(own_mod);
  const uint64_t gmask = (G >= 64) ? ~0ull : (((1ull << G) - 1ull) << (grp * G));
  QEnt* q = qw + grp * (G * U);
  Counts c{};
  if (needs) {
    for (int r = 0; r < G; ++r) {
      const int rl = r * W + grp;
      const int64_t rrow = __shfl(row, rl);
      const int64_t rs = __shfl(s, rl);
      const int64_t rd = __shfl(deg, rl);
      bool chg = false;
      if ((needs >> rl) & 1ull) {
        const bool rmod = ((mods >> rl) & 1ull) != 0ull;
        // In passes that gather only changed successors, a row that finds
        // none and did not change before is left as it is, so its own
        // counter and accumulators are read only once a changed successor
        // turned up (most rows of a sparse tail find none).
        const bool lazy = lazy_row<Q>(A, rmod);
        RowPre pre;
        if (!lazy) pre = preload<B, FL>(A, rrow, gl);
        bool got = false;
        uint4 acc;
        if constexpr (Q)
          acc = gather_group_q<B>(A, q, rs, rs + rd, gl, gmask, lanes_below(lane), rrow, got, c);
        else
          acc = gather<B>(A, rs, rs + rd, 1, gl, rrow, got, c);
        if (gl == 0) c.arcs += (uint32_t)rd;
        if (lazy && got) pre = preload<B, FL>(A, rrow, gl);
        // Multi-graph passes run many short rows per byte moved, so there the
        // change bits of a round are combined into one atomic per bitmap
        // word; single-graph kernels keep one atomic per row (fewer live
        // registers).
        if (!lazy || got) chg = finish_row<B, MG, FL, MG>(A, rrow, acc, got, pre, rmod, gl, grp, c);
      }
      if constexpr (MG) set_change_bits(A.mod_cur, rrow, chg && gl == 0, lane);
    }
  }
  flush_counts<FL>(A, c, lw, lane);
}

// Medium rows per wavefront where their finish is batched (first passes, and
// the queued passes of plain single-graph contexts): one per lane group, at
// most 8.
__host__ __device__ constexpr int batched_med_rows(int B) { return (1024 >> B) < 8 ? (1024 >> B) : 8; }

template <int B, bool Q, bool MG, int FL>
__host__ __device__ constexpr int med_rows_per_wave() {
  return Q && !MG && FL == FL_PLAIN ? batched_med_rows(B) : 1;
}

// Medium rows of a plain single-graph queued pass, R to a wavefront: the
// whole wavefront gathers each row's changed successors in turn (as
// medium_wave does), lane group r keeps row r's maximum, and the R rows are
// finished together in two steps (finish_group, finish_lane).  The rows' list
// entries and offsets are loaded once for all R rows, and their own counters
// and accumulators after all the gathers, in one round trip.
template <int B>
__device__ __forceinline__ void medium_rows_q(const PassArgs& A, QEnt* qw, RowSum* sums, int64_t mw, int lane) {
  constexpr int P = 1 << B;
  constexpr int G = P / 16;
  constexpr int R = batched_med_rows(B);
  const int gl = lane % G;
  const int grp = lane / G;
  const int64_t i = mw * R + lane;
  int64_t row = 0, s = 0, deg = 0;
  bool own_mod = false, need = false;
  if (lane < R && i < A.n_medium) {
    row = A.medium[i];
    s = A.off[row];
    deg = A.off[row + 1] - s;
    row_flags<false>(A, row, own_mod, need);
  }
  const uint64_t live = __ballot(need);
  Counts c{};
  uint4 mine = zero4();
  bool mine_got = false;
#pragma unroll 1
  for (int r = 0; r < R; ++r) {
    if (((live >> r) & 1ull) == 0ull) continue;  // uniform
    const int64_t rrow = __shfl(row, r);
    const int64_t rs = __shfl(s, r);
    const int64_t rd = __shfl(deg, r);
    bool got = false;
    uint4 acc = gather_wave_q<B>(A, qw, rs, rs + rd, lane, gl, grp, lanes_below(lane), rrow, got, c);
    if (lane == 0) c.arcs += (uint32_t)rd;
#pragma unroll
    for (int o = G; o < 64; o <<= 1) acc = bmax(acc, shfl_xor4(acc, o));
    got = __ballot(got) != 0ull;
    if (grp == r) {
      mine = acc;
      mine_got = got;
    }
  }
  // As in medium_wave, a lazy row (see light_wave) that found no changed
  // successor is left as it is.
  const bool got_r = __shfl((int)mine_got, (lane % R) * G) != 0;
  const bool done = need && (!lazy_row<true>(A, own_mod) || got_r);
  double e0 = 0.0, s0 = 0.0, h0 = 0.0;
  if (done) {
    e0 = ld_stream(A.E + row);
    s0 = ld_stream(A.S + row);
    h0 = ld_stream(A.H + row);
  }
  const int64_t grow = __shfl(row, grp % R);
  const bool gmod = __shfl((int)own_mod, grp % R) != 0;
  const bool gdone = __shfl((int)done, grp % R) != 0 && grp < R;
  if (gdone) {
    const uint4 own = ld_stream(reinterpret_cast<const uint4*>(A.cur + (size_t)grow * P + (size_t)gl * 16));
    finish_group<B>(A, grow, mine, mine_got, own, gmod, gl, grp, sums + grp);
  }
  wave_sync();
  finish_lane<B, false>(A, row, done, own_mod, sums, lane, e0, s0, h0, c);
  flush_counts(A, c, mw, lane);
}

// One medium row per wavefront: the groups share its arcs and reduce their
// partial maxima by shuffles.
template <int B, bool Q, bool MG, int FL = FL_PLAIN>
__device__ __forceinline__ void medium_wave(const PassArgs& A, QEnt* qw, int64_t mi, int lane) {
  constexpr int P = 1 << B;
  constexpr int G = P / 16;
  constexpr int W = 64 / G;
  const int gl = lane % G;
  const int grp = lane / G;
  const int64_t row = A.medium[mi];
  const int64_t s = A.off[row];
  const int64_t deg = A.off[row + 1] - s;
  bool own_mod, need;
  row_flags<MG>(A, row, own_mod, need);
  Counts c{};
  if (need) {
    const bool lazy = lazy_row<Q>(A, own_mod);  // as in light_wave
    RowPre pre;
    if (grp == 0 && !lazy) pre = preload<B, FL>(A, row, gl);
    bool got = false;
    uint4 acc;
    if constexpr (Q)
      acc = gather_wave_q<B>(A, qw, s, s + deg, lane, gl, grp, lanes_below(lane), row, got, c);
    else
      acc = gather<B>(A, s + grp, s + deg, W, gl, row, got, c);
    if (lane == 0) c.arcs += (uint32_t)deg;
#pragma unroll
    for (int o = G; o < 64; o <<= 1) acc = bmax(acc, shfl_xor4(acc, o));
    got = __ballot(got) != 0ull;
    if (grp == 0 && lazy && got) pre = preload<B, FL>(A, row, gl);
    if (grp == 0 && (!lazy || got)) finish_row<B, MG, FL>(A, row, acc, got, pre, own_mod, gl, 0, c);
  }
  flush_counts<FL>(A, c, mi, lane);
}

// One chunk of a heavy row per workgroup (4 wavefronts): writes the chunk's
// partial maximum for the merge kernel.
template <int B, bool Q, bool MG>
__device__ __forceinline__ void heavy_chunk(const PassArgs& A, QEnt* qw, int64_t item, int lane, int wave) {
  constexpr int P = 1 << B;
  constexpr int G = P / 16;
  constexpr int W = 64 / G;
  __shared__ uint4 red[4][16];
  const int gl = lane % G;
  const int grp = lane / G;
  const HeavyItem it = A.items[item];
  bool own_mod, need;
  row_flags<MG>(A, it.row, own_mod, need);
  if (!need) return;  // uniform over the workgroup; the merge kernel skips the row too
  bool got = false;
  Counts c{};
  uint4 acc;
  if constexpr (Q) {
    const int64_t quarter = (it.e1 - it.e0 + 3) / 4;
    const int64_t a0 = it.e0 + wave * quarter;
    const int64_t a1 = a0 + quarter < it.e1 ? a0 + quarter : it.e1;
    acc = gather_wave_q<B>(A, qw, a0, a1, lane, gl, grp, lanes_below(lane), it.row, got, c);
  } else {
    acc = gather<B>(A, it.e0 + wave * W + grp, it.e1, 4 * W, gl, it.row, got, c);
  }
  if (lane == 0 && wave == 0) c.arcs += (uint32_t)(it.e1 - it.e0);
#pragma unroll
  for (int o = G; o < 64; o <<= 1) acc = bmax(acc, shfl_xor4(acc, o));
  if (grp == 0) red[wave][gl] = acc;
  flush_counts(A, c, item, lane);
  __syncthreads();
  if (wave == 0 && grp == 0) {
    uint4 a = red[0][gl];
    a = bmax(a, red[1][gl]);
    a = bmax(a, red[2][gl]);
    a = bmax(a, red[3][gl]);
    *reinterpret_cast<uint4*>(A.partial + (size_t)item * P + (size_t)gl * 16) = a;
  }
}

// Work items of a pass, one per workgroup: [heavy chunks][medium rows, 4 R
// per workgroup (R = med_rows_per_wave)][light rows, 256 per workgroup].  Q
// selects the queued gather (slice, edge and sparse passes, or dense passes
// on request) over the direct one.
template <int B, bool Q, bool MG, int FL = FL_PLAIN>
__device__ __forceinline__ void expand_item(const PassArgs& A, QEnt* qw, RowSum* sums, int64_t b) {
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  if (b == 0)
    for (int i = threadIdx.x; i < STAT_SLOTS * STAT_K; i += blockDim.x) A.stats_next[i] = 0ull;
  if (b < A.n_items) {
    heavy_chunk<B, Q, MG>(A, qw, b, lane, wave);
    return;
  }
  b -= A.n_items;
  constexpr int R = med_rows_per_wave<B, Q, MG, FL>();
  const int64_t med_wgs = (A.n_medium + 4 * R - 1) / (4 * R);
  if (b < med_wgs) {
    const int64_t mw = b * 4 + wave;
    if constexpr (R > 1) {
      if (mw * R < A.n_medium) medium_rows_q<B>(A, qw, sums, mw, lane);
    } else {
      if (mw < A.n_medium) medium_wave<B, Q, MG, FL>(A, qw, mw, lane);
    }
    return;
  }
  b -= med_wgs;
  const int64_t lw = b * 4 + wave;
  if (lw * 64 < A.n_light) light_wave<B, Q, MG, FL>(A, qw, sums, lw, lane);
}

// Items of a multi-graph pass (R = 1).
__device__ __forceinline__ int64_t pass_items(const PassArgs& A) {
  return A.n_items + (A.n_medium + 3) / 4 + (A.n_light + 255) / 256;
}

// Tickets of the persistent kernels' work cursor: one per heavy chunk and
// per medium workgroup item, one per K light-row items.  A ticket is one
// atomic on a single address: where most rows have little or nothing to do
// (queued passes, and direct passes of a batch once a third of its rows
// belong to converged graphs) one item per ticket makes that atomic the
// bottleneck, so light items are taken K = 8 at a time.  Other direct passes
// take one item per ticket: with the whole GPU on a narrow window of
// consecutive rows the counters of nearby successors stay in L2 (measured on
// the 4096-graph batch: K = 8 makes its all-active dense passes 20 % slower,
// K = 1 its first half-converged pass 45 % slower).
// Batching needs far more light items than workgroups (a served engine's
// pass may have only thousands: taking them eight at a time would leave most
// of the grid idle).
__device__ __forceinline__ int ticket_batch(const PassArgs& A0, bool queued) {
  const int64_t light_items = (A0.n_light + 255) / 256;
  if (light_items < 64 * (int64_t)gridDim.x) return 1;
  if (queued) return 8;
  const PassCtl* c = A0.ctl;
  return c->batch && 3ull * c->rows_done > (unsigned long long)A0.n ? 8 : 1;
}

struct Tickets {
  int64_t single;  // heavy + medium items
  int64_t total;   // items
  int64_t count;   // tickets
};

__device__ __forceinline__ int64_t next_ticket(PassCtl* ctl) { return (int64_t)atomicAdd(&ctl->work, 1ull); }

// `single` items taken one per ticket, then the rest K per ticket.
__device__ __forceinline__ Tickets tickets_of(int64_t single, int64_t total, int K) {
  Tickets t;
  t.single = single;
  t.total = total;
  t.count = t.single + (t.total - t.single + K - 1) / K;
  return t;
}

__device__ __forceinline__ Tickets pass_tickets(const PassArgs& A, int K) {
  return tickets_of(A.n_items + (A.n_medium + 3) / 4, pass_items(A), K);
}

// Items [*b0, *b1) of ticket k.
__device__ __forceinline__ void ticket_items(const Tickets& t, int K, int64_t k, int64_t* b0, int64_t* b1) {
  if (k < t.single) {
    *b0 = k;
    *b1 = k + 1;
  } else {
    *b0 = t.single + (k - t.single) * K;
    *b1 = *b0 + K < t.total ? *b0 + K : t.total;
  }
}

__device__ __forceinline__ bool queued_mode(const PassArgs& A) {
  return !(A.mode == MODE_FIRST || A.mode == MODE_DENSE) || A.qdense;
}

#if HB_WAVES > 0
#define HB_EXPAND_ATTR __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(HB_WAVES)))
#else
#define HB_EXPAND_ATTR __launch_bounds__(256)
#endif
// Waves per SIMD the persistent (multi-graph) expand kernel is compiled for:
// it holds more state than the grid kernels (work cursor, graph lookups), and
// at 4 waves its 128 registers avoid the spills it has at 5 (measured 15 %
// faster on the 4096-graph batch).
#ifndef HB_PERSIST_WAVES
#define HB_PERSIST_WAVES 4
#endif
#if HB_PERSIST_WAVES > 0
#define HB_PERSIST_ATTR __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(HB_PERSIST_WAVES)))
#else
#define HB_PERSIST_ATTR __launch_bounds__(256)
#endif

template <int B, int FL = FL_PLAIN>
__global__ HB_EXPAND_ATTR void k_expand(PassArgs A) {
  if constexpr (FL == FL_PLAIN) {
    __shared__ RowSum sums[4][64];
    if constexpr (B >= 6) {
      __shared__ QEnt qbuf[4][QCAP];  // successor ids of light rows (light_wave_staged)
      expand_item<B, false, false, FL>(A, qbuf[threadIdx.x >> 6], sums[threadIdx.x >> 6], blockIdx.x);
    } else {
      expand_item<B, false, false, FL>(A, nullptr, sums[threadIdx.x >> 6], blockIdx.x);
    }
  } else {
    expand_item<B, false, false, FL>(A, nullptr, nullptr, blockIdx.x);
  }
}

template <int B, int FL = FL_PLAIN>
__global__ HB_EXPAND_ATTR void k_expand_q(PassArgs A) {
  __shared__ QEnt qbuf[4][QCAP];
  if constexpr (FL == FL_PLAIN) {
    __shared__ RowSum sums[4][64];  // light_wave_scanned
    expand_item<B, true, false, FL>(A, qbuf[threadIdx.x >> 6], sums[threadIdx.x >> 6], blockIdx.x);
  } else {
    expand_item<B, true, false, FL>(A, qbuf[threadIdx.x >> 6], nullptr, blockIdx.x);
  }
}

// Persistent form for device-driven passes: a fixed grid whose workgroups
// take items from the pass's work cursor until none is left.  Both gather
// forms are launched every pass; the one that does not match the pass mode
// returns at once.
template <int B, bool Q>
__global__ HB_PERSIST_ATTR void k_expand_p(PassArgs A0) {
  const PassArgs A = resolve(A0);
  if (queued_mode(A) != Q) return;
  if (!Q && A.mode == MODE_FIRST && A0.singletons) return;  // k_expand_codes_p runs it
  __shared__ QEnt qbuf[Q ? 4 : 1][Q ? QCAP : 1];
  __shared__ RowSum sums[Q ? 1 : 4][64];  // light_wave_direct
  __shared__ int64_t ticket;
  const int K = ticket_batch(A0, Q);
  const Tickets tk = pass_tickets(A, K);
  for (;;) {
    if (threadIdx.x == 0) ticket = next_ticket(A0.ctl);
    __syncthreads();
    const int64_t k = ticket;
    __syncthreads();
    if (k >= tk.count) break;
    int64_t b0, b1;
    ticket_items(tk, K, k, &b0, &b1);
    for (int64_t b = b0; b < b1; ++b)
      expand_item<B, Q, true>(A, Q ? qbuf[threadIdx.x >> 6] : nullptr, Q ? nullptr : sums[threadIdx.x >> 6], b);
  }
}

// Folds the partial counters of every heavy row into the row (one wavefront
// per heavy row) and finishes it like any other row.
template <int B, bool MG, int FL = FL_PLAIN>
__global__ __launch_bounds__(256) void k_merge(PassArgs A0) {
  const PassArgs A = resolve(A0);
  constexpr int P = 1 << B;
  constexpr int G = P / 16;
  constexpr int W = 64 / G;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int gl = lane % G;
  const int grp = lane / G;
  const int64_t h = (int64_t)blockIdx.x * 4 + wave;
  if (h >= A.n_hrows) return;
  const HeavyRow hr = A.hrows[h];
  bool own_mod, need;
  row_flags<MG>(A, hr.row, own_mod, need);
  if (!need) return;
  RowPre pre;
  if (grp == 0) pre = preload<B, FL>(A, hr.row, gl);
  uint4 acc = zero4();
  for (int64_t j = grp; j < hr.nitems; j += W)
    acc = bmax(acc, *reinterpret_cast<const uint4*>(A.partial + (size_t)(hr.item0 + j) * P +
                                                    (size_t)gl * 16));
#pragma unroll
  for (int o = G; o < 64; o <<= 1) acc = bmax(acc, shfl_xor4(acc, o));
  Counts c{};
  if (grp == 0) finish_row<B, MG, FL>(A, hr.row, acc, true, pre, own_mod, gl, 0, c);
  flush_counts<FL>(A, c, h, lane);
}

// --- the first pass from node hashes --------------------------------------------
//
// Before the first pass every counter holds its own node's single item, so it
// is fully described by the index j and value of its one nonzero register,
// both taken from the node's hash (code = j << 8 | value), and the
// register-wise maximum over a row's successors is the maximum, per register
// index, of their codes' values.  The first pass of an unweighted
// single-graph context therefore recomputes each successor's code from its id
// instead of reading its p-byte counter: lanes take consecutive arcs, hash
// the successor, and fold the code into a register array in LDS (one 32-bit
// word per register, LDS atomic max), which the row's lane group then packs
// into its 16-byte slices.  The pass reads only the arc list; the counters,
// accumulators and change bits it writes are the ones the gather over
// counters writes.

constexpr int CODE_WORDS = 1024;  // LDS words per wavefront: (64 / G) rows x p registers

// Code of node v's singleton counter: register index j (the hash's top B
// bits) and value rho+ of the remaining bits, as the counters are initialised.
template <int B>
__device__ __forceinline__ uint32_t singleton_code(uint64_t v, uint64_t seed) {
  const uint64_t h = node_hash(v, seed);
  const uint32_t j = (uint32_t)(h >> (64 - B));
  const uint64_t rest = h << B;
  const uint32_t r = rest == 0ull ? (uint32_t)(65 - B) : (uint32_t)__clzll((long long)rest) + 1u;
  return (j << 8) | r;
}

// Lane gl's 16-byte slice of the singleton counter with code x.
__device__ __forceinline__ uint4 code_slice(uint32_t x, int gl) {
  const uint32_t j = x >> 8;
  const uint32_t val = (x & 0xffu) << (8u * (j & 3u));
  const uint32_t q = (j >> 2) & 3u;
  const bool mine = (int)(j >> 4) == gl;
  return make_uint4(mine && q == 0u ? val : 0u, mine && q == 1u ? val : 0u, mine && q == 2u ? val : 0u,
                    mine && q == 3u ? val : 0u);
}

// Registers gl*16 .. gl*16+15 of an LDS register array packed into the
// lane's slice; the words are cleared for the next row.
__device__ __forceinline__ uint4 take_slice(uint32_t* regs, int gl) {
  uint4* q = reinterpret_cast<uint4*>(regs + gl * 16);
  const uint4 a = q[0], b = q[1], c = q[2], d = q[3];
  q[0] = zero4();
  q[1] = zero4();
  q[2] = zero4();
  q[3] = zero4();
  return make_uint4(a.x | a.y << 8 | a.z << 16 | a.w << 24, b.x | b.y << 8 | b.z << 16 | b.w << 24,
                    c.x | c.y << 8 | c.z << 16 | c.w << 24, d.x | d.y << 8 | d.z << 16 | d.w << 24);
}

// Folds the codes of successors idx[k], idx[k + st], ... < e into regs, UC
// ids in flight.  The hash is the costly part (two 64-bit products), so a
// slot no lane of the wavefront has is branched over, not computed and
// discarded (light rows have only a few arcs per lane).
constexpr int UC = 8;

// Hash key of a row's graph: arena base and hash seed (multi-graph contexts
// number nodes within their graph; every arc stays inside it, so a row's
// successors share the row's key).
struct GraphKey {
  int64_t base;
  uint64_t seed;
};

template <bool MG>
__device__ __forceinline__ GraphKey key_of(const PassArgs& A, int64_t row) {
  if constexpr (MG) {
    const GraphDev& gd = A.graphs[A.blk_graph[row >> 6]];
    return GraphKey{gd.node_base, gd.seed};
  }
  return GraphKey{0, A.seed};
}

template <int B>
__device__ __forceinline__ void fold_codes(const PassArgs& A, uint32_t* regs, int64_t k, int64_t e, int64_t st,
                                           GraphKey key) {
  for (; k < e; k += st * UC) {
    int32_t w[UC];
#pragma unroll
    for (int u = 0; u < UC; ++u) {
      const int64_t kk = k + u * st;
      w[u] = kk < e ? ld_stream(A.idx + kk) : -1;
    }
#pragma unroll
    for (int u = 0; u < UC; ++u)
      if (w[u] >= 0) {
        const uint32_t x = singleton_code<B>((uint64_t)(w[u] - key.base), key.seed);
        __hip_atomic_fetch_max(regs + (x >> 8), x & 0xffu, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
      }
  }
}

// Light rows of a first pass, 64 list entries per wavefront, W rows at a
// time (one per lane group): the group folds its row's successor codes into
// an LDS register array, packs it and finishes the row in two steps
// (finish_group, finish_lane).  Each lane looks up its own row's hash key,
// hashes the row's node and loads the row's estimate and accumulators once,
// up front.
template <int B, bool MG>
__device__ __forceinline__ void light_codes_1(const PassArgs& A, uint32_t* lds, RowSum* sums, int64_t lw, int lane) {
  constexpr int P = 1 << B;
  constexpr int G = P / 16;
  constexpr int W = 64 / G;
  const int gl = lane % G;
  const int grp = lane / G;
  const int64_t i = lw * 64 + lane;
  int64_t row = 0, s = 0, deg = 0;
  bool own_mod = false, need = false;
  uint32_t code = 0u;
  GraphKey key{0, A.seed};
  double e0 = 0.0, s0 = 0.0, h0 = 0.0;
  if (i < A.n_light) {
    row = A.light[i];
    s = A.off[row];
    deg = A.off[row + 1] - s;
    row_flags<MG>(A, row, own_mod, need);
    if (need) {
      key = key_of<MG>(A, row);
      e0 = ld_stream(A.E + row);
      s0 = ld_stream(A.S + row);
      h0 = ld_stream(A.H + row);
      code = singleton_code<B>((uint64_t)(row - key.base), key.seed);
    }
  }
  const uint64_t live = __ballot(need);
  uint32_t* regs = lds + grp * P;
  Counts c{};
  for (int r = 0; r < G; ++r) {
    const int rl = r * W + grp;
    const int64_t rrow = __shfl(row, rl);
    const int64_t rs = __shfl(s, rl);
    const int64_t rd = __shfl(deg, rl);
    const uint32_t rcode = __shfl(code, rl);
    GraphKey rkey{0, A.seed};
    if constexpr (MG) {
      rkey.base = __shfl(key.base, rl);
      rkey.seed = __shfl(key.seed, rl);
    }
    const bool on = ((live >> rl) & 1ull) != 0ull;
    if (on) fold_codes<B>(A, regs, rs + gl, rs + rd, G, rkey);
    wave_sync();
    if (on) {
      const uint4 acc = take_slice(regs, gl);
      finish_group<B>(A, rrow, acc, rd > 0, code_slice(rcode, gl), false, gl, grp, sums + rl);
      if (gl == 0) {
        c.gath += (uint32_t)rd;
        c.arcs += (uint32_t)rd;
      }
    }
    wave_sync();
  }
  finish_lane<B, MG>(A, row, need, false, sums, lane, e0, s0, h0, c);
  flush_counts(A, c, lw, lane);
}

// Medium rows of a first pass, R to a wavefront (R = batched_med_rows(B)):
// all 64 lanes fold each row's successor codes in turn into that row's own
// LDS register array, then the rows' lane groups pack and finish them
// together in two steps (finish_group, finish_lane), so that the per-row work
// runs once per R rows instead of once per row.

template <int B, bool MG>
__device__ __forceinline__ void medium_codes(const PassArgs& A, uint32_t* lds, RowSum* sums, int64_t mw, int lane) {
  constexpr int P = 1 << B;
  constexpr int G = P / 16;
  constexpr int R = batched_med_rows(B);
  const int gl = lane % G;
  const int grp = lane / G;
  const int64_t i = mw * R + lane;
  int64_t row = 0, s = 0, deg = 0;
  bool own_mod = false, need = false;
  uint32_t code = 0u;
  GraphKey key{0, A.seed};
  double e0 = 0.0, s0 = 0.0, h0 = 0.0;
  if (lane < R && i < A.n_medium) {
    row = A.medium[i];
    s = A.off[row];
    deg = A.off[row + 1] - s;
    row_flags<MG>(A, row, own_mod, need);
    if (need) {
      key = key_of<MG>(A, row);
      e0 = ld_stream(A.E + row);
      s0 = ld_stream(A.S + row);
      h0 = ld_stream(A.H + row);
      code = singleton_code<B>((uint64_t)(row - key.base), key.seed);
    }
  }
  const uint64_t live = __ballot(need);
  Counts c{};
#pragma unroll 1
  for (int r = 0; r < R; ++r) {
    const int64_t rs = __shfl(s, r);
    const int64_t rd = __shfl(deg, r);
    GraphKey rkey{0, A.seed};
    if constexpr (MG) {
      rkey.base = __shfl(key.base, r);
      rkey.seed = __shfl(key.seed, r);
    }
    if (((live >> r) & 1ull) == 0ull) continue;  // uniform
    fold_codes<B>(A, lds + r * P, rs + lane, rs + rd, 64, rkey);
    if (lane == 0) {
      c.gath += (uint32_t)rd;
      c.arcs += (uint32_t)rd;
    }
  }
  wave_sync();
  const int64_t grow = __shfl(row, grp);
  const int64_t gdeg = __shfl(deg, grp);
  const uint32_t gcode = __shfl(code, grp);
  if (grp < R && ((live >> grp) & 1ull) != 0ull) {
    const uint4 acc = take_slice(lds + grp * P, gl);
    finish_group<B>(A, grow, acc, gdeg > 0, code_slice(gcode, gl), false, gl, grp, sums + grp);
  }
  wave_sync();
  finish_lane<B, MG>(A, row, need, false, sums, lane, e0, s0, h0, c);
  flush_counts(A, c, mw, lane);
}

// Work items of a first pass: [heavy chunks][medium: 4 R rows each][light: 256 rows each].
template <int B>
__host__ __device__ constexpr int64_t codes_items(int64_t n_items, int64_t n_medium, int64_t n_light) {
  return n_items + (n_medium + 4 * batched_med_rows(B) - 1) / (4 * batched_med_rows(B)) + (n_light + 255) / 256;
}

// One chunk of a heavy row per workgroup: its four wavefronts fold into one
// register array; the chunk's maximum goes to its partial counter (merged
// with the row's own counter by k_merge).
template <int B, bool MG>
__device__ __forceinline__ void heavy_codes(const PassArgs& A, uint32_t* lds, int64_t item, int lane, int wave) {
  constexpr int P = 1 << B;
  constexpr int G = P / 16;
  const int gl = lane % G;
  const int grp = lane / G;
  const HeavyItem it = A.items[item];
  bool own_mod, need;
  row_flags<MG>(A, it.row, own_mod, need);
  if (!need) return;  // uniform over the workgroup; the merge kernel skips the row too
  fold_codes<B>(A, lds, it.e0 + wave * 64 + lane, it.e1, 256, key_of<MG>(A, it.row));
  Counts c{};
  if (lane == 0 && wave == 0) {
    c.gath += (uint32_t)(it.e1 - it.e0);
    c.arcs += (uint32_t)(it.e1 - it.e0);
  }
  flush_counts(A, c, item, lane);
  __syncthreads();
  if (wave == 0 && grp == 0)
    *reinterpret_cast<uint4*>(A.partial + (size_t)item * P + (size_t)gl * 16) = take_slice(lds, gl);
}

// One work item, numbered as codes_items counts them.
template <int B, bool MG>
__device__ __forceinline__ void codes_item(const PassArgs& A, uint32_t (*regs)[CODE_WORDS], RowSum (*sums)[64],
                                           int64_t b, int lane, int wave) {
  if (b == 0)
    for (int i = threadIdx.x; i < STAT_SLOTS * STAT_K; i += blockDim.x) A.stats_next[i] = 0ull;
  if (b < A.n_items) {
    heavy_codes<B, MG>(A, regs[0], b, lane, wave);
    return;
  }
  b -= A.n_items;
  constexpr int R = batched_med_rows(B);
  const int64_t med_wgs = (A.n_medium + 4 * R - 1) / (4 * R);
  if (b < med_wgs) {
    const int64_t mw = b * 4 + wave;
    if (mw * R < A.n_medium) medium_codes<B, MG>(A, regs[wave], sums[wave], mw, lane);
    return;
  }
  b -= med_wgs;
  const int64_t lw = b * 4 + wave;
  if (lw * 64 < A.n_light) light_codes_1<B, MG>(A, regs[wave], sums[wave], lw, lane);
}

template <int B>
__global__ HB_EXPAND_ATTR void k_expand_codes(PassArgs A) {
  __shared__ uint32_t regs[4][CODE_WORDS];
  __shared__ RowSum sums[4][64];
  uint4* z = reinterpret_cast<uint4*>(&regs[0][0]);
  for (int i = threadIdx.x; i < CODE_WORDS; i += 256) z[i] = zero4();  // 4 waves x CODE_WORDS words
  __syncthreads();
  codes_item<B, false>(A, regs, sums, blockIdx.x, threadIdx.x & 63, threadIdx.x >> 6);
}

// Persistent form for the first device-driven pass of a batched context (a
// no-op in any other pass); items from the pass's work cursor.  The register
// arrays are left clear by every item, so they are zeroed once.
template <int B>
__global__ HB_PERSIST_ATTR void k_expand_codes_p(PassArgs A0) {
  const PassArgs A = resolve(A0);
  if (A.mode != MODE_FIRST || !A0.singletons) return;
  __shared__ uint32_t regs[4][CODE_WORDS];
  __shared__ RowSum sums[4][64];
  __shared__ int64_t ticket;
  uint4* z = reinterpret_cast<uint4*>(&regs[0][0]);
  for (int i = threadIdx.x; i < CODE_WORDS; i += 256) z[i] = zero4();
  // no counter gathers, so no L2 window to keep narrow: batch when there are enough items
  const int K = (A.n_light + 255) / 256 >= 64 * (int64_t)gridDim.x ? 8 : 1;
  const int64_t total = codes_items<B>(A.n_items, A.n_medium, A.n_light);
  const Tickets tk = tickets_of(total - (A.n_light + 255) / 256, total, K);
  for (;;) {
    __syncthreads();
    if (threadIdx.x == 0) ticket = next_ticket(A0.ctl);
    __syncthreads();
    const int64_t k = ticket;
    if (k >= tk.count) break;
    int64_t b0, b1;
    ticket_items(tk, K, k, &b0, &b1);
    for (int64_t b = b0; b < b1; ++b) codes_item<B, true>(A, regs, sums, b, threadIdx.x & 63, threadIdx.x >> 6);
  }
}

// Counters wider than 256 bytes: one workgroup per 64-row block, rows in
// sequence, each thread owning 16-byte chunks tid, tid+256, ...; the new
// counter is staged in LDS (p bytes) until the change decision is known.
__global__ __launch_bounds__(256) void k_expand_wide(PassArgs A, int log2m) {
  extern __shared__ uint4 stage[];
  __shared__ double red_big[256];
  __shared__ double red_small[256];
  __shared__ int red_v[256];
  const int P = 1 << log2m;
  const int C = P / 16;
  const int tid = threadIdx.x;
  if (blockIdx.x == 0)
    for (int i = tid; i < STAT_SLOTS * STAT_K; i += blockDim.x) A.stats_next[i] = 0ull;
  const int64_t blk = blockIdx.x;
  const int64_t r0 = blk * 64;
  const uint64_t own_word = A.mode == MODE_FIRST ? 0ull : A.mod_prev[blk];
  const bool all = A.mode != MODE_SPARSE;
  uint64_t bits = 0;
  uint32_t ngath = 0, nload = 0, nwrite = 0;
  unsigned long long narcs = 0;
  for (int rl = 0; rl < 64; ++rl) {
    const int64_t row = r0 + rl;
    if (row >= A.n) break;
    const int64_t s = A.off[row], e = A.off[row + 1];
    const bool own_mod = ((own_word >> rl) & 1ull) != 0ull;
    int mine = 0;
    for (int64_t k = s + tid; k < e; k += 256) {
      const int32_t w = A.idx[k];
      if (all || bit_of(A.mod_prev, w)) ++mine;
    }
    const int ngot = __syncthreads_count(mine);
    const bool got = ngot > 0;
    ngath += (uint32_t)ngot;
    narcs += (unsigned long long)(e - s);
    if (!got && !own_mod) continue;
    ++nload;
    int diff = 0;
    for (int c = tid; c < C; c += 256) {
      const uint4 own = *reinterpret_cast<const uint4*>(A.cur + (size_t)row * P + (size_t)c * 16);
      uint4 a = own;
      if (got)
        for (int64_t k = s; k < e; ++k) {
          const int32_t w = A.idx[k];
          if (all || bit_of(A.mod_prev, w))
            a = bmax(a, *reinterpret_cast<const uint4*>(A.cur + (size_t)w * P + (size_t)c * 16));
        }
      diff |= differs(a, own) ? 1 : 0;
      stage[c] = a;
    }
    const bool changed = __syncthreads_or(diff) != 0;
    if (changed || own_mod) {
      ++nwrite;
      for (int c = tid; c < C; c += 256)
        *reinterpret_cast<uint4*>(A.nxt + (size_t)row * P + (size_t)c * 16) = stage[c];
    }
    if (changed) {
      double big = 0.0, small = 0.0;
      int V = 0;
      for (int c = tid; c < C; c += 256) {
        const Parts pr = reg_parts(stage[c]);
        big += pr.big;
        small += pr.small;
        V += pr.zeros;
      }
      red_big[tid] = big;
      red_small[tid] = small;
      red_v[tid] = V;
      __syncthreads();
      for (int o = 128; o > 0; o >>= 1) {
        if (tid < o) {
          red_big[tid] += red_big[tid + o];
          red_small[tid] += red_small[tid + o];
          red_v[tid] += red_v[tid + o];
        }
        __syncthreads();
      }
      if (tid == 0) {
        const double En = estimate(red_big[0], red_small[0], red_v[0], A.alpha_pp, (double)P, A.lc);
        const double delta = En - A.E[row];
        A.S[row] = A.S[row] + A.d * delta;
        A.H[row] = A.H[row] + delta / A.d;
        A.E[row] = En;
      }
      bits |= 1ull << rl;
      __syncthreads();
    }
  }
  if (tid == 0) {
    A.mod_cur[blk] = bits;
    unsigned long long* st = A.stats + (blk & (STAT_SLOTS - 1)) * STAT_K;
    Counts c{};
    c.gath = ngath;
    c.load = nload;
    c.write = nwrite;
    c.chg = (uint32_t)__popcll(bits);
    add_stats(st, c);
    if (narcs) atomicAdd(st + 4, narcs);
    if (ngath) atomicAdd(st + 5, (unsigned long long)ngath * (unsigned long long)C);
  }
}

__global__ void k_fill_zero(uint4* p, size_t n16, uint8_t* tail, size_t ntail) {
  const size_t stride = (size_t)gridDim.x * blockDim.x;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) p[i] = zero4();
  if (blockIdx.x == 0)
    for (size_t i = threadIdx.x; i < ntail; i += blockDim.x) tail[i] = 0;
}

// --- streamed graphs ----------------------------------------------------------
//
// A streamed graph's arcs are uploaded in row chunks every pass.  While its
// first pass streams every chunk, k_pred_masks records for every node w which
// chunks hold an arc into w (bit c % 32 of mask[w] for chunk c).  A later
// pass only needs the chunks that hold a row with a changed successor or a
// row that changed itself (its write-back): k_chunk_activity ORs, over the
// nodes changed in the previous pass, their masks and the bit of their own
// chunk.  With more than 32 chunks a bit stands for every 32nd chunk, so the
// selection is a superset of the chunks that have work.

__global__ void k_pred_masks(const int32_t* __restrict__ idx, int64_t count, uint32_t bit, uint32_t* mask) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count; e += stride) {
    const int32_t w = idx[e];
    if ((__ldg(mask + w) & bit) == 0u) atomicOr(mask + w, bit);
  }
}

__global__ void k_chunk_activity(const uint64_t* __restrict__ mod_prev, int64_t n_words, const uint32_t* __restrict__ mask,
                                 const int64_t* __restrict__ chunk_rows, int32_t n_chunks, uint32_t* act) {
  uint32_t acc = 0u;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_words; i += stride) {
    uint64_t word = mod_prev[i];
    while (word) {
      const int b = __ffsll((long long)word) - 1;
      word &= word - 1ull;
      const int64_t w = i * 64 + b;
      // own chunk: the last c with chunk_rows[c] <= w
      int32_t lo = 0, hi = n_chunks - 1;
      while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (chunk_rows[mid] <= w) lo = mid; else hi = mid - 1;
      }
      acc |= mask[w] | (1u << (lo & 31));
    }
  }
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) acc |= __shfl_xor(acc, o);
  if ((threadIdx.x & 63) == 0 && acc) atomicOr(act, acc);
}

// Compressed streamed chunks: a chunk's arcs are cut into blocks of
// STREAM_BLOCK_ARCS consecutive arcs (across row boundaries).  A block is a
// header byte, its first successor id as a variable-length integer (7 bits
// per byte, low bits first, high bit set on every byte but the last), then
// the zigzag-coded differences between consecutive ids: as variable-length
// integers too (header 0), or bit-packed, each W = header - 1 bits wide, low
// bits first.  boff[b] is the byte offset of block b in the chunk's bytes,
// which are followed by at least 8 readable bytes.  Each workgroup first
// copies the bytes of its 256 blocks into LDS (one coalesced copy), then each
// thread decodes one block into ids.
constexpr int DECODE_LDS = 256 * (1 + STREAM_BLOCK_ARCS * 5);  // bytes of 256 blocks at worst

// At most 5 bytes (a 32-bit value), so a damaged stream cannot run on.
__device__ __forceinline__ uint32_t read_varint(const uint8_t* p, int& at) {
  uint32_t v = 0;
#pragma unroll
  for (int k = 0; k < 5; ++k) {
    const uint32_t byte = p[at++];
    v |= (byte & 0x7fu) << (7 * k);
    if (!(byte & 0x80u)) break;
  }
  return v;
}

// W <= 32 bits at bit position `bit` of p (reads 5 bytes from bit / 8 on).
__device__ __forceinline__ uint32_t read_bits(const uint8_t* p, uint32_t bit, uint32_t W) {
  const uint8_t* q = p + (bit >> 3);
  const uint64_t x = (uint64_t)q[0] | ((uint64_t)q[1] << 8) | ((uint64_t)q[2] << 16) | ((uint64_t)q[3] << 24) |
                     ((uint64_t)q[4] << 32);
  return (uint32_t)((x >> (bit & 7u)) & ((1ull << W) - 1ull));
}

__global__ __launch_bounds__(256) void k_decode_chunk(const uint32_t* __restrict__ boff, const uint8_t* __restrict__ bytes,
                                                      int64_t n_arcs, int64_t n_blocks, int32_t* __restrict__ ids) {
  __shared__ uint32_t buf[DECODE_LDS / 4 + 4];  // + the partial words at both ends and the read-ahead
  const int64_t b0 = (int64_t)blockIdx.x * 256;
  const int64_t b1 = b0 + 256 < n_blocks ? b0 + 256 : n_blocks;
  const uint32_t lo = boff[b0], hi = boff[b1];
  // the workgroup's bytes [lo, hi) and the 8 after them into LDS, in 4-byte
  // words from lo rounded down
  const uint32_t w0 = lo >> 2, w1 = ((hi + 3) >> 2) + 2;
  const uint32_t* src = reinterpret_cast<const uint32_t*>(bytes);
  for (uint32_t w = w0 + threadIdx.x; w < w1; w += 256) buf[w - w0] = src[w];
  __syncthreads();
  const int64_t b = b0 + threadIdx.x;
  if (b >= b1) return;
  const uint8_t* lds = reinterpret_cast<const uint8_t*>(buf);
  int at = (int)(boff[b] - (w0 << 2));
  const int64_t a0 = b * STREAM_BLOCK_ARCS;
  const int64_t a1 = a0 + STREAM_BLOCK_ARCS < n_arcs ? a0 + STREAM_BLOCK_ARCS : n_arcs;
  const uint32_t head = lds[at++];
  uint32_t cur = read_varint(lds, at);
  ids[a0] = (int32_t)cur;
  if (head == 0u) {
    for (int64_t a = a0 + 1; a < a1; ++a) {
      const uint32_t z = read_varint(lds, at);
      cur += (z >> 1) ^ (0u - (z & 1u));  // zigzag: 2d for d >= 0, -2d-1 for d < 0
      ids[a] = (int32_t)cur;
    }
  } else {
    const uint32_t W = head - 1u < 32u ? head - 1u : 32u;
    uint32_t bit = (uint32_t)at * 8u;
    for (int64_t a = a0 + 1; a < a1; ++a) {
      const uint32_t z = read_bits(lds, bit, W);
      bit += W;
      cur += (z >> 1) ^ (0u - (z & 1u));
      ids[a] = (int32_t)cur;
    }
  }
}

// Algorithm 2 initialisation: c[v] = add(empty counter, v) written into both
// buffers, one thread per 16-byte chunk of a counter (coalesced stores, no
// separate zero fill); the first chunk's thread also zeroes S and H and
// caches E(c[v]) for the singleton counter (p-1 empty registers).
__global__ void k_init_nodes(int log2m, int64_t n, uint64_t seed, uint8_t* cur, uint8_t* nxt,
                             double* S, double* H, double* E, const double* lc, double alpha_pp) {
  const int64_t P = (int64_t)1 << log2m;
  const int64_t C = P / 16;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * C) return;
  const int64_t v = i / C;
  const int64_t chunk = i - v * C;
  const uint64_t h = node_hash((uint64_t)v, seed);
  const uint32_t j = (uint32_t)(h >> (64 - log2m));
  const uint64_t rest = h << log2m;
  const uint32_t r = rest == 0ull ? (uint32_t)(65 - log2m) : (uint32_t)__clzll((long long)rest) + 1u;
  uint32_t w[4] = {0u, 0u, 0u, 0u};
  if ((int64_t)(j >> 4) == chunk) w[(j >> 2) & 3u] = r << (8u * (j & 3u));
  const uint4 val = make_uint4(w[0], w[1], w[2], w[3]);
  *reinterpret_cast<uint4*>(cur + v * P + chunk * 16) = val;
  *reinterpret_cast<uint4*>(nxt + v * P + chunk * 16) = val;
  if (chunk == 0) {
    S[v] = 0.0;
    H[v] = 0.0;
    double big = (double)(P - 1), small = 0.0;
    if (r <= 26u)
      big += pow2neg(r);
    else
      small += pow2neg(r);
    E[v] = estimate(big, small, (int)(P - 1), alpha_pp, (double)P, lc);
  }
}

// Sec. 3 / Sec. 5 finalisation.
__global__ void k_finalize(int64_t n, const double* S, const double* H, const double* E, double* clo,
                           double* lin, double* harm, double* core) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const double s = S[v];
  const double size = E[v];
  if (core) core[v] = size;
  if (clo) clo[v] = (s == 0.0) ? 0.0 : 1.0 / s;
  if (lin) lin[v] = (s == 0.0) ? 1.0 : (size * size) / s;
  if (harm) harm[v] = H[v];
}

// Weighted initialisation (Sec. 6): counter v is the HyperLogLog of the w[v]
// replicas of v, replica j hashing as item v + j * 2^32 (v itself for j = 0);
// thread i writes 16-byte chunk i of the counters into both buffers.  The
// estimates are computed afterwards by k_row_estimate.
__global__ void k_init_weighted(int log2m, int64_t n, uint64_t seed, const int32_t* w, uint8_t* cur, uint8_t* nxt) {
  const int64_t P = (int64_t)1 << log2m;
  const int64_t C = P / 16;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * C) return;
  const int64_t v = i / C;
  const int64_t chunk = i - v * C;
  uint8_t reg[16];
#pragma unroll
  for (int k = 0; k < 16; ++k) reg[k] = 0;
  const int64_t reps = w[v];
  for (int64_t j = 0; j < reps; ++j) {
    const uint64_t h = node_hash((uint64_t)v + ((uint64_t)j << 32), seed);
    const uint32_t idx = (uint32_t)(h >> (64 - log2m));
    if ((int64_t)(idx >> 4) != chunk) continue;
    const uint64_t rest = h << log2m;
    const uint32_t r = rest == 0ull ? (uint32_t)(65 - log2m) : (uint32_t)__clzll((long long)rest) + 1u;
    const uint32_t k = idx & 15u;
#pragma unroll
    for (int q = 0; q < 16; ++q)
      if ((uint32_t)q == k && r > reg[q]) reg[q] = (uint8_t)r;
  }
  uint32_t wd[4];
#pragma unroll
  for (int q = 0; q < 4; ++q)
    wd[q] = (uint32_t)reg[4 * q] | ((uint32_t)reg[4 * q + 1] << 8) | ((uint32_t)reg[4 * q + 2] << 16) |
            ((uint32_t)reg[4 * q + 3] << 24);
  const uint4 val = make_uint4(wd[0], wd[1], wd[2], wd[3]);
  *reinterpret_cast<uint4*>(cur + v * P + chunk * 16) = val;
  *reinterpret_cast<uint4*>(nxt + v * P + chunk * 16) = val;
}

// E[v] = size(counter v) (Algorithm 1), S = H = 0 and, if D is set, D = 0;
// one thread per counter, the register sum accumulated exactly as in the
// pass kernels (terms above and below 2^-26 summed apart, rounded once).
__global__ void k_row_estimate(int log2m, int64_t n, const uint8_t* cnt, double* S, double* H, double* D, double* E,
                               const double* lc, double alpha_pp) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  const int64_t P = (int64_t)1 << log2m;
  const uint4* row = reinterpret_cast<const uint4*>(cnt + v * P);
  double big = 0.0, small = 0.0;
  int V = 0;
  for (int64_t c = 0; c < P / 16; ++c) {
    const Parts pr = reg_parts(row[c]);
    big += pr.big;
    small += pr.small;
    V += pr.zeros;
  }
  E[v] = estimate(big, small, V, alpha_pp, (double)P, lc);
  S[v] = 0.0;
  H[v] = 0.0;
  if (D) D[v] = 0.0;
}

// --- exact sum of the estimates (neighbourhood function) ------------------
// Every estimate is 0 or at least 1, hence a multiple of 2^-52 below 2^66:
// E * 2^52 is an integer below 2^118, and the sum of up to 2^31 of them fits
// 192 bits.  Integer addition is associative, so the sum does not depend on
// the reduction order; it is rounded to double once, on the host.
struct Fix192 {
  unsigned long long w0, w1, w2;
};

__device__ __forceinline__ void fix_add(Fix192& a, const Fix192& b) {
  const unsigned long long s0 = a.w0 + b.w0;
  const unsigned long long c0 = s0 < a.w0 ? 1ull : 0ull;
  const unsigned long long s1a = a.w1 + b.w1;
  const unsigned long long c1a = s1a < a.w1 ? 1ull : 0ull;
  const unsigned long long s1 = s1a + c0;
  const unsigned long long c1b = s1 < s1a ? 1ull : 0ull;
  a.w0 = s0;
  a.w1 = s1;
  a.w2 = a.w2 + b.w2 + c1a + c1b;
}

// E * 2^52 as a 192-bit integer; sets *inexact if E is not a multiple of 2^-52.
__device__ __forceinline__ Fix192 fix_of(double e, int* inexact) {
  Fix192 f{0ull, 0ull, 0ull};
  const unsigned long long bits = (unsigned long long)__double_as_longlong(e);
  const int ex = (int)((bits >> 52) & 0x7FFull);
  if (ex == 0) {
    if (bits != 0ull) *inexact = 1;  // subnormal
    return f;
  }
  const unsigned long long mant = (bits & ((1ull << 52) - 1ull)) | (1ull << 52);
  const int sh = ex - 1023;  // E * 2^52 = mant * 2^sh
  if (sh < 0) {
    if (sh <= -53 || (mant & ((1ull << (-sh)) - 1ull))) *inexact = 1;
    f.w0 = sh <= -53 ? 0ull : mant >> (-sh);
  } else if (sh < 64) {
    f.w0 = mant << sh;
    f.w1 = sh == 0 ? 0ull : mant >> (64 - sh);
  } else if (sh < 128) {
    f.w1 = mant << (sh - 64);
    f.w2 = sh == 64 ? 0ull : mant >> (128 - sh);
  } else {
    *inexact = 1;  // beyond 2^75: not an estimate of any counter
  }
  return f;
}

__global__ __launch_bounds__(256) void k_esum(const double* E, int64_t n, Fix192* partial, int* inexact) {
  __shared__ Fix192 red[256];
  Fix192 acc{0ull, 0ull, 0ull};
  int bad = 0;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride)
    fix_add(acc, fix_of(E[v], &bad));
  if (bad) atomicOr(inexact, 1);
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) fix_add(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

__global__ void k_check_weights(const int32_t* w, int64_t n, int* bad) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride)
    if (w[v] < 1) *bad = 1;
}

// Sums the block partials; out[3] receives the inexact flag, which is
// cleared for the next sum.
__global__ __launch_bounds__(256) void k_esum_final(const Fix192* partial, int nblocks, uint64_t* out, int* inexact) {
  __shared__ Fix192 red[256];
  Fix192 acc{0ull, 0ull, 0ull};
  for (int b = (int)threadIdx.x; b < nblocks; b += (int)blockDim.x) fix_add(acc, partial[b]);
  red[threadIdx.x] = acc;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if ((int)threadIdx.x < h) fix_add(red[threadIdx.x], red[threadIdx.x + h]);
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    out[0] = red[0].w0;
    out[1] = red[0].w1;
    out[2] = red[0].w2;
    out[3] = (uint64_t)(*inexact != 0 ? 1 : 0);
    *inexact = 0;
  }
}

// Ensemble initialisation: as k_init_nodes, with K = 2^seg_log counters per
// row; thread i writes 16-byte chunk i of the rows, counter k of node v
// hashes v with seeds[k], and E, S, H hold K values per node.
__global__ void k_init_ensemble(int log2m, int seg_log, int64_t n, const uint64_t* seeds, uint8_t* cur, uint8_t* nxt,
                                double* S, double* H, double* E, const double* lc, double alpha_pp) {
  const int64_t P = (int64_t)1 << log2m;
  const int64_t C = P / 16;                 // chunks per counter
  const int64_t K = (int64_t)1 << seg_log;  // counters per row
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n * C * K) return;
  const int64_t v = i / (C * K);
  const int64_t chunk = i - v * C * K;
  const int64_t k = chunk / C;
  const int64_t ck = chunk - k * C;
  const uint64_t h = node_hash((uint64_t)v, seeds[k]);
  const uint32_t j = (uint32_t)(h >> (64 - log2m));
  const uint64_t rest = h << log2m;
  const uint32_t r = rest == 0ull ? (uint32_t)(65 - log2m) : (uint32_t)__clzll((long long)rest) + 1u;
  uint32_t w[4] = {0u, 0u, 0u, 0u};
  if ((int64_t)(j >> 4) == ck) w[(j >> 2) & 3u] = r << (8u * (j & 3u));
  const uint4 val = make_uint4(w[0], w[1], w[2], w[3]);
  *reinterpret_cast<uint4*>(cur + (v * K) * P + chunk * 16) = val;
  *reinterpret_cast<uint4*>(nxt + (v * K) * P + chunk * 16) = val;
  if (ck == 0) {
    S[v * K + k] = 0.0;
    H[v * K + k] = 0.0;
    double big = (double)(P - 1), small = 0.0;
    if (r <= 26u)
      big += pow2neg(r);
    else
      small += pow2neg(r);
    E[v * K + k] = estimate(big, small, (int)(P - 1), alpha_pp, (double)P, lc);
  }
}

// One run's centrality `which` of entry i (0 closeness, 1 Lin, 2 harmonic,
// 3 coreachable size), as k_finalize computes it.
__device__ __forceinline__ double centrality_of(int which, const double* S, const double* H, const double* E,
                                                int64_t i) {
  const double s = S[i];
  const double size = E[i];
  if (which == 0) return (s == 0.0) ? 0.0 : 1.0 / s;
  if (which == 1) return (s == 0.0) ? 1.0 : (size * size) / s;
  if (which == 2) return H[i];
  return size;
}

// Mean and empirical standard deviation (K - 1 in the denominator) over the
// K seeds of a node, summing in seed order.
__global__ void k_ensemble_summary(int64_t n, int K, int which, const double* S, const double* H, const double* E,
                                   double* mean, double* sd) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n) return;
  double m = centrality_of(which, S, H, E, v * K);
  for (int k = 1; k < K; ++k) m = m + centrality_of(which, S, H, E, v * K + k);
  m = m / (double)K;
  double q = 0.0;
  for (int k = 0; k < K; ++k) {
    const double d = centrality_of(which, S, H, E, v * K + k) - m;
    q = q + d * d;
  }
  if (mean) mean[v] = m;
  if (sd) sd[v] = K > 1 ? sqrt(q / (double)(K - 1)) : 0.0;
}

__global__ void k_widen(const int32_t* in, int64_t* out, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) out[i] = (int64_t)in[i];
}

__global__ void k_validate(const int64_t* off, const int32_t* idx, int64_t n, int64_t m, int* bad) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t i = t0; i <= n; i += stride) {
    const int64_t o = off[i];
    bool ok = o >= 0 && o <= m;
    if (i == 0) ok = ok && o == 0;
    if (i == n) ok = ok && o == m;
    if (i < n) ok = ok && off[i + 1] >= o;
    if (!ok) atomicOr(bad, 1);
  }
  for (int64_t k = t0; k < m; k += stride) {
    const int32_t w = idx[k];
    if (w < 0 || (int64_t)w >= n) atomicOr(bad, 2);
  }
}

// --- reverse CSR and push activation ---------------------------------------

// Rows with lo <= degree <= hi (row classes of the degree-aware schedule).
struct DegreeIn {
  const int64_t* off;
  int64_t lo, hi;
  __host__ __device__ bool operator()(const int32_t& v) const {
    const int64_t d = off[v + 1] - off[v];
    return d >= lo && d <= hi;
  }
};

__global__ void k_take_offsets(const int32_t* rows, int64_t count, const int64_t* off, int64_t* out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  out[2 * i] = off[rows[i]];
  out[2 * i + 1] = off[rows[i] + 1];
}

// Reverse CSR by sorting: the arcs (v -> w) as (key w, value v) pairs are
// radix-sorted by w, which lists the predecessors of each node in increasing
// order; k_arc_rows makes the values, k_lower_bound the offsets.
__global__ void k_arc_rows(const int64_t* off, int64_t n, int32_t* rows) {
  const int lane = threadIdx.x & 63;
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x / 64);
  for (int64_t v = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); v < n; v += nw) {
    const int64_t e1 = off[v + 1];
    for (int64_t e = off[v] + lane; e < e1; e += 64) rows[e] = (int32_t)v;
  }
}

// roff[w] = number of sorted keys below w, for w = 0..n.
__global__ void k_lower_bound(const int32_t* keys, int64_t m, int64_t n, int64_t* roff) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; w <= n; w += stride) {
    int64_t lo = 0, hi = m;
    while (lo < hi) {
      const int64_t mid = lo + ((hi - lo) >> 1);
      if ((int64_t)keys[mid] < w)
        lo = mid + 1;
      else
        hi = mid;
    }
    roff[w] = lo;
  }
}

// One thread per bitmap word: every set bit w (a counter changed in the
// previous pass) becomes ceil(rdeg(w)/PUSH_CHUNK) items (at least one with
// OWN, whose first item also carries w's own write-back).  Slots are
// reserved with one atomic per wavefront.
template <bool OWN = false>
__device__ __forceinline__ uint32_t push_item_count(const int64_t* roff, int64_t w) {
  const uint32_t k = (uint32_t)((roff[w + 1] - roff[w] + PUSH_CHUNK - 1) / PUSH_CHUNK);
  return OWN && k == 0u ? 1u : k;
}

template <bool OWN = false>
__device__ __forceinline__ void push_items_body(const uint64_t* mod_prev, int64_t n_words, int64_t n,
                                                const int64_t* roff, uint2* items, unsigned long long* count) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t word = i < n_words ? mod_prev[i] : 0ull;
  uint32_t mine = 0;
  for (uint64_t bits = word; bits; bits &= bits - 1ull) {
    const int64_t w = i * 64 + __builtin_ctzll(bits);
    if (w < n) mine += push_item_count<OWN>(roff, w);
  }
  uint32_t incl = mine;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(incl, o);
    if (lane >= o) incl += t;
  }
  const uint32_t total = __shfl(incl, 63);
  unsigned long long base = 0;
  if (lane == 63 && total) base = atomicAdd(count, (unsigned long long)total);
  base = __shfl(base, 63);
  unsigned long long pos = base + incl - mine;
  for (uint64_t bits = word; bits; bits &= bits - 1ull) {
    const int64_t w = i * 64 + __builtin_ctzll(bits);
    if (w >= n) continue;
    const uint32_t k = push_item_count<OWN>(roff, w);
    for (uint32_t c = 0; c < k; ++c) items[pos++] = make_uint2((uint32_t)w, c);
  }
}

// Grid-stride over the items: one wavefront stamps act[v] = epoch for the
// (at most PUSH_CHUNK) predecessors of one item.
__device__ __forceinline__ void push_apply_body(const uint2* items, const unsigned long long* count,
                                                const int64_t* roff, const int32_t* ridx, int32_t* act,
                                                int32_t epoch) {
  const int lane = threadIdx.x & 63;
  const int64_t total = (int64_t)*count;
  const int64_t nw = (int64_t)gridDim.x * (blockDim.x / 64);
  for (int64_t it = (int64_t)blockIdx.x * (blockDim.x / 64) + (threadIdx.x >> 6); it < total; it += nw) {
    const uint2 item = items[it];
    const int64_t e0 = roff[item.x] + (int64_t)item.y * PUSH_CHUNK;
    const int64_t end = roff[item.x + 1];
    const int64_t e1 = e0 + PUSH_CHUNK < end ? e0 + PUSH_CHUNK : end;
    for (int64_t e = e0 + lane; e < e1; e += 64) act[ridx[e]] = epoch;
  }
}

__global__ void k_push_items(const uint64_t* mod_prev, int64_t n_words, int64_t n, const int64_t* roff,
                             uint2* items, unsigned long long* count) {
  push_items_body(mod_prev, n_words, n, roff, items, count);
}

__global__ void k_push_apply(const uint2* items, const unsigned long long* count, const int64_t* roff,
                             const int32_t* ridx, int32_t* act, int32_t epoch) {
  push_apply_body(items, count, roff, ridx, act, epoch);
}

// Device-driven forms: no-ops unless the pass is sparse.
__global__ void k_push_items_d(PassArgs A0, uint2* items, unsigned long long* count) {
  const PassArgs A = resolve(A0);
  if (A.mode != MODE_SPARSE) return;
  push_items_body(A.mod_prev, A.n_blocks, A.n, A.roff, items, count);
}

__global__ void k_push_apply_d(PassArgs A0, const uint2* items, const unsigned long long* count) {
  const PassArgs A = resolve(A0);
  if (A.mode != MODE_SPARSE) return;
  push_apply_body(items, count, A.roff, A.ridx, const_cast<int32_t*>(A0.act), A.epoch);
}

// --- sparse passes from pair lists (single-graph contexts) -------------------
//
// A row can change in pass t only through a successor whose counter changed
// in pass t-1, and must be rewritten if its own counter changed then.  Rather
// than have every row with such a successor scan all its arcs and test each
// successor's change bit, the pass lists exactly the pairs (v, u) with u
// changed (u's in-arcs, from the reverse CSR) plus (u, -1) for every changed
// u, sorts them by v, and runs each row over its own run of changed
// successors.

// One thread per bitmap word, as push_items_body with OWN, and also the
// position of each item's pairs: a changed u owns rdeg(u) + 1 consecutive
// pairs (its in-arcs in chunks of PUSH_CHUNK, its own entry after the first
// chunk), reserved with one atomic per wavefront.
__global__ void k_pair_items(const uint64_t* mod_prev, int64_t n_words, int64_t n, const int64_t* roff,
                             uint2* items, uint32_t* ppos, unsigned long long* count, unsigned long long* npairs) {
  const int lane = threadIdx.x & 63;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t word = i < n_words ? mod_prev[i] : 0ull;
  uint32_t mine = 0;
  unsigned long long mine_p = 0;
  for (uint64_t bits = word; bits; bits &= bits - 1ull) {
    const int64_t w = i * 64 + __builtin_ctzll(bits);
    if (w >= n) continue;
    mine += push_item_count<true>(roff, w);
    mine_p += (unsigned long long)(roff[w + 1] - roff[w]) + 1ull;
  }
  uint32_t incl = mine;
  unsigned long long incl_p = mine_p;
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    const uint32_t t = __shfl_up(incl, o);
    const unsigned long long tp = __shfl_up(incl_p, o);
    if (lane >= o) {
      incl += t;
      incl_p += tp;
    }
  }
  const uint32_t total = __shfl(incl, 63);
  const unsigned long long total_p = __shfl(incl_p, 63);
  unsigned long long base = 0, base_p = 0;
  if (lane == 63 && total) {
    base = atomicAdd(count, (unsigned long long)total);
    base_p = atomicAdd(npairs, total_p);
  }
  base = __shfl(base, 63);
  base_p = __shfl(base_p, 63);
  unsigned long long pos = base + incl - mine;
  unsigned long long pp = base_p + incl_p - mine_p;
  for (uint64_t bits = word; bits; bits &= bits - 1ull) {
    const int64_t w = i * 64 + __builtin_ctzll(bits);
    if (w >= n) continue;
    const uint32_t k = push_item_count<true>(roff, w);
    for (uint32_t c = 0; c < k; ++c) {
      items[pos] = make_uint2((uint32_t)w, c);
      ppos[pos] = (uint32_t)(pp + (unsigned long long)c * PUSH_CHUNK + (c > 0u ? 1ull : 0ull));
      ++pos;
    }
    pp += (unsigned long long)(roff[w + 1] - roff[w]) + 1ull;
  }
}

// One team of PAIR_TEAM lanes per push item (u, c): the pairs of u's in-arcs
// c*PUSH_CHUNK .. at the item's position and, in u's first item, (u, -1)
// after them (most changed nodes have few in-arcs, so a wavefront serves
// several items at once).  Writes stop at cap (the host compares the reserved
// total with its plan).
constexpr int PAIR_TEAM = 8;

__global__ void k_pair_apply(const uint2* items, const uint32_t* ppos, const unsigned long long* count,
                             const int64_t* roff, const int32_t* ridx, uint32_t* keys, int32_t* vals, int64_t cap) {
  const int tl = threadIdx.x % PAIR_TEAM;
  const int64_t total = (int64_t)*count;
  const int64_t nt = (int64_t)gridDim.x * (blockDim.x / PAIR_TEAM);
  for (int64_t it = (int64_t)blockIdx.x * (blockDim.x / PAIR_TEAM) + threadIdx.x / PAIR_TEAM; it < total;
       it += nt) {
    const uint2 item = items[it];
    const int64_t e0 = roff[item.x] + (int64_t)item.y * PUSH_CHUNK;
    const int64_t left = roff[item.x + 1] - e0;
    const int64_t ne = left < 0 ? 0 : (left < PUSH_CHUNK ? left : PUSH_CHUNK);
    const int64_t base = ppos[it];
    for (int64_t i = tl; i < ne; i += PAIR_TEAM) {
      const int64_t at = base + i;
      if (at < cap) {
        keys[at] = (uint32_t)ridx[e0 + i];
        vals[at] = (int32_t)item.x;
      }
    }
    if (item.y == 0u && tl == 0 && base + ne < cap) {
      keys[base + ne] = item.x;
      vals[base + ne] = -1;
    }
  }
}

// Per run r < R: its items and partial slots; entries from R to total are
// cleared so that the scans over `total` entries see zeros there.
__global__ void k_run_parts(const int32_t* num_runs, int64_t total, uint32_t* cnt, uint32_t* ni, uint32_t* mp) {
  const int64_t R = *num_runs;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < total; r += stride) {
    uint32_t k = 0;
    if (r < R)
      k = (cnt[r] + RUN_CHUNK - 1) / RUN_CHUNK;
    else
      cnt[r] = 0u;
    ni[r] = k;
    mp[r] = k > 1u ? k : 0u;
  }
}

// Writes the items of every run, the list of multi-item runs and the item count.
__global__ void k_run_items(const int32_t* num_runs, const uint32_t* uniq, const uint32_t* cnt,
                            const uint32_t* rstart, const uint32_t* ni, const uint32_t* ioff, const uint32_t* pbase,
                            PairItem* items, uint32_t* multi, uint32_t* num_multi, uint32_t* num_items) {
  const int64_t R = *num_runs;
  const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (r == 0 && R == 0) *num_items = 0u;
  if (r >= R) return;
  const uint32_t k = ni[r];
  for (uint32_t j = 0; j < k; ++j) {
    PairItem it;
    it.start = (int64_t)rstart[r] + (int64_t)j * RUN_CHUNK;
    const uint32_t rest = cnt[r] - j * RUN_CHUNK;
    it.len = (int32_t)(rest < (uint32_t)RUN_CHUNK ? rest : (uint32_t)RUN_CHUNK);
    it.row = (int32_t)uniq[r];
    it.nparts = (int32_t)k;
    it.slot = k > 1u ? (int32_t)(pbase[r] + j) : -1;
    it.pad[0] = it.pad[1] = 0;
    items[ioff[r] + j] = it;
  }
  if (k > 1u) multi[atomicAdd(num_multi, 1u)] = ioff[r];
  if (r == R - 1) *num_items = ioff[r] + k;
}

// One lane group per item: gathers the item's changed successors; an item
// that is its row's whole run finishes the row, the others leave a partial
// counter for k_pair_merge.
template <int B, int FL>
__global__ HB_EXPAND_ATTR void k_pair_expand(PassArgs A, const int32_t* vals, const PairItem* items,
                                             const uint32_t* num_items, uint8_t* partial) {
  constexpr int P = 1 << B;
  constexpr int G = P / 16;
  constexpr int W = 64 / G;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int gl = lane % G;
  const int grp = lane / G;
  if (blockIdx.x == 0)
    for (int i = threadIdx.x; i < STAT_SLOTS * STAT_K; i += blockDim.x) A.stats_next[i] = 0ull;
  const int64_t wi = (int64_t)blockIdx.x * 4 + wave;
  const int64_t it = wi * W + grp;
  Counts c{};
  if (it < (int64_t)*num_items) {
    const PairItem pi = items[it];
    PassArgs L = A;
    L.idx = vals;
    const bool whole = pi.nparts == 1;
    RowPre pre;
    if (whole) pre = preload<B, FL>(A, pi.row, gl);
    bool got = false;
    const uint32_t g0 = c.gath;
    const uint4 acc = gather<B, true>(L, pi.start, pi.start + pi.len, 1, gl, pi.row, got, c);
    if (gl == 0) c.arcs += c.gath - g0;
    if (whole)
      (void)finish_row<B, false, FL>(A, pi.row, acc, got, pre, bit_of(A.mod_prev, pi.row), gl, grp, c);
    else
      *reinterpret_cast<uint4*>(partial + (size_t)pi.slot * P + (size_t)gl * 16) = acc;
  }
  flush_counts<FL>(A, c, wi, lane);
}

// One wavefront per multi-item run: folds its partial counters into the row
// and finishes it like any other row.
template <int B, int FL>
__global__ __launch_bounds__(256) void k_pair_merge(PassArgs A, const PairItem* items, const uint32_t* multi,
                                                    const uint32_t* num_multi, const uint8_t* partial) {
  constexpr int P = 1 << B;
  constexpr int G = P / 16;
  constexpr int W = 64 / G;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int gl = lane % G;
  const int grp = lane / G;
  const int64_t h = (int64_t)blockIdx.x * 4 + wave;
  if (h >= (int64_t)*num_multi) return;
  const PairItem pi = items[multi[h]];
  RowPre pre;
  if (grp == 0) pre = preload<B, FL>(A, pi.row, gl);
  uint4 acc = zero4();
  for (int j = grp; j < pi.nparts; j += W)
    acc = bmax(acc, *reinterpret_cast<const uint4*>(partial + (size_t)(pi.slot + j) * P + (size_t)gl * 16));
#pragma unroll
  for (int o = G; o < 64; o <<= 1) acc = bmax(acc, shfl_xor4(acc, o));
  Counts c{};
  if (grp == 0) (void)finish_row<B, false, FL>(A, pi.row, acc, true, pre, bit_of(A.mod_prev, pi.row), gl, 0, c);
  flush_counts<FL>(A, c, h, lane);
}

// --- end-of-pass bookkeeping of multi-graph contexts ------------------------

// One wavefront per graph: a started, unconverged graph none of whose
// counters changed in this pass has converged after epoch - t0 passes.
__global__ void k_graph_done(PassArgs A0) {
  const PassArgs A = resolve(A0);
  const int lane = threadIdx.x & 63;
  const int64_t g = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  if (g >= A0.n_graphs) return;
  GraphDev* gd = A0.graphs + g;
  if (!gd->active || gd->done || A.epoch - 1 < gd->t0) return;
  const int64_t w0 = gd->node_base >> 6;
  const int64_t w1 = (gd->node_base + gd->n + 63) >> 6;
  uint64_t any = 0;
  for (int64_t w = w0 + lane; w < w1; w += 64) any |= A.mod_cur[w];
  const uint64_t changed = __ballot(any != 0ull);
  if (lane == 0 && changed == 0ull) {
    gd->done = 1;
    gd->passes = A.epoch - gd->t0;
    atomicAdd(&A0.ctl->n_done, 1);
    if (A0.ctl->batch) atomicAdd(&A0.ctl->rows_done, (unsigned long long)gd->n);
  }
}

// Mode of the next pass from the changed rows (chg) and their in-arcs
// (pairs) of the last pass, the same rule the host applies to single graphs.
__device__ __forceinline__ int32_t plan_mode(const PassCtl* c) {
  if (!c->frontier) return MODE_DENSE;
  const int64_t N = c->listed_rows > 0 ? c->listed_rows : 1;
  const int64_t M = c->arcs > 0 ? c->arcs : 1;
  const bool dense = c->has_reverse ? 100 * (int64_t)c->pairs >= (int64_t)c->dense_pct * M
                                    : 100 * (int64_t)c->chg >= (int64_t)c->dense_pct * N;
  if (dense) return MODE_DENSE;
  if (c->has_reverse && 100 * (int64_t)c->chg < (int64_t)c->sparse_pct * N) return MODE_SPARSE;
  return MODE_EDGE;
}

// Plans the next pass from this pass's counters (the same rule the host
// applies to single graphs), then advances the pass index and parity.
__global__ void k_pass_ctl(PassArgs A0) {
  const PassArgs A = resolve(A0);
  PassCtl* c = A0.ctl;
  const int lane = threadIdx.x;
  unsigned long long chg = 0, pairs = 0;
  for (int sl = lane; sl < STAT_SLOTS; sl += 64) {
    chg += A.stats[sl * STAT_K + 3];
    pairs += A.stats[sl * STAT_K + 7];
  }
#pragma unroll
  for (int o = 1; o < 64; o <<= 1) {
    chg += __shfl_xor(chg, o);
    pairs += __shfl_xor(pairs, o);
  }
  for (int i = lane; i < STAT_SLOTS * STAT_K; i += 64) A.stats_next[i] = 0ull;
  if (lane == 0) {
    c->chg = chg;
    c->pairs = pairs;
    c->mode = plan_mode(c);
    c->t += 1;
    c->parity ^= 1;
    c->work = 0ull;
  }
}

// Clears the change bitmap the next pass writes (the one this pass read).
__global__ void k_clear_next(PassArgs A0) {
  uint64_t* m = A0.modb[A0.ctl->parity ^ 1];
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < A0.n_blocks; i += stride) m[i] = 0ull;
}

// Multi-graph initialisation (see k_init_nodes): graph-local ids, per-graph
// seeds, padding rows empty.
__global__ void k_init_arena(int log2m, int64_t v0, int64_t v1, const int32_t* blk_graph, const GraphDev* graphs,
                             uint8_t* cur, uint8_t* nxt, double* S, double* H, double* E, const double* lc,
                             double alpha_pp) {
  const int64_t P = (int64_t)1 << log2m;
  const int64_t C = P / 16;
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (v1 - v0) * C) return;
  const int64_t v = v0 + i / C;
  const int64_t chunk = i % C;
  const GraphDev gd = graphs[blk_graph[v >> 6]];
  const int64_t local = v - gd.node_base;
  uint32_t w[4] = {0u, 0u, 0u, 0u};
  uint32_t r = 0;
  if (local < gd.n) {
    const uint64_t h = node_hash((uint64_t)local, gd.seed);
    const uint32_t j = (uint32_t)(h >> (64 - log2m));
    const uint64_t rest = h << log2m;
    r = rest == 0ull ? (uint32_t)(65 - log2m) : (uint32_t)__clzll((long long)rest) + 1u;
    if ((int64_t)(j >> 4) == chunk) w[(j >> 2) & 3u] = r << (8u * (j & 3u));
  }
  const uint4 val = make_uint4(w[0], w[1], w[2], w[3]);
  *reinterpret_cast<uint4*>(cur + v * P + chunk * 16) = val;
  *reinterpret_cast<uint4*>(nxt + v * P + chunk * 16) = val;
  if (chunk == 0) {
    S[v] = 0.0;
    H[v] = 0.0;
    if (local < gd.n) {
      double big = (double)(P - 1), small = 0.0;
      if (r <= 26u)
        big += pow2neg(r);
      else
        small += pow2neg(r);
      E[v] = estimate(big, small, (int)(P - 1), alpha_pp, (double)P, lc);
    } else {
      E[v] = 0.0;
    }
  }
}

__global__ void k_pack(const double* src, double* dst, int64_t n_arena, const int32_t* blk_graph,
                       const GraphDev* graphs) {
  const int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= n_arena) return;
  const GraphDev gd = graphs[blk_graph[v >> 6]];
  const int64_t local = v - gd.node_base;
  if (gd.active && local < gd.n) dst[gd.packed + local] = src[v];
}

__global__ void k_pack_u8(const uint8_t* src, uint8_t* dst, int64_t n_arena, int p, const int32_t* blk_graph,
                          const GraphDev* graphs) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t C = p / 16;
  if (i >= n_arena * C) return;
  const int64_t v = i / C, chunk = i % C;
  const GraphDev gd = graphs[blk_graph[v >> 6]];
  const int64_t local = v - gd.node_base;
  if (gd.active && local < gd.n)
    *reinterpret_cast<uint4*>(dst + (gd.packed + local) * p + chunk * 16) =
        *reinterpret_cast<const uint4*>(src + v * p + chunk * 16);
}

// --- serving: admission and retirement of one graph in a live engine ------

// Moves a graph's CSR into its pool regions: offsets (int32 or int64, local)
// become arc_base + offset at node_base + v; indices, already copied to
// their arc region, get node_base added in place.
__global__ void k_rebase_csr(const void* off_l, int bits, int64_t n, int64_t m, int64_t node_base, int64_t arc_base,
                             int64_t* off, int32_t* idx) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t v = t0; v <= n; v += stride) {
    const int64_t o = bits == 64 ? static_cast<const int64_t*>(off_l)[v] : (int64_t) static_cast<const int32_t*>(off_l)[v];
    off[node_base + v] = arc_base + o;
  }
  for (int64_t e = t0; e < m; e += stride) idx[arc_base + e] += (int32_t)node_base;
}

// Puts a graph into slot `slot` so that the engine's next pass is its pass 0:
// t0 is the engine pass index at that point, the region's blocks map to the
// slot, and every node of the graph counts as changed in the previous pass
// (so any pass mode gathers all of its successors) and as unchanged so far in
// the next one.
__global__ void k_admit(PassCtl* ctl, GraphDev* graphs, int32_t slot, GraphDev val, int64_t m, int32_t* blk_graph,
                        uint64_t* mod0, uint64_t* mod1, int64_t b0, int64_t b1) {
  const int par = ctl->parity;
  uint64_t* prev = par ? mod1 : mod0;
  uint64_t* next = par ? mod0 : mod1;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t b = b0 + t0; b < b1; b += stride) {
    // the graph's own rows only (padding rows never count as changed)
    const int64_t real = val.node_base + val.n - b * 64;
    blk_graph[b] = slot;
    prev[b] = real >= 64 ? ~0ull : (real > 0 ? (1ull << real) - 1ull : 0ull);
    next[b] = 0ull;
  }
  if (t0 == 0) {
    val.t0 = ctl->t;
    val.done = 0;
    val.passes = 0;
    val.active = 1;
    graphs[slot] = val;
    ctl->chg += (unsigned long long)val.n;
    ctl->pairs += (unsigned long long)m;
  }
}

// One wavefront per 64-entry chunk of the light list: the graph all its rows
// belong to, or -1.
__global__ void k_chunk_graph(const int32_t* light, int64_t n_light, const int32_t* blk_graph, int32_t* chunk_graph) {
  const int lane = threadIdx.x & 63;
  const int64_t j = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int64_t i = j * 64 + lane;
  if (j * 64 >= n_light) return;
  const int32_t g = i < n_light ? blk_graph[light[i] >> 6] : -1;
  const int32_t g0 = __shfl(g, 0);
  const bool same = i >= n_light || g == g0;
  const bool all = __ballot(!same) == 0ull;
  if (lane == 0) chunk_graph[j] = all ? g0 : -1;
}

// New planning totals; the mode of the pass about to run is planned again
// with them (admissions since the last pass changed both its inputs).
__global__ void k_set_plan(PassCtl* ctl, int64_t listed_rows, int64_t arcs) {
  if (threadIdx.x == 0) {
    ctl->listed_rows = listed_rows;
    ctl->arcs = arcs;
    ctl->mode = plan_mode(ctl);
  }
}

__global__ void k_set_slot(GraphDev* graphs, int32_t slot, GraphDev val) {
  if (threadIdx.x == 0) graphs[slot] = val;
}

int grid_for(int64_t work, int per_block, int cap) {
  int64_t g = (work + per_block - 1) / per_block;
  if (g < 1) g = 1;
  if (g > cap) g = cap;
  return (int)g;
}

}  // namespace

hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s) {
  if (bytes == 0) return hipSuccess;
  const size_t n16 = bytes / 16;
  const size_t tail = bytes - n16 * 16;
  hipLaunchKernelGGL(k_fill_zero, dim3(grid_for((int64_t)n16, 256 * 8, 65536)), dim3(256), 0, s,
                     reinterpret_cast<uint4*>(p), n16, reinterpret_cast<uint8_t*>(p) + n16 * 16, tail);
  return hipGetLastError();
}

hipError_t launch_pred_masks(const int32_t* idx, int64_t count, uint32_t bit, uint32_t* mask, hipStream_t s) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pred_masks, dim3(grid_for(count, 256 * 4, 65536)), dim3(256), 0, s, idx, count, bit, mask);
  return hipGetLastError();
}

hipError_t launch_chunk_activity(const uint64_t* mod_prev, int64_t n_words, const uint32_t* mask,
                                 const int64_t* chunk_rows, int32_t n_chunks, uint32_t* act, hipStream_t s) {
  hipError_t e = launch_fill_zero(act, sizeof(uint32_t), s);
  if (e != hipSuccess || n_words == 0) return e;
  hipLaunchKernelGGL(k_chunk_activity, dim3(grid_for(n_words, 256, 8192)), dim3(256), 0, s, mod_prev, n_words, mask,
                     chunk_rows, n_chunks, act);
  return hipGetLastError();
}

hipError_t launch_decode_chunk(const uint32_t* boff, const uint8_t* bytes, int64_t n_arcs, int32_t* ids, hipStream_t s) {
  if (n_arcs == 0) return hipSuccess;
  const int64_t nb = (n_arcs + STREAM_BLOCK_ARCS - 1) / STREAM_BLOCK_ARCS;
  hipLaunchKernelGGL(k_decode_chunk, dim3((unsigned)((nb + 255) / 256)), dim3(256), 0, s, boff, bytes, n_arcs, nb, ids);
  return hipGetLastError();
}

hipError_t launch_init_nodes(int log2m, int64_t n, uint64_t seed, uint8_t* cur, uint8_t* nxt,
                             double* S, double* H, double* E, const double* lc, double alpha_pp,
                             hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int64_t threads = n * (((int64_t)1 << log2m) / 16);
  hipLaunchKernelGGL(k_init_nodes, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, log2m, n, seed,
                     cur, nxt, S, H, E, lc, alpha_pp);
  return hipGetLastError();
}

hipError_t launch_init_weighted(int log2m, int64_t n, uint64_t seed, const int32_t* w, uint8_t* cur, uint8_t* nxt,
                                double* S, double* H, double* D, double* E, const double* lc, double alpha_pp,
                                hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int64_t threads = n * (((int64_t)1 << log2m) / 16);
  hipLaunchKernelGGL(k_init_weighted, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, log2m, n, seed, w,
                     cur, nxt);
  hipLaunchKernelGGL(k_row_estimate, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, log2m, n, cur, S, H, D, E,
                     lc, alpha_pp);
  return hipGetLastError();
}

hipError_t launch_check_weights(const int32_t* w, int64_t n, int* bad, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_check_weights, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, w, n, bad);
  return hipGetLastError();
}

hipError_t launch_esum(const double* E, int64_t n, uint64_t* partial, int max_blocks, uint64_t* out, int* inexact,
                       hipStream_t s) {
  const int blocks = (int)grid_for(n, 256 * 8, max_blocks);
  Fix192* part = reinterpret_cast<Fix192*>(partial);
  hipLaunchKernelGGL(k_esum, dim3((unsigned)blocks), dim3(256), 0, s, E, n, part, inexact);
  hipLaunchKernelGGL(k_esum_final, dim3(1), dim3(256), 0, s, part, blocks, out, inexact);
  return hipGetLastError();
}

hipError_t launch_init_ensemble(int log2m, int seg_log, int64_t n, const uint64_t* seeds, uint8_t* cur, uint8_t* nxt,
                                double* S, double* H, double* E, const double* lc, double alpha_pp, hipStream_t s) {
  if (n == 0) return hipSuccess;
  const int64_t threads = n * ((((int64_t)1 << log2m) / 16) << seg_log);
  hipLaunchKernelGGL(k_init_ensemble, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, log2m, seg_log, n,
                     seeds, cur, nxt, S, H, E, lc, alpha_pp);
  return hipGetLastError();
}

hipError_t launch_ensemble_summary(int64_t n, int k, int which, const double* S, const double* H, const double* E,
                                   double* mean, double* sd, hipStream_t s) {
  if (n == 0) return hipSuccess;
  if (k < 1 || k > 64) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_ensemble_summary, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, k, which, S, H, E,
                     mean, sd);
  return hipGetLastError();
}

// Expand and merge kernels of one lane-group pass for flavour FL.
template <int FL>
hipError_t launch_lanes(int log2m, const PassArgs& a, hipStream_t s, hipEvent_t ev_mid) {
  const bool q = !(a.mode == MODE_FIRST || a.mode == MODE_DENSE) || a.qdense;
  const int64_t R = q && FL == FL_PLAIN ? batched_med_rows(log2m) : 1;  // med_rows_per_wave
  const int64_t grid = a.n_items + (a.n_medium + 4 * R - 1) / (4 * R) + (a.n_light + 255) / 256;
  if (grid > 0) {
    const dim3 g((unsigned)grid), t(256);
    switch (log2m * 2 + (q ? 1 : 0)) {
      case 8: hipLaunchKernelGGL((k_expand<4, FL>), g, t, 0, s, a); break;
      case 9: hipLaunchKernelGGL((k_expand_q<4, FL>), g, t, 0, s, a); break;
      case 10: hipLaunchKernelGGL((k_expand<5, FL>), g, t, 0, s, a); break;
      case 11: hipLaunchKernelGGL((k_expand_q<5, FL>), g, t, 0, s, a); break;
      case 12: hipLaunchKernelGGL((k_expand<6, FL>), g, t, 0, s, a); break;
      case 13: hipLaunchKernelGGL((k_expand_q<6, FL>), g, t, 0, s, a); break;
      case 14: hipLaunchKernelGGL((k_expand<7, FL>), g, t, 0, s, a); break;
      case 15: hipLaunchKernelGGL((k_expand_q<7, FL>), g, t, 0, s, a); break;
      case 16: hipLaunchKernelGGL((k_expand<8, FL>), g, t, 0, s, a); break;
      case 17: hipLaunchKernelGGL((k_expand_q<8, FL>), g, t, 0, s, a); break;
      default: return hipErrorInvalidValue;
    }
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (ev_mid) {
    e = hipEventRecord(ev_mid, s);
    if (e != hipSuccess) return e;
  }
  if (a.n_hrows > 0) {
    const unsigned mg = (unsigned)((a.n_hrows + 3) / 4);
    switch (log2m) {
      case 4: hipLaunchKernelGGL((k_merge<4, false, FL>), dim3(mg), dim3(256), 0, s, a); break;
      case 5: hipLaunchKernelGGL((k_merge<5, false, FL>), dim3(mg), dim3(256), 0, s, a); break;
      case 6: hipLaunchKernelGGL((k_merge<6, false, FL>), dim3(mg), dim3(256), 0, s, a); break;
      case 7: hipLaunchKernelGGL((k_merge<7, false, FL>), dim3(mg), dim3(256), 0, s, a); break;
      default: hipLaunchKernelGGL((k_merge<8, false, FL>), dim3(mg), dim3(256), 0, s, a); break;
    }
  }
  return hipGetLastError();
}

// First pass from node hashes: the codes kernel, then the plain merge of heavy
// rows.
template <int B>
void launch_codes_b(const PassArgs& a, hipStream_t s) {
  const int64_t grid = codes_items<B>(a.n_items, a.n_medium, a.n_light);
  if (grid > 0) hipLaunchKernelGGL(k_expand_codes<B>, dim3((unsigned)grid), dim3(256), 0, s, a);
}

hipError_t launch_codes(int log2m, const PassArgs& a, hipStream_t s, hipEvent_t ev_mid) {
  switch (log2m) {
    case 4: launch_codes_b<4>(a, s); break;
    case 5: launch_codes_b<5>(a, s); break;
    case 6: launch_codes_b<6>(a, s); break;
    case 7: launch_codes_b<7>(a, s); break;
    case 8: launch_codes_b<8>(a, s); break;
    default: return hipErrorInvalidValue;
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (ev_mid) {
    e = hipEventRecord(ev_mid, s);
    if (e != hipSuccess) return e;
  }
  if (a.n_hrows > 0) {
    const unsigned mg = (unsigned)((a.n_hrows + 3) / 4);
    switch (log2m) {
      case 4: hipLaunchKernelGGL((k_merge<4, false>), dim3(mg), dim3(256), 0, s, a); break;
      case 5: hipLaunchKernelGGL((k_merge<5, false>), dim3(mg), dim3(256), 0, s, a); break;
      case 6: hipLaunchKernelGGL((k_merge<6, false>), dim3(mg), dim3(256), 0, s, a); break;
      case 7: hipLaunchKernelGGL((k_merge<7, false>), dim3(mg), dim3(256), 0, s, a); break;
      default: hipLaunchKernelGGL((k_merge<8, false>), dim3(mg), dim3(256), 0, s, a); break;
    }
  }
  return hipGetLastError();
}

hipError_t launch_pass(int log2m, const PassArgs& a, hipStream_t s, hipEvent_t ev_mid) {
  if (a.n_blocks == 0) return hipSuccess;
  if (a.singletons && a.mode == MODE_FIRST && !a.D && log2m <= 8 && !(a.seg_lanes > 0 && a.seg_lanes < (1 << log2m) / 16))
    return launch_codes(log2m, a, s, ev_mid);
  if (log2m <= 8) {
    if (a.seg_lanes > 0 && a.seg_lanes < (1 << log2m) / 16) return launch_lanes<FL_ENS>(log2m, a, s, ev_mid);
    if (a.D) return launch_lanes<FL_DISC>(log2m, a, s, ev_mid);
    return launch_lanes<FL_PLAIN>(log2m, a, s, ev_mid);
  }
  if (a.D) return hipErrorInvalidValue;  // discounted sums need the lane-group kernels
  const size_t lds = (size_t)1 << log2m;
  if (lds > 32768) {
    const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(k_expand_wide),
                                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
  }
  hipLaunchKernelGGL(k_expand_wide, dim3((unsigned)a.n_blocks), dim3(256), lds, s, a, log2m);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (ev_mid) e = hipEventRecord(ev_mid, s);
  return e;
}

hipError_t launch_finalize(int64_t n, const double* S, const double* H, const double* E, double* clo,
                           double* lin, double* harm, double* core, hipStream_t s) {
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_finalize, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, n, S, H, E, clo, lin,
                     harm, core);
  return hipGetLastError();
}

hipError_t launch_widen_offsets(const int32_t* in, int64_t* out, int64_t count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_widen, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, in, out, count);
  return hipGetLastError();
}

hipError_t launch_validate(const int64_t* off, const int32_t* idx, int64_t n, int64_t m, int* bad,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_validate, dim3(grid_for(n + m + 1, 256, 16384)), dim3(256), 0, s, off, idx, n, m,
                     bad);
  return hipGetLastError();
}

hipError_t select_rows(const int64_t* off, int64_t n, int64_t lo, int64_t hi, int32_t* out, int* count, void* tmp,
                       size_t* tmp_bytes, hipStream_t s) {
  hipcub::CountingInputIterator<int32_t> rows(0);
  DegreeIn op{off, lo, hi};
  return hipcub::DeviceSelect::If(tmp, *tmp_bytes, rows, out, count, (int)n, op, s);
}

hipError_t launch_take_offsets(const int32_t* rows, int64_t count, const int64_t* off, int64_t* out, hipStream_t s) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(k_take_offsets, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, rows, count, off, out);
  return hipGetLastError();
}

hipError_t build_reverse(const int64_t* off, const int32_t* idx, int64_t n, int64_t m, int64_t* roff,
                         int32_t* ridx, hipStream_t s) {
  if (m == 0) return launch_fill_zero(roff, sizeof(int64_t) * (size_t)(n + 1), s);
  if (m > 0x7fffffffLL) return hipErrorInvalidValue;
  int32_t* rows = nullptr;
  int32_t* keys = nullptr;
  void* tmp = nullptr;
  size_t tmp_bytes = 0;
  int end_bit = 1;
  while (end_bit < 31 && ((int64_t)1 << end_bit) < n) ++end_bit;
  hipError_t e = hipMalloc(reinterpret_cast<void**>(&rows), sizeof(int32_t) * (size_t)m);
  if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void**>(&keys), sizeof(int32_t) * (size_t)m);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_arc_rows, dim3(grid_for(n, 4, 65536)), dim3(256), 0, s, off, n, rows);
    e = hipGetLastError();
  }
  if (e == hipSuccess)
    e = hipcub::DeviceRadixSort::SortPairs(nullptr, tmp_bytes, idx, keys, rows, ridx, (int)m, 0, end_bit, s);
  if (e == hipSuccess) e = hipMalloc(&tmp, tmp_bytes > 0 ? tmp_bytes : 1);
  if (e == hipSuccess)
    e = hipcub::DeviceRadixSort::SortPairs(tmp, tmp_bytes, idx, keys, rows, ridx, (int)m, 0, end_bit, s);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_lower_bound, dim3(grid_for(n + 1, 256, 65536)), dim3(256), 0, s, keys, m, n, roff);
    e = hipGetLastError();
  }
  const hipError_t e2 = hipStreamSynchronize(s);
  if (e == hipSuccess) e = e2;
  (void)hipFree(tmp);
  (void)hipFree(keys);
  (void)hipFree(rows);
  return e;
}

hipError_t launch_push(const uint64_t* mod_prev, int64_t n_words, int64_t n, const int64_t* roff,
                       const int32_t* ridx, uint2* items, unsigned long long* count, int32_t* act,
                       int32_t epoch, hipStream_t s) {
  if (n_words == 0) return hipSuccess;
  hipError_t e = launch_fill_zero(count, sizeof(unsigned long long), s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_push_items, dim3((unsigned)((n_words + 255) / 256)), dim3(256), 0, s, mod_prev, n_words,
                     n, roff, items, count);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_push_apply, dim3(4096), dim3(256), 0, s, items, count, roff, ridx, act, epoch);
  return hipGetLastError();
}

size_t pair_tmp_bytes(int64_t cap, int end_bit) {
  size_t a = 0, b = 0, c = 0;
  const int N = (int)cap;
  (void)hipcub::DeviceRadixSort::SortPairs(nullptr, a, (const uint32_t*)nullptr, (uint32_t*)nullptr,
                                           (const int32_t*)nullptr, (int32_t*)nullptr, N, 0, end_bit);
  (void)hipcub::DeviceRunLengthEncode::Encode(nullptr, b, (const uint32_t*)nullptr, (uint32_t*)nullptr,
                                              (uint32_t*)nullptr, (int32_t*)nullptr, N);
  (void)hipcub::DeviceScan::ExclusiveSum(nullptr, c, (const uint32_t*)nullptr, (uint32_t*)nullptr, N);
  return std::max(a, std::max(b, c));
}

hipError_t launch_pair_build(const PassArgs& a, const PairBufs& pb, int64_t total, uint2* items,
                             unsigned long long* count, hipStream_t s) {
  if (total <= 0 || total > pb.cap) return hipErrorInvalidValue;
  const int N = (int)total;
  size_t tb = pb.tmp_bytes;
  hipError_t e = launch_fill_zero(count, sizeof(unsigned long long), s);
  if (e == hipSuccess) e = launch_fill_zero(pb.npairs, sizeof(unsigned long long), s);
  if (e == hipSuccess) e = launch_fill_zero(pb.num_multi, sizeof(uint32_t), s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_pair_items, dim3((unsigned)((a.n_blocks + 255) / 256)), dim3(256), 0, s, a.mod_prev,
                     a.n_blocks, a.n, a.roff, items, pb.ppos, count, pb.npairs);
  hipLaunchKernelGGL(k_pair_apply, dim3(4096), dim3(256), 0, s, items, pb.ppos, count, a.roff, a.ridx, pb.keys[0],
                     pb.vals[0], pb.cap);
  e = hipGetLastError();
  if (e == hipSuccess)
    e = hipcub::DeviceRadixSort::SortPairs(pb.tmp, tb, pb.keys[0], pb.keys[1], pb.vals[0], pb.vals[1], N, 0,
                                           pb.end_bit, s);
  tb = pb.tmp_bytes;
  if (e == hipSuccess)
    e = hipcub::DeviceRunLengthEncode::Encode(pb.tmp, tb, pb.keys[1], pb.uniq, pb.cnt, pb.num_runs, N, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_run_parts, dim3(grid_for(total, 256, 16384)), dim3(256), 0, s, pb.num_runs, total, pb.cnt,
                     pb.ni, pb.mp);
  e = hipGetLastError();
  tb = pb.tmp_bytes;
  if (e == hipSuccess) e = hipcub::DeviceScan::ExclusiveSum(pb.tmp, tb, pb.cnt, pb.rstart, N, s);
  tb = pb.tmp_bytes;
  if (e == hipSuccess) e = hipcub::DeviceScan::ExclusiveSum(pb.tmp, tb, pb.ni, pb.ioff, N, s);
  tb = pb.tmp_bytes;
  if (e == hipSuccess) e = hipcub::DeviceScan::ExclusiveSum(pb.tmp, tb, pb.mp, pb.pbase, N, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_run_items, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, pb.num_runs, pb.uniq,
                     pb.cnt, pb.rstart, pb.ni, pb.ioff, pb.pbase, pb.items, pb.multi, pb.num_multi, pb.num_items);
  return hipGetLastError();
}

template <int B, int FL>
hipError_t pair_pass_b(const PassArgs& a, const PairBufs& pb, int64_t total, hipStream_t s, hipEvent_t ev_mid) {
  constexpr int W = 64 / ((1 << B) / 16);
  const int64_t items_up = total + total / RUN_CHUNK + 1;  // runs <= total, plus the extra items of long runs
  hipLaunchKernelGGL((k_pair_expand<B, FL>), dim3((unsigned)((items_up + 4 * W - 1) / (4 * W))), dim3(256), 0, s,
                     a, pb.vals[1], pb.items, pb.num_items, pb.partial);
  hipError_t e = hipGetLastError();
  if (e == hipSuccess && ev_mid) e = hipEventRecord(ev_mid, s);
  if (e != hipSuccess) return e;
  const int64_t multi_up = total / (RUN_CHUNK + 1) + 1;
  hipLaunchKernelGGL((k_pair_merge<B, FL>), dim3((unsigned)((multi_up + 3) / 4)), dim3(256), 0, s, a, pb.items,
                     pb.multi, pb.num_multi, pb.partial);
  return hipGetLastError();
}

template <int FL>
hipError_t pair_pass_fl(int log2m, const PassArgs& a, const PairBufs& pb, int64_t total, hipStream_t s,
                        hipEvent_t ev_mid) {
  switch (log2m) {
    case 4: return pair_pass_b<4, FL>(a, pb, total, s, ev_mid);
    case 5: return pair_pass_b<5, FL>(a, pb, total, s, ev_mid);
    case 6: return pair_pass_b<6, FL>(a, pb, total, s, ev_mid);
    case 7: return pair_pass_b<7, FL>(a, pb, total, s, ev_mid);
    case 8: return pair_pass_b<8, FL>(a, pb, total, s, ev_mid);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_pair_pass(int log2m, const PassArgs& a, const PairBufs& pb, int64_t total, hipStream_t s,
                            hipEvent_t ev_mid) {
  if (total <= 0 || total > pb.cap || log2m > 8) return hipErrorInvalidValue;
  if (a.seg_lanes > 0 && a.seg_lanes < (1 << log2m) / 16) return pair_pass_fl<FL_ENS>(log2m, a, pb, total, s, ev_mid);
  if (a.D) return pair_pass_fl<FL_DISC>(log2m, a, pb, total, s, ev_mid);
  return pair_pass_fl<FL_PLAIN>(log2m, a, pb, total, s, ev_mid);
}

hipError_t launch_init_arena(int log2m, int64_t v0, int64_t v1, const int32_t* blk_graph,
                             const GraphDev* graphs, uint8_t* cur, uint8_t* nxt, double* S, double* H,
                             double* E, const double* lc, double alpha_pp, hipStream_t s) {
  if (v1 <= v0) return hipSuccess;
  const int64_t threads = (v1 - v0) * (((int64_t)1 << log2m) / 16);
  hipLaunchKernelGGL(k_init_arena, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, log2m, v0, v1,
                     blk_graph, graphs, cur, nxt, S, H, E, lc, alpha_pp);
  return hipGetLastError();
}

template <int B>
hipError_t device_pass_b(const PassArgs& a, int persist_wgs, uint2* push_items, unsigned long long* push_count,
                         hipStream_t s) {
  hipError_t e = hipSuccess;
  if (a.roff && a.act && a.n_blocks > 0) {
    e = launch_fill_zero(push_count, sizeof(unsigned long long), s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_push_items_d, dim3((unsigned)((a.n_blocks + 255) / 256)), dim3(256), 0, s, a, push_items,
                       push_count);
    hipLaunchKernelGGL(k_push_apply_d, dim3(4096), dim3(256), 0, s, a, push_items, push_count);
  }
  if (a.singletons) hipLaunchKernelGGL((k_expand_codes_p<B>), dim3(persist_wgs), dim3(256), 0, s, a);
  hipLaunchKernelGGL((k_expand_p<B, false>), dim3(persist_wgs), dim3(256), 0, s, a);
  hipLaunchKernelGGL((k_expand_p<B, true>), dim3(persist_wgs), dim3(256), 0, s, a);
  if (a.n_hrows > 0) hipLaunchKernelGGL((k_merge<B, true>), dim3((unsigned)((a.n_hrows + 3) / 4)), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_graph_done, dim3((unsigned)((a.n_graphs + 3) / 4)), dim3(256), 0, s, a);
  hipLaunchKernelGGL(k_pass_ctl, dim3(1), dim3(64), 0, s, a);
  hipLaunchKernelGGL(k_clear_next, dim3(grid_for(a.n_blocks, 256, 4096)), dim3(256), 0, s, a);
  e = hipGetLastError();
  return e;
}

hipError_t launch_device_pass(int log2m, const PassArgs& a, int persist_wgs, uint2* push_items,
                              unsigned long long* push_count, int64_t n_arena, hipStream_t s) {
  (void)n_arena;
  switch (log2m) {
    case 4: return device_pass_b<4>(a, persist_wgs, push_items, push_count, s);
    case 5: return device_pass_b<5>(a, persist_wgs, push_items, push_count, s);
    case 6: return device_pass_b<6>(a, persist_wgs, push_items, push_count, s);
    case 7: return device_pass_b<7>(a, persist_wgs, push_items, push_count, s);
    case 8: return device_pass_b<8>(a, persist_wgs, push_items, push_count, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_pack(const double* src, double* dst, int64_t n_arena, const int32_t* blk_graph,
                       const GraphDev* graphs, hipStream_t s) {
  if (n_arena == 0) return hipSuccess;
  hipLaunchKernelGGL(k_pack, dim3((unsigned)((n_arena + 255) / 256)), dim3(256), 0, s, src, dst, n_arena,
                     blk_graph, graphs);
  return hipGetLastError();
}

hipError_t launch_pack_u8(const uint8_t* src, uint8_t* dst, int64_t n_arena, int p, const int32_t* blk_graph,
                          const GraphDev* graphs, hipStream_t s) {
  if (n_arena == 0) return hipSuccess;
  const int64_t threads = n_arena * (p / 16);
  hipLaunchKernelGGL(k_pack_u8, dim3((unsigned)((threads + 255) / 256)), dim3(256), 0, s, src, dst, n_arena, p,
                     blk_graph, graphs);
  return hipGetLastError();
}

hipError_t launch_rebase_csr(const void* off_l, int bits, int64_t n, int64_t m, int64_t node_base, int64_t arc_base,
                             int64_t* off, int32_t* idx, hipStream_t s) {
  hipLaunchKernelGGL(k_rebase_csr, dim3(grid_for((n > m ? n : m) + 1, 256, 16384)), dim3(256), 0, s, off_l, bits, n,
                     m, node_base, arc_base, off, idx);
  return hipGetLastError();
}

hipError_t launch_admit(PassCtl* ctl, GraphDev* graphs, int32_t slot, const GraphDev& val, int64_t m,
                        int32_t* blk_graph, uint64_t* mod0, uint64_t* mod1, int64_t b0, int64_t b1, hipStream_t s) {
  hipLaunchKernelGGL(k_admit, dim3(grid_for(b1 - b0 + 1, 256, 4096)), dim3(256), 0, s, ctl, graphs, slot, val, m,
                     blk_graph, mod0, mod1, b0, b1);
  return hipGetLastError();
}

hipError_t launch_chunk_graph(const int32_t* light, int64_t n_light, const int32_t* blk_graph, int32_t* chunk_graph,
                              hipStream_t s) {
  const int64_t chunks = (n_light + 63) / 64;
  if (chunks == 0) return hipSuccess;
  hipLaunchKernelGGL(k_chunk_graph, dim3((unsigned)((chunks + 3) / 4)), dim3(256), 0, s, light, n_light, blk_graph,
                     chunk_graph);
  return hipGetLastError();
}

hipError_t launch_set_plan(PassCtl* ctl, int64_t listed_rows, int64_t arcs, hipStream_t s) {
  hipLaunchKernelGGL(k_set_plan, dim3(1), dim3(64), 0, s, ctl, listed_rows, arcs);
  return hipGetLastError();
}

hipError_t launch_set_slot(GraphDev* graphs, int32_t slot, const GraphDev& val, hipStream_t s) {
  hipLaunchKernelGGL(k_set_slot, dim3(1), dim3(64), 0, s, graphs, slot, val);
  return hipGetLastError();
}

}  // namespace hb
