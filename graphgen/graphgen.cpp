// Seeded synthetic graph generators and CSR construction.
//
// These produce the inputs shared by the HyperBall library's tests and
// benchmarks and by the CPU oracle that checks it.  Nothing here computes
// anything of the HyperBall method itself: this file only draws random arcs
// and arranges them as compressed sparse rows.
//
// Randomness comes from the Philox-4x32-10 counter-based generator (Salmon,
// Moraes, Dror, Shaw, "Parallel random numbers: as easy as 1, 2, 3", SC 2011),
// so every draw is a pure function of (seed, counter) and the output does not
// depend on the number of threads.
//
// Generators:
//   * R-MAT (Chakrabarti, Zhan, Faloutsos 2004): each arc descends `scale`
//     levels of the adjacency matrix, picking a quadrant with probabilities
//     (a, b, c, d).
//   * Barabasi-Albert preferential attachment: a K_m seed clique, then every
//     new node attaches to m distinct existing nodes chosen with probability
//     proportional to their degree.
//   * Watts-Strogatz: a ring lattice where every node links to its k/2 nearest
//     neighbours on each side; each lattice edge is rewired with probability
//     beta to a uniform target, avoiding self-loops and duplicate edges.
#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstring>
#include <vector>
#include <omp.h>

namespace {

struct Ctr {
  uint32_t c[4];
};

inline void mulhilo32(uint32_t a, uint32_t b, uint32_t* hi, uint32_t* lo) {
  uint64_t p = (uint64_t)a * (uint64_t)b;
  *hi = (uint32_t)(p >> 32);
  *lo = (uint32_t)p;
}

// Philox-4x32 with 10 rounds.  Key = the 64-bit seed, counter = 128 bits.
inline Ctr philox(uint64_t seed, uint64_t c_lo, uint64_t c_hi) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t k0 = (uint32_t)seed, k1 = (uint32_t)(seed >> 32);
  uint32_t x0 = (uint32_t)c_lo, x1 = (uint32_t)(c_lo >> 32);
  uint32_t x2 = (uint32_t)c_hi, x3 = (uint32_t)(c_hi >> 32);
  for (int r = 0; r < 10; ++r) {
    uint32_t hi0, lo0, hi1, lo1;
    mulhilo32(M0, x0, &hi0, &lo0);
    mulhilo32(M1, x2, &hi1, &lo1);
    uint32_t y0 = hi1 ^ x1 ^ k0;
    uint32_t y1 = lo1;
    uint32_t y2 = hi0 ^ x3 ^ k1;
    uint32_t y3 = lo0;
    x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    k0 += W0; k1 += W1;
  }
  Ctr out;
  out.c[0] = x0; out.c[1] = x1; out.c[2] = x2; out.c[3] = x3;
  return out;
}

inline uint64_t philox_u64(uint64_t seed, uint64_t c_lo, uint64_t c_hi) {
  Ctr r = philox(seed, c_lo, c_hi);
  return ((uint64_t)r.c[1] << 32) | r.c[0];
}

// Uniform integer in [0, bound) by the multiply-shift reduction of a 64-bit
// draw (bias below 2^-32 for every bound used here).
inline uint64_t below(uint64_t draw, uint64_t bound) {
  return (uint64_t)(((unsigned __int128)draw * bound) >> 64);
}

// Probability -> 32-bit threshold so that a uniform u32 `u` falls below it
// with that probability (rounded to the nearest multiple of 2^-32).
inline uint64_t thresh32(double prob) {
  if (prob <= 0) return 0;
  if (prob >= 1) return 1ull << 32;
  return (uint64_t)(prob * 4294967296.0 + 0.5);
}

// Stream tags keep the generators' counter spaces apart.
const uint64_t TAG_RMAT = 0x524D4154ull << 32;
const uint64_t TAG_PERM = 0x5045524Dull << 32;
const uint64_t TAG_BA = 0x42415F5Full << 32;
const uint64_t TAG_WS = 0x57535F5Full << 32;

}  // namespace

extern "C" {

// R-MAT arc list: arc k (0 <= k < n_arcs) is a pure function of (seed, k).
// Level l (0 = most significant bit) uses one 32-bit uniform.  Self-loops and
// duplicates are kept; gg_csr removes them.
void gg_rmat_arcs(int scale, int64_t n_arcs, double a, double b, double c,
                  uint64_t seed, int32_t* src, int32_t* dst) {
  const uint64_t ta = thresh32(a), tab = thresh32(a + b), tabc = thresh32(a + b + c);
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < n_arcs; ++k) {
    uint32_t s = 0, d = 0;
    Ctr r{};
    for (int l = 0; l < scale; ++l) {
      if ((l & 3) == 0) r = philox(seed, (uint64_t)k, TAG_RMAT | (uint64_t)(l >> 2));
      uint64_t u = r.c[l & 3];
      uint32_t bit = 1u << (scale - 1 - l);
      if (u < ta) {
      } else if (u < tab) {
        d |= bit;
      } else if (u < tabc) {
        s |= bit;
      } else {
        s |= bit;
        d |= bit;
      }
    }
    src[k] = (int32_t)s;
    dst[k] = (int32_t)d;
  }
}

// Seeded uniform random permutation of [0, n) by Fisher-Yates; draw i is a
// pure function of (seed, i).
void gg_permutation(int64_t n, uint64_t seed, int32_t* perm) {
  for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
  for (int64_t i = n - 1; i > 0; --i) {
    uint64_t j = below(philox_u64(seed, (uint64_t)i, TAG_PERM), (uint64_t)(i + 1));
    std::swap(perm[i], perm[j]);
  }
}

// x[i] <- perm[x[i]] for an array of node ids.
void gg_relabel(int64_t m, const int32_t* perm, int32_t* x) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < m; ++i) x[i] = perm[x[i]];
}

// Compressed sparse rows from a pair list: row r lists cols[k] for every k
// with rows[k] == r, in increasing order.  With drop_self, pairs with
// rows[k] == cols[k] are skipped; with dedup, repeated pairs are kept once.
// offsets gets n+1 entries; cols_out must hold m entries.  Returns the number
// of stored entries, or -1 if a pair names a node outside [0, n).
int64_t gg_csr(int64_t n, int64_t m, const int32_t* rows, const int32_t* cols,
               int drop_self, int dedup, int64_t* offsets, int32_t* cols_out) {
  std::atomic<int64_t> bad{0};
  std::vector<std::atomic<int64_t>> cnt(n + 1);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i <= n; ++i) cnt[i].store(0, std::memory_order_relaxed);
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < m; ++k) {
    int32_t r = rows[k], c = cols[k];
    if (r < 0 || r >= n || c < 0 || c >= n) {
      bad.fetch_add(1, std::memory_order_relaxed);
      continue;
    }
    if (drop_self && r == c) continue;
    cnt[r].fetch_add(1, std::memory_order_relaxed);
  }
  if (bad.load()) return -1;
  // Exclusive scan of the raw row counts.
  std::vector<int64_t> start(n + 1);
  start[0] = 0;
  for (int64_t i = 0; i < n; ++i) start[i + 1] = start[i] + cnt[i].load(std::memory_order_relaxed);
  const int64_t raw = start[n];
  std::vector<int32_t> tmp(raw > 0 ? raw : 1);
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) cnt[i].store(start[i], std::memory_order_relaxed);
#pragma omp parallel for schedule(static)
  for (int64_t k = 0; k < m; ++k) {
    int32_t r = rows[k], c = cols[k];
    if (drop_self && r == c) continue;
    int64_t pos = cnt[r].fetch_add(1, std::memory_order_relaxed);
    tmp[pos] = c;
  }
  // Sort every row (and drop repeats), recording the kept length.
  std::vector<int64_t> keep(n);
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t i = 0; i < n; ++i) {
    int32_t* b0 = tmp.data() + start[i];
    int32_t* e0 = tmp.data() + start[i + 1];
    std::sort(b0, e0);
    keep[i] = dedup ? (int64_t)(std::unique(b0, e0) - b0) : (int64_t)(e0 - b0);
  }
  offsets[0] = 0;
  for (int64_t i = 0; i < n; ++i) offsets[i + 1] = offsets[i] + keep[i];
#pragma omp parallel for schedule(dynamic, 1024)
  for (int64_t i = 0; i < n; ++i)
    if (keep[i]) std::memcpy(cols_out + offsets[i], tmp.data() + start[i], (size_t)keep[i] * 4);
  return offsets[n];
}

// Barabasi-Albert edge list (each undirected edge once).  Nodes 0..m-1 form a
// clique; node v >= m then draws m distinct targets among 0..v-1, each target
// picked with probability proportional to its current degree (uniform choice
// over the list of edge endpoints).  Returns the number of edges written;
// src/dst must hold m*(m-1)/2 + m*(n-m) entries.
int64_t gg_ba_edges(int64_t n, int m, uint64_t seed, int32_t* src, int32_t* dst) {
  if (n <= 0 || m <= 0) return 0;
  if (n < m) m = (int)n;
  std::vector<int32_t> ends;
  ends.reserve((size_t)(2 * ((int64_t)m * (m - 1) / 2 + (int64_t)m * (n - m))) + 1);
  int64_t e = 0;
  for (int i = 0; i < m; ++i)
    for (int j = i + 1; j < m; ++j) {
      src[e] = i; dst[e] = j; ++e;
      ends.push_back(i); ends.push_back(j);
    }
  std::vector<int32_t> picked(m);
  uint64_t draw = 0;
  for (int64_t v = m; v < n; ++v) {
    int got = 0;
    while (got < m) {
      uint64_t u = philox_u64(seed, (uint64_t)v, TAG_BA | draw++);
      int32_t w;
      if (ends.empty())
        w = (int32_t)below(u, (uint64_t)v);
      else
        w = ends[below(u, ends.size())];
      bool dup = false;
      for (int q = 0; q < got; ++q) dup |= (picked[q] == w);
      if (!dup) picked[got++] = w;
    }
    for (int q = 0; q < m; ++q) {
      src[e] = (int32_t)v; dst[e] = picked[q]; ++e;
      ends.push_back((int32_t)v); ends.push_back(picked[q]);
    }
  }
  return e;
}

// Watts-Strogatz edge list (each undirected edge once): ring lattice with k/2
// neighbours per side; for j = 1..k/2 and every node u, the edge (u, u+j) is
// replaced with probability beta by (u, w), w uniform among nodes that are
// neither u nor already adjacent to u.  Returns the number of edges written;
// src/dst must hold n*(k/2) entries.
int64_t gg_ws_edges(int64_t n, int k, double beta, uint64_t seed, int32_t* src, int32_t* dst) {
  const int half = k / 2;
  if (n <= 0 || half <= 0) return 0;
  std::vector<std::vector<int32_t>> adj((size_t)n);
  auto has = [&](int32_t x, int32_t y) {
    for (int32_t z : adj[x])
      if (z == y) return true;
    return false;
  };
  auto add = [&](int32_t x, int32_t y) { adj[x].push_back(y); adj[y].push_back(x); };
  auto del = [&](int32_t x, int32_t y) {
    auto& ax = adj[x];
    ax.erase(std::find(ax.begin(), ax.end(), y));
    auto& ay = adj[y];
    ay.erase(std::find(ay.begin(), ay.end(), x));
  };
  for (int64_t u = 0; u < n; ++u)
    for (int j = 1; j <= half; ++j) {
      int32_t v = (int32_t)((u + j) % n);
      if (v != u && !has((int32_t)u, v)) add((int32_t)u, v);
    }
  const uint64_t tb = thresh32(beta);
  uint64_t draw = 0;
  for (int j = 1; j <= half; ++j)
    for (int64_t u = 0; u < n; ++u) {
      int32_t v = (int32_t)((u + j) % n);
      uint64_t r = philox_u64(seed, (uint64_t)u, TAG_WS | draw++);
      if ((r & 0xffffffffull) >= tb) continue;
      if ((int64_t)adj[u].size() >= n - 1) continue;  // u already adjacent to all
      if (!has((int32_t)u, v)) continue;
      int32_t w;
      do {
        w = (int32_t)below(philox_u64(seed, (uint64_t)u, TAG_WS | draw++), (uint64_t)n);
      } while (w == u || has((int32_t)u, w));
      del((int32_t)u, v);
      add((int32_t)u, w);
    }
  int64_t e = 0;
  for (int64_t u = 0; u < n; ++u)
    for (int32_t v : adj[u])
      if (v > u) { src[e] = (int32_t)u; dst[e] = v; ++e; }
  return e;
}

// Arc count of a symmetric batch graph: kind 0 = Barabasi-Albert with
// `param` edges per node, kind 1 = Watts-Strogatz with `param` neighbours.
// Both generators produce no duplicate edges and no self-loops.
int64_t gg_batch_arcs(int32_t kind, int64_t n, int param) {
  if (n <= 0) return 0;
  if (kind == 0) {
    const int64_t m = param < n ? param : n;
    return 2 * (m * (m - 1) / 2 + m * (n - m));
  }
  return n * (int64_t)(param / 2) * 2;
}

// Many symmetric graphs at once (OpenMP over graphs).  Graph i is written as
// a CSR at offsets_all + off_start[i] (n_i + 1 entries) and indices_all +
// idx_start[i] (gg_batch_arcs entries), rows sorted.  Returns 0, or the
// 1-based index of a graph whose arc count did not match.
int32_t gg_batch_build(int32_t k, const int32_t* kinds, const int64_t* ns, const uint64_t* seeds, int ba_m,
                       int ws_k, double ws_beta, const int64_t* off_start, const int64_t* idx_start,
                       int64_t* offsets_all, int32_t* indices_all) {
  int32_t bad = 0;
#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t i = 0; i < k; ++i) {
    const int64_t n = ns[i];
    const int param = kinds[i] == 0 ? ba_m : ws_k;
    const int64_t edges = gg_batch_arcs(kinds[i], n, param) / 2;
    std::vector<int32_t> src((size_t)(edges > 0 ? edges : 1)), dst((size_t)(edges > 0 ? edges : 1));
    const int64_t got = kinds[i] == 0 ? gg_ba_edges(n, ba_m, seeds[i], src.data(), dst.data())
                                      : gg_ws_edges(n, ws_k, ws_beta, seeds[i], src.data(), dst.data());
    int64_t* off = offsets_all + off_start[i];
    int32_t* idx = indices_all + idx_start[i];
    if (got != edges) {
#pragma omp critical
      bad = i + 1;
      continue;
    }
    std::vector<int64_t> cnt((size_t)n + 1, 0);
    for (int64_t e = 0; e < edges; ++e) {
      ++cnt[(size_t)src[e]];
      ++cnt[(size_t)dst[e]];
    }
    off[0] = 0;
    for (int64_t v = 0; v < n; ++v) off[v + 1] = off[v] + cnt[(size_t)v];
    for (int64_t v = 0; v < n; ++v) cnt[(size_t)v] = off[v];
    for (int64_t e = 0; e < edges; ++e) {
      idx[cnt[(size_t)src[e]]++] = dst[e];
      idx[cnt[(size_t)dst[e]]++] = src[e];
    }
    for (int64_t v = 0; v < n; ++v) std::sort(idx + off[v], idx + off[v + 1]);
  }
  return bad;
}

int gg_num_threads(void) { return omp_get_max_threads(); }

}  // extern "C"
