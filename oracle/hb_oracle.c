/*
 * HyperBall oracle: a plain, slow, single-threaded CPU implementation.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or
 * load this file: only the tests, the smoke check and the CPU-baseline leg of
 * the benchmark use it.  It shares no code with the HIP library.
 *
 * What it computes (Boldi & Vigna, "In-Core Computation of Geometric
 * Centralities with HyperBall"):
 *   - HyperLogLog counters with p = 2^b registers (Sec. 4.1, Algorithm 1);
 *   - the ball recurrence B(x,0) = {x}, B(x,r+1) = {x} u U_{x->y} B(y,r)
 *     (Sec. 4.2), run with one counter per node, synchronous updates and
 *     termination when no counter changes (Algorithm 2);
 *   - the two per-node accumulators of Sec. 5, sum_t t*(|B_t|-|B_{t-1}|) and
 *     sum_t (|B_t|-|B_{t-1}|)/t, and the centralities of Sec. 3 built from
 *     them (closeness, Lin, harmonic).
 *
 * Readings of points the paper leaves open (each one is also listed in the
 * design notes of the repository):
 *   hash      h(x) = SplitMix64 finalizer applied to x + (seed+1)*0x9E3779B97F4A7C15
 *             (Steele, Lea, Flood 2014); the paper only asks for a fixed hash.
 *   index     the leftmost b bits of h (Sec. 4.1: h_b).
 *   rank      rho+ of the remaining 64-b bits, left-aligned; all-zero remainder
 *             gives 65-b (the paper's sequence is infinite).
 *   empty     registers start at 0 instead of -infinity (rho+ >= 1).
 *   alpha_p   Flajolet-Fusy-Gandouet-Meunier 2007 constants: 0.673 (p=16),
 *             0.697 (p=32), 0.709 (p=64), 0.7213/(1+1.079/p) otherwise.
 *   Z         the exact value of sum_j 2^-M[j], rounded once to double.
 *   small     the "different estimator for very small numbers" of Sec. 5.2 is
 *             linear counting: if the raw estimate is <= 5p/2 and V > 0
 *             registers are zero, the size is p*ln(p/V).
 *   distance  in pass t (counting from 0) the new counter estimates the ball of
 *             radius t+1, so the pass adds (t+1)*delta and delta/(t+1).
 *   finalize  S == 0 means "no distance mass": closeness 0, Lin 1.
 *
 * Floating point is IEEE double with no contraction (-ffp-contract=off).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef unsigned __int128 u128;

/* Sec. 4.1: a fixed hash from items to bit sequences. */
uint64_t hbo_hash(uint64_t x, uint64_t seed) {
  uint64_t z = x + (seed + 1u) * 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

/* Sec. 4.1: rho+(w) = number of leading zeroes of w plus one, where w is the
 * sequence of the 64-b bits of h that follow its leftmost b bits. */
int hbo_rho(uint64_t h, int b) {
  int width = 64 - b;
  int zeros = 0;
  for (int i = width - 1; i >= 0; --i) {
    if ((h >> i) & 1u) break;
    ++zeros;
  }
  return zeros + 1;
}

/* Adding an item to a counter (Algorithm 1): the leftmost b bits of its hash
 * select a register, which keeps the larger of its value and rho+ of the
 * other 64-b bits. */
void hbo_add(uint8_t* M, int b, uint64_t item, uint64_t seed) {
  uint64_t h = hbo_hash(item, seed);
  uint64_t i = h >> (64 - b);
  int r = hbo_rho(h, b);
  if (r > M[i]) M[i] = (uint8_t)r;
}

/* alpha_p from Flajolet et al. 2007, which Algorithm 1 defers to. */
double hbo_alpha(int b) {
  int p = 1 << b;
  if (p == 16) return 0.673;
  if (p == 32) return 0.697;
  if (p == 64) return 0.709;
  return 0.7213 / (1.0 + 1.079 / (double)p);
}

/* sum_{j<p} 2^-M[j], computed exactly as the integer sum_j 2^(K-M[j]) with
 * K = 65-b (the largest possible register value), then rounded once. */
double hbo_register_sum(const uint8_t* M, int b) {
  int p = 1 << b;
  int K = 65 - b;
  u128 z = 0;
  for (int j = 0; j < p; ++j) z += (u128)1 << (K - M[j]);
  return ldexp((double)z, -K);
}

/* Algorithm 1, function size, with the small-range estimator of Sec. 5.2. */
double hbo_size(const uint8_t* M, int b) {
  int p = 1 << b;
  double sum = hbo_register_sum(M, b);
  /* alpha_p p^2 Z with Z = 1/sum, evaluated as one division. */
  double E = ((hbo_alpha(b) * (double)p) * (double)p) / sum;
  int V = 0;
  for (int j = 0; j < p; ++j)
    if (M[j] == 0) ++V;
  if (E <= 2.5 * (double)p && V > 0) E = (double)p * log((double)p / (double)V);
  return E;
}

/* Register-wise maximum: the counter of a union of sets (Sec. 4.2). */
static void hbo_union(uint8_t* M, const uint8_t* N, int p) {
  for (int i = 0; i < p; ++i)
    if (N[i] > M[i]) M[i] = N[i];
}

/* Item of replica j of node x (Sec. 6 simulates an integer weight w(x) by
 * w(x) distinct replicas): x itself for j = 0, x + j * 2^32 for j > 0, which
 * no node id (< 2^31) and no other replica can equal. */
static uint64_t replica_item(int64_t x, int64_t j) { return (uint64_t)x + ((uint64_t)j << 32); }

/* Number of threads a pass may use: 1 in the plain build; the OpenMP build of
 * this same file (used only to time the all-core CPU baseline) runs the node
 * loop of hbo_pass over all its threads.  Nodes of one pass are independent
 * (each reads only the old counters and writes only its own entries), so both
 * builds give the same results. */
int hbo_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

/* Counters of radius 0 (Sec. 4.2: B(x, 0) = {x}): c (n*p bytes, node-major)
 * receives, for every node x, the HyperLogLog counter of x alone, or of its
 * w(x) replicas when weights are given (Sec. 6). */
void hbo_init_counters(int64_t n, int b, uint64_t seed, const int32_t* weights, uint8_t* c) {
  int p = 1 << b;
  memset(c, 0, (size_t)n * (size_t)p);
  for (int64_t v = 0; v < n; ++v) {
    const int64_t w = weights ? weights[v] : 1;
    for (int64_t j = 0; j < w; ++j) hbo_add(c + (size_t)v * p, b, replica_item(v, j), seed);
  }
}

/*
 * Pass t of the computation (Sec. 4.2 and Algorithm 2), restricted to the
 * nodes in [v_begin, v_end): the counter of radius t+1 of v is the union of
 * v's own counter of radius t with those of its successors, because
 * B(v, t+1) = B(v, t) u U_{v->w} B(w, t).  Old counters are read from c, new
 * ones written to next (never the same array: the update is synchronous).
 * With delta = |B(v,t+1)| - |B(v,t)| as estimated by the two counters, the
 * Sec. 5 accumulators receive S[v] += (t+1)*delta and H[v] += delta/(t+1),
 * and, with a discount (Sec. 7), D[v] += f*delta.  lastmod (nullable)
 * receives t+1 for every node whose registers changed.  Returns the number
 * of such nodes.
 */
int64_t hbo_pass(const int64_t* offsets, const int32_t* indices, int b, int t, const uint8_t* c, uint8_t* next,
                 double* S, double* H, double f, double* D, int32_t* lastmod, int64_t v_begin, int64_t v_end) {
  const int p = 1 << b;
  const double d = (double)(t + 1);
  int64_t changed = 0;
#ifdef _OPENMP
#pragma omp parallel for schedule(dynamic, 4096) reduction(+ : changed)
#endif
  for (int64_t v = v_begin; v < v_end; ++v) {
    const uint8_t* old = c + (size_t)v * p;
    uint8_t* a = next + (size_t)v * p;
    memcpy(a, old, (size_t)p);
    for (int64_t e = offsets[v]; e < offsets[v + 1]; ++e) hbo_union(a, c + (size_t)indices[e] * p, p);
    double delta = hbo_size(a, b) - hbo_size(old, b);
    S[v] = S[v] + d * delta;
    H[v] = H[v] + delta / d;
    if (D) D[v] = D[v] + f * delta;
    if (memcmp(a, old, (size_t)p) != 0) {
      ++changed;
      if (lastmod) lastmod[v] = t + 1;
    }
  }
  return changed;
}

/* The whole computation (Algorithm 2 with the Sec. 5 accumulators): passes
 * t = 0, 1, ... until one leaves every counter unchanged (that pass is
 * counted) or max_passes passes have run (max_passes <= 0: no cap).
 *   weights  (nullable) w(x) >= 1: counters start as the HyperLogLog of the
 *            replicas (Sec. 6), so sizes and accumulators count weighted nodes;
 *   disc     (nullable) a discount table f(1..disc_len): pass t adds
 *            f(t+1) * delta to D[v] (Sec. 7), f(d) = f(disc_len) beyond it;
 *   etrace   (nullable) (trace_rows * n) doubles: row t receives the size
 *            estimate of every counter after t passes (row 0: before pass 0),
 *            for the rows the run reaches;
 *   lastmod  (nullable) n int32: the largest t+1 such that pass t changed the
 *            node's counter, 0 if no pass did.
 * Outputs regs (n*p bytes, node-major: the final counters), S, H, D, and
 * nmod[t] (counters changed by pass t; room for the cap, or n+2 entries when
 * uncapped) may each be NULL.  *passes receives the number of passes run.
 * Returns 0, or -1 on bad arguments / allocation failure. */
int hbo_run_full(int64_t n, const int64_t* offsets, const int32_t* indices, int b, uint64_t seed, int max_passes,
                 const int32_t* weights, const double* disc, int disc_len, uint8_t* regs, double* S, double* H,
                 double* D, double* etrace, int64_t trace_rows, int64_t* nmod, int32_t* lastmod, int* passes) {
  if (n < 0 || b < 4 || b > 16) return -1;
  if (disc && disc_len < 1) return -1;
  int p = 1 << b;
  size_t nn = (size_t)(n > 0 ? n : 1);
  size_t bytes = nn * (size_t)p;
  uint8_t* c = (uint8_t*)calloc(bytes, 1);
  uint8_t* next = (uint8_t*)calloc(bytes, 1);
  double* s = (double*)calloc(nn, sizeof(double));
  double* h = (double*)calloc(nn, sizeof(double));
  double* dsum = (double*)calloc(nn, sizeof(double));
  if (!c || !next || !s || !h || !dsum) {
    free(c); free(next); free(s); free(h); free(dsum);
    return -1;
  }
  hbo_init_counters(n, b, seed, weights, c);
  if (lastmod && n > 0) memset(lastmod, 0, (size_t)n * sizeof(int32_t));
  if (etrace && trace_rows > 0)
    for (int64_t v = 0; v < n; ++v) etrace[v] = hbo_size(c + (size_t)v * p, b);
  int t = 0;
  int64_t changed;
  do {
    const double f = disc ? disc[t + 1 <= disc_len ? t : disc_len - 1] : 0.0;
    changed = hbo_pass(offsets, indices, b, t, c, next, s, h, f, disc ? dsum : NULL, lastmod, 0, n);
    uint8_t* tmp = c; c = next; next = tmp; /* the new counters become the current ones */
    if (nmod) nmod[t] = changed;
    ++t;
    if (etrace && t < trace_rows)
      for (int64_t v = 0; v < n; ++v) etrace[(size_t)t * nn + v] = hbo_size(c + (size_t)v * p, b);
  } while (changed != 0 && (max_passes <= 0 || t < max_passes));
  if (regs && n > 0) memcpy(regs, c, (size_t)n * p);
  if (S && n > 0) memcpy(S, s, (size_t)n * sizeof(double));
  if (H && n > 0) memcpy(H, h, (size_t)n * sizeof(double));
  if (D && n > 0) memcpy(D, dsum, (size_t)n * sizeof(double));
  if (passes) *passes = t;
  free(c); free(next); free(s); free(h); free(dsum);
  return 0;
}

int hbo_run_ext(int64_t n, const int64_t* offsets, const int32_t* indices, int b, uint64_t seed, int max_passes,
                const int32_t* weights, const double* disc, int disc_len, uint8_t* regs, double* S, double* H,
                double* D, double* etrace, int64_t trace_rows, int64_t* nmod, int* passes) {
  return hbo_run_full(n, offsets, indices, b, seed, max_passes, weights, disc, disc_len, regs, S, H, D, etrace,
                      trace_rows, nmod, NULL, passes);
}

int hbo_run(int64_t n, const int64_t* offsets, const int32_t* indices, int b, uint64_t seed,
            int max_passes, uint8_t* regs, double* S, double* H, int64_t* nmod, int* passes) {
  return hbo_run_ext(n, offsets, indices, b, seed, max_passes, NULL, NULL, 0, regs, S, H, NULL, NULL, 0, nmod,
                     passes);
}

/* The discount functions of Sec. 7 at distance d >= 1 (logarithms in base 2,
 * the paper's convention): kind 0 harmonic 1/d, 1 quadratic 1/d^2,
 * 2 logarithmic 1/log2(d+1), 3 constant 1.  NaN for an unknown kind. */
double hbo_discount(int kind, int d) {
  const double x = (double)d;
  switch (kind) {
    case 0: return 1.0 / x;
    case 1: return 1.0 / (x * x);
    case 2: return 1.0 / log2(x + 1.0);
    case 3: return 1.0;
    default: return NAN;
  }
}

void hbo_finalize(int64_t n, const uint8_t* regs, int b, const double* S, const double* H,
                  double* closeness, double* lin, double* harmonic, double* coreach) {
  int p = 1 << b;
  for (int64_t v = 0; v < n; ++v) {
    double size = hbo_size(regs + (size_t)v * p, b);
    if (coreach) coreach[v] = size;
    if (closeness) closeness[v] = (S[v] == 0.0) ? 0.0 : 1.0 / S[v];
    if (lin) lin[v] = (S[v] == 0.0) ? 1.0 : (size * size) / S[v];
    if (harmonic) harmonic[v] = H[v];
  }
}

/*
 * One node at a time, from the definition of the counters (Sec. 4.2): after
 * pass t the counter of x holds exactly the HyperLogLog state of the ball
 * B(x, t), because the union of counters is the counter of the union.  A
 * breadth-first visit from x along the CSR's arcs gives the balls, so this
 * reproduces x's registers, accumulators and change history without running
 * the whole graph.
 *
 * regs_at: if radius >= 0, receives the registers of B(x, radius); otherwise
 * those of the whole reachable set.  S, H: accumulators of x after the run.
 * last_change: the largest t+1 such that pass t changed x's counter (0 if no
 * pass does).  ecc: the eccentricity of x (largest finite distance).
 * With weights, the balls hold the replicas of their nodes; weights and disc
 * are as in hbo_run_full (nullable), and D receives the discounted sum.
 * Returns 0, or -1 on bad arguments / allocation failure.
 */
int hbo_node_ext(int64_t n, const int64_t* offsets, const int32_t* indices, int b, uint64_t seed, int64_t x,
                 int radius, const int32_t* weights, const double* disc, int disc_len, uint8_t* regs_at, double* S,
                 double* H, double* D, int* last_change, int* ecc) {
  if (x < 0 || x >= n || b < 4 || b > 16) return -1;
  if (disc && disc_len < 1) return -1;
  int p = 1 << b;
  uint8_t* seen = (uint8_t*)calloc((size_t)n, 1);
  int32_t* queue = (int32_t*)malloc((size_t)n * sizeof(int32_t));
  uint8_t* cur = (uint8_t*)calloc((size_t)p, 1);
  uint8_t* nxt = (uint8_t*)calloc((size_t)p, 1);
  if (!seen || !queue || !cur || !nxt) {
    free(seen); free(queue); free(cur); free(nxt);
    return -1;
  }
  double s = 0.0, h = 0.0, dsum = 0.0;
  int last = 0;
  /* B(x, 0) = {x}. */
  {
    const int64_t w = weights ? weights[x] : 1;
    for (int64_t j = 0; j < w; ++j) hbo_add(cur, b, replica_item(x, j), seed);
  }
  seen[x] = 1;
  queue[0] = (int32_t)x;
  int64_t layer_begin = 0, layer_end = 1, tail = 1;
  if (regs_at && radius == 0) memcpy(regs_at, cur, (size_t)p);
  int t = 0;
  for (;;) {
    /* Layer t+1: unseen successors of layer t. */
    for (int64_t q = layer_begin; q < layer_end; ++q) {
      int32_t u = queue[q];
      for (int64_t e = offsets[u]; e < offsets[u + 1]; ++e) {
        int32_t w = indices[e];
        if (!seen[w]) {
          seen[w] = 1;
          queue[tail++] = w;
        }
      }
    }
    if (tail == layer_end) break; /* the ball stops growing: no later pass changes x */
    memcpy(nxt, cur, (size_t)p);
    for (int64_t q = layer_end; q < tail; ++q) {
      const int64_t y = queue[q];
      const int64_t w = weights ? weights[y] : 1;
      for (int64_t j = 0; j < w; ++j) hbo_add(nxt, b, replica_item(y, j), seed);
    }
    double delta = hbo_size(nxt, b) - hbo_size(cur, b);
    double d = (double)(t + 1);
    s = s + d * delta;
    h = h + delta / d;
    if (disc) dsum = dsum + disc[t + 1 <= disc_len ? t : disc_len - 1] * delta;
    if (memcmp(nxt, cur, (size_t)p) != 0) last = t + 1;
    memcpy(cur, nxt, (size_t)p);
    layer_begin = layer_end;
    layer_end = tail;
    ++t;
    if (regs_at && radius == t) memcpy(regs_at, cur, (size_t)p);
  }
  if (regs_at && (radius < 0 || radius > t)) memcpy(regs_at, cur, (size_t)p);
  if (S) *S = s;
  if (H) *H = h;
  if (D) *D = dsum;
  if (last_change) *last_change = last;
  if (ecc) *ecc = t;
  free(seen); free(queue); free(cur); free(nxt);
  return 0;
}

int hbo_node(int64_t n, const int64_t* offsets, const int32_t* indices, int b, uint64_t seed,
             int64_t x, int radius, uint8_t* regs_at, double* S, double* H, int* last_change,
             int* ecc) {
  return hbo_node_ext(n, offsets, indices, b, seed, x, radius, NULL, NULL, 0, regs_at, S, H, NULL, last_change, ecc);
}
