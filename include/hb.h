/*
 * hb.h - C ABI of the MI355X HyperBall library (libhb.so).
 *
 * HyperBall (Boldi & Vigna, "In-Core Computation of Geometric Centralities
 * with HyperBall") keeps one HyperLogLog counter per node (Sec. 4.1,
 * Algorithm 1) and repeatedly replaces every counter by the register-wise
 * maximum of itself and the counters of its successors (the ball recurrence
 * of Sec. 4.2, Algorithm 2) until no counter changes.  While it runs it
 * accumulates, per node, sum_t t*(|B_t|-|B_{t-1}|) and
 * sum_t (|B_t|-|B_{t-1}|)/t (Sec. 5), from which closeness, Lin's and
 * harmonic centrality follow (Sec. 3).
 *
 * Conventions shared by every entry point:
 *   - Every function returns an hb_status; nothing throws across the ABI.
 *     On a non-OK status hb_last_error() describes the failure (per thread).
 *   - Balls grow along the arcs of the CSR that is passed in: row v lists the
 *     arcs v->w.  Centralities on incoming distances (Sec. 3, Sec. 5) need the
 *     transposed graph; undirected graphs pass a symmetric CSR.
 *   - Counters are p = 2^log2m byte-wide registers, node-major (register j of
 *     node v at byte v*p + j), 4 <= log2m <= 16.
 *   - Hash of node v: SplitMix64 finalizer of v + (seed+1)*0x9E3779B97F4A7C15;
 *     register index = leftmost log2m bits; value = rho+ of the remaining
 *     bits (65-log2m if they are all zero); empty registers hold 0.
 *   - Estimator: alpha_p p^2 / sum_j 2^-M[j] with the register sum exact and
 *     rounded once; linear counting p*ln(p/V) when that estimate is <= 5p/2
 *     and V > 0 registers are zero.  alpha_p = 0.673, 0.697, 0.709 for
 *     p = 16, 32, 64, else 0.7213/(1+1.079/p).
 *   - Pass t (from 0) turns counters of radius t into radius t+1 and adds
 *     (t+1)*delta to S[v] and delta/(t+1) to H[v], delta = E(new) - E(old).
 *   - All device work runs on the stream given at init (NULL: the default
 *     stream).  Calls that return host data synchronise that stream.
 *   - One context must not be used by two threads at once.
 */
#ifndef HB_H
#define HB_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HB_OK = 0,
  HB_EINVAL = -1,  /* bad argument: log2m range, malformed CSR, NULL pointer */
  HB_ENOMEM = -2,  /* device or host allocation failed, or over a memory budget */
  HB_EDEVICE = -3, /* a HIP call failed; the message names it */
  HB_ESTATE = -4   /* call not valid in the context's state (failed / freed / busy) */
} hb_status;

typedef struct hb_ctx hb_ctx;

/* A graph in compressed sparse rows.
 *   offsets: n+1 entries, offsets[0] = 0, nondecreasing, offsets[n] = m;
 *            int32 or int64 as offsets_bits says (32 or 64).
 *   indices: m int32 entries in [0, n); row v is indices[offsets[v]..offsets[v+1]).
 *   on_device = 0: host pointers, copied at hb_init and not retained.
 *   on_device = 1: device pointers, BORROWED: they must stay valid and
 *            unchanged until hb_free.  int32 offsets are widened into a
 *            library-owned copy; int64 offsets and indices are used in place. */
typedef struct {
  int64_t n;
  int64_t m;
  const void* offsets;
  int32_t offsets_bits;
  const int32_t* indices;
  int32_t on_device;
} hb_csr;

/* Tuning and behaviour switches; hb_default_options fills the defaults.
 *   frontier   1: skip work the previous pass makes unnecessary (exact: a
 *              successor whose counter did not change is already contained
 *              in the node's own counter, and a node none of whose successors
 *              changed cannot change); 0: every pass gathers every arc.
 *   light_max  rows with 1..light_max arcs are handled by one lane group.
 *   heavy_min  rows with at least this many arcs are split into chunks of
 *              `chunk` arcs reduced by separate workgroups; rows in between
 *              are handled by a whole wavefront.  (<= 0: library default.)
 *   validate   1: check the CSR (offsets monotone and bounded, indices in
 *              range) at init and fail with HB_EINVAL if it is malformed.
 *   timing     1: time every pass's kernels with HIP events (hb_pass_stats).
 *   dense_pct  with the frontier on, a pass after the first runs dense (every
 *              non-empty row gathers every successor, no per-arc test) when
 *              at least dense_pct percent of the arcs lead to a counter that
 *              changed in the previous pass (known exactly when push = 1,
 *              else estimated from the fraction of changed rows).  (< 0:
 *              default.)
 *   sparse_pct below that, the pass runs in edge mode (every non-empty row
 *              runs and gathers only its changed successors) when at least
 *              sparse_pct percent of the non-empty rows changed, and sparse
 *              (only rows with a changed successor run; needs push = 1)
 *              otherwise.  (< 0: default.)
 *   push       1: build the reverse CSR at init (m int32 + n+1 int64 more
 *              device memory) for sparse passes and exact pass planning.
 *   qdense     1: dense passes use the queued two-phase gather as well
 *              (tuning knob; results are identical).
 *   slice      1: keep a mask of changed 16-byte register slices per node
 *              (2n bytes) and let edge passes gather only changed slices.
 *   wgs_per_cu batched and served contexts: workgroups per compute unit of
 *              their persistent pass kernels (<= 0: 5).
 *   graph_passes batched contexts: passes per captured hipGraph replay in
 *              hb_run (<= 0: 4; convergence is read back once per replay).
 *   neighbourhood  single-graph contexts: 1 records the neighbourhood
 *              function N(t) at every pass (hb_neighbourhood).
 *   pairs      single-graph contexts with push = 1: 1 runs sparse passes
 *              from lists of the arcs into changed counters (sorted by
 *              source row) instead of activation stamps, when they fit the
 *              list capacity sized at init (about (m + n) / 16 pairs, all of
 *              them for m + n <= 2^16; about 80 bytes of device memory per
 *              pair); 0: activation stamps only.
 *   stream_graph  graphs whose arcs do not fit in device memory (Sec. 5.1
 *              keeps the graph out of core and only the counters in core):
 *              1 keeps the CSR in library-owned pinned host memory and
 *              streams it to the device in row chunks every pass (two
 *              staging buffers, uploads overlapping the previous chunk's
 *              kernels; passes after the first skip chunks none of whose
 *              rows has a changed successor or changed itself); 0 does so
 *              only when the CSR (8 (n+1) + 4 m bytes) exceeds graph_budget;
 *              -1 never.  Needs a host CSR (on_device = 0), a single-graph,
 *              single-seed context and log2m <= 8; push, pairs are ignored.
 *   graph_budget  device bytes for the graph (<= 0: no limit).  A streamed
 *              graph stages chunks of at most graph_budget / 2 bytes
 *              (<= 0: 256 MiB each); a row must fit one chunk.
 *   stream_compress  streamed graphs: 1 keeps the arcs in host memory
 *              compressed (each row's successors sorted, then blocks of 32
 *              arcs coded as the first id and the differences between
 *              consecutive ids, as 7-bit variable-length bytes or bit-packed
 *              at the block's widest difference, whichever is shorter) and
 *              decodes each uploaded chunk on the device: fewer bytes over
 *              the host link for the same results.  Each staging buffer then has a
 *              second buffer beside it for the chunk's coded form.  Ignored
 *              when the graph is not streamed. */
typedef struct {
  int32_t frontier;
  int32_t light_max;
  int32_t heavy_min;
  int32_t chunk;
  int32_t validate;
  int32_t timing;
  int32_t dense_pct;
  int32_t push;
  int32_t sparse_pct;
  int32_t qdense;
  int32_t slice;
  int32_t wgs_per_cu;
  int32_t graph_passes;
  int32_t neighbourhood;
  int32_t pairs;
  int32_t stream_graph;
  int64_t graph_budget;
  int32_t stream_compress;
} hb_options;

void hb_default_options(hb_options* opt);

/* Sec. 4.2 / Algorithm 2 set-up: allocates device state for g, feeds every
 * counter its own node (counter of radius 0), zeroes the accumulators.
 * log2m in [4, 16]; seed selects the hash.  opt may be NULL (defaults).
 * stream: a hipStream_t (e.g. torch.cuda.current_stream().cuda_stream) or NULL.
 * On success *out owns the context; release it with hb_free. */
hb_status hb_init(hb_ctx** out, const hb_csr* g, int32_t log2m, uint64_t seed,
                  const hb_options* opt, void* stream);

/* Restart the computation on the same graph with another hash seed, without
 * reallocating: counters back to radius 0, accumulators to zero, pass 0. */
hb_status hb_reset(hb_ctx* c, uint64_t seed);

/* One synchronous pass of Algorithm 2 (all new counters computed from the
 * old ones, then applied together), with the Sec. 5 accumulation fused in.
 * *n_modified (nullable) receives the number of counters that changed.  The
 * pass that changes nothing marks the context converged; later calls are
 * no-ops that report 0.  Synchronises the stream (one 8 KB readback). */
hb_status hb_iterate(hb_ctx* c, int64_t* n_modified);

/* Iterate until a pass changes no counter (that pass included) or until
 * max_passes passes have run in total (max_passes <= 0: no cap).
 * *passes (nullable) receives the number of passes run so far. */
hb_status hb_run(hb_ctx* c, int32_t max_passes, int32_t* passes);

/* Sec. 3 / Sec. 5 finalisation, per node v:
 *   coreach[v]   = size estimate of v's counter (coreachable set on G^T),
 *   closeness[v] = S == 0 ? 0 : 1/S,
 *   lin[v]       = S == 0 ? 1 : coreach^2 / S,
 *   harmonic[v]  = H,
 * where S = sum of distance-weighted increments and H = sum of reciprocal
 * ones.  Each output holds n doubles; any of them may be NULL.  dst_on_device
 * says whether the pointers are device (1) or host (0) memory.  Valid before
 * convergence too (partial sums); hb_stats tells whether it converged. */
hb_status hb_centralities(hb_ctx* c, double* closeness, double* lin, double* harmonic,
                          double* coreach, int32_t dst_on_device);

/* The current counters, n*p bytes, node-major. */
hb_status hb_get_registers(hb_ctx* c, uint8_t* dst, int32_t dst_on_device);

/* The raw accumulators S (sum of t*delta) and H (sum of delta/t), n doubles
 * each; either may be NULL. */
hb_status hb_get_accumulators(hb_ctx* c, double* S, double* H, int32_t dst_on_device);

typedef struct {
  int64_t n, m;
  int32_t log2m;
  int32_t passes;          /* passes run since init/reset */
  int32_t converged;       /* 1 once a pass changed no counter */
  int64_t last_modified;   /* counters changed by the last pass */
  int64_t heavy_rows;      /* rows split across workgroups */
  int64_t heavy_chunks;
  int64_t medium_rows;     /* rows handled by a whole wavefront */
  int64_t light_rows;      /* rows handled by one lane group */
  int32_t reverse_built;   /* 1 if the reverse CSR exists (push = 1) */
  double total_kernel_ms;  /* sum of timed pass kernels (timing = 1) */
  int32_t streamed;        /* 1 if the CSR lives in host memory and is streamed */
  int32_t chunks;          /* row chunks of a streamed graph */
  int64_t chunk_bytes;     /* capacity of each of its two staging buffers */
  int64_t host_graph_bytes; /* pinned host bytes holding a streamed graph */
  int32_t compressed;      /* 1 if its arcs are kept compressed */
} hb_stats_t;

hb_status hb_stats(hb_ctx* c, hb_stats_t* s);

/* Per-pass record (pass in [0, passes)).  Work counters are exact:
 *   arcs_scanned       successor ids read (every arc of every row the pass runs)
 *   counters_gathered  successors whose counter (or part of it) was read
 *   slices_gathered    16-byte counter slices read for them (0 in a first pass
 *                      of an unweighted single-seed context with p <= 256,
 *                      which recomputes each successor's singleton counter
 *                      from its hash)
 *   rows_loaded        rows whose own counter the pass read (in edge, slice and
 *                      sparse passes only rows with a changed successor or a
 *                      counter changed in the previous pass)
 *   rows_written       counters written into the next buffer
 *   rows_changed       counters that changed (= n_modified)
 *   slices_changed     16-byte slices that changed
 *   arcs_to_changed    arcs whose successor changed in this pass (what the
 *                      next pass gathers with edge skipping; needs push = 1)
 *   mode               0 first pass, 1 dense, 2 sparse, 3 edge with slice
 *                      masks, 4 edge
 *   path               0 counters gathered over the arcs, 1 first pass with
 *                      successor counters recomputed from node hashes, 2
 *                      sparse pass from pair lists (push_ms then includes
 *                      building and sorting them)
 *   push_ms / expand_ms / merge_ms: kernel times from HIP events (timing = 1);
 *                      in a streamed pass expand_ms spans all its chunks'
 *                      uploads and kernels, push_ms the chunk selection
 *   host_bytes         bytes streamed from host memory by the pass
 *   chunks_run         row chunks the pass streamed and ran (of hb_stats.chunks) */
typedef struct {
  int64_t arcs_scanned;
  int64_t counters_gathered;
  int64_t slices_gathered;
  int64_t rows_loaded;
  int64_t rows_written;
  int64_t rows_changed;
  int64_t slices_changed;
  int64_t arcs_to_changed;
  int32_t mode;
  double push_ms;
  double expand_ms;
  double merge_ms;
  int32_t path;
  int64_t host_bytes;
  int32_t chunks_run;
} hb_pass_info;

hb_status hb_pass_stats(hb_ctx* c, int32_t pass, hb_pass_info* info);

/* ---- Batched form: many independent graphs in one context -------------
 * hb_batch_init packs k host CSRs into one device arena (graph i keeps its
 * own node ids 0..n_i-1 for hashing, with seed seeds[i]) and runs every graph
 * exactly as hb_init/hb_run would run it alone: the same registers, pass
 * counts and floating-point results, bit for bit.  Passes are driven from the
 * device (mode, pass index and convergence live in device memory), run
 * persistent kernels over all unconverged graphs at once, and hb_run replays
 * them as a captured hipGraph with one small readback per replay.
 * log2m in [4, 8].  Graphs may be empty (n = 0), but not all of them
 * (HB_EINVAL).  With stream NULL the context creates its own stream.
 * On a batched context: hb_run runs until every graph converged (or the
 * engine pass cap); hb_iterate runs one pass over all graphs; outputs of
 * hb_centralities / hb_get_accumulators / hb_get_registers are packed: graph
 * 0's n_0 nodes, then graph 1's, ... (sum n_i entries); hb_reset restarts with
 * the same seeds (hb_batch_reset changes them); hb_pass_stats is kept for
 * passes run with hb_iterate (its work counts summed over all graphs; with
 * opt.timing, expand_ms is the whole device pass), not for hb_run. */
typedef struct {
  int64_t n;              /* nodes of the graph */
  int64_t packed_offset;  /* its first entry in packed outputs */
  int32_t passes;         /* its pass count (valid once converged) */
  int32_t converged;
} hb_graph_info;

hb_status hb_batch_init(hb_ctx** out, const hb_csr* graphs, int32_t k, int32_t log2m,
                        const uint64_t* seeds, const hb_options* opt, void* stream);
/* New seeds (k entries; NULL keeps them) and a restart from pass 0. */
hb_status hb_batch_reset(hb_ctx* c, const uint64_t* seeds);
hb_status hb_batch_graph(hb_ctx* c, int32_t g, hb_graph_info* info);
/* Per-graph pass counts (k entries; -1 for a graph not converged yet). */
hb_status hb_batch_passes(hb_ctx* c, int32_t* passes);

/* Autotuner for batched contexts.  Times complete batched runs (reset +
 * passes to convergence) on `sample` of the k graphs (<= 0: 256; graphs
 * sorted by size, evenly spaced) and picks, by coordinate descent from *opt:
 * light_max (rows up to this many arcs go to one lane group, longer ones to
 * a wavefront), heavy_min / chunk (rows from heavy_min arcs are cut into
 * workgroup tiles of chunk arcs), push (reverse CSR and sparse passes, or
 * edge passes only), wgs_per_cu, graph_passes, dense_pct, sparse_pct and
 * qdense.  The options never change results; the tuner checks
 * that every candidate gives the same per-graph pass counts.  *opt receives
 * the winner.  cache_path (nullable): a text file of earlier winners keyed
 * by a signature of the batch (log2m, sizes, degree histogram) and the
 * device; a hit returns at once, a new winner is appended. */
typedef struct {
  int32_t candidates;     /* configurations timed */
  int32_t from_cache;     /* 1: options came from the cache */
  int32_t sample_graphs;
  double start_ms;        /* one run over the sample with the starting options */
  double best_ms;         /* the same with the chosen options */
  double tune_s;          /* wall time of the call */
} hb_tune_report;

hb_status hb_batch_autotune(const hb_csr* graphs, int32_t k, int32_t log2m, const uint64_t* seeds,
                            int32_t sample, const char* cache_path, hb_options* opt,
                            hb_tune_report* report);

/* ---- Multi-seed ensembles ---------------------------------------------
 * Sec. 5 recommends running HyperBall several times and reporting the
 * empirical standard deviation of the results.  An ensemble context runs k
 * independent runs on one graph at once, run i with hash seed seeds[i]: the
 * row of node v holds the k counters (k * 2^log2m bytes; register j of run i
 * at byte (v*k + i) * 2^log2m + j), so each arc's successor id is read once
 * for all k runs, and every run gets its own estimator and accumulators.
 * Run i's registers, pass count and floating-point results equal those of
 * hb_init(seed = seeds[i]) + hb_run bit for bit.  k in {2, 4, 8, 16} and
 * k * 2^log2m <= 256.  On an ensemble context hb_iterate / hb_run run until
 * every seed converged (a row counts as changed if any of its counters did);
 * hb_centralities and hb_get_accumulators give n*k values, entry v*k + i;
 * hb_get_registers gives n*k*2^log2m bytes; hb_reset is refused. */
hb_status hb_ensemble_init(hb_ctx** out, const hb_csr* g, int32_t log2m, const uint64_t* seeds, int32_t k,
                           const hb_options* opt, void* stream);
/* Restart from pass 0 with new seeds (k entries; NULL keeps them). */
hb_status hb_ensemble_reset(hb_ctx* c, const uint64_t* seeds);
/* Pass count of each run (k entries; -1 for a run not converged yet). */
hb_status hb_ensemble_passes(hb_ctx* c, int32_t* passes);
/* Per node, over the k runs: mean and empirical standard deviation
 * (sqrt(sum_i (x_i - mean)^2 / (k - 1)), summed in run order) of one
 * centrality, which = 0 closeness, 1 Lin, 2 harmonic, 3 coreachable size.
 * mean and sd hold n doubles (either may be NULL). */
hb_status hb_ensemble_summary(hb_ctx* c, int32_t which, double* mean, double* sd, int32_t dst_on_device);

/* ---- Serving form: a request loop over resident engines ----------------
 * A server owns one multi-graph engine per log2m in [4, 8] (made on first
 * use) and a thread that runs them.  A request is one centrality query: a
 * host CSR, log2m and a hash seed; its result is exactly what hb_init +
 * hb_run + hb_centralities give for the same graph alone (same registers,
 * pass count and floating-point values, bit for bit), whatever else is
 * resident.  Requests are admitted in submission order while the counter
 * memory of the resident requests, sum of 2*n*2^log2m bytes, stays within
 * budget_bytes and the engine's node/arc pools and slots have room.  An
 * admitted request joins its engine at the next pass: its nodes start from
 * their singleton counters and count as changed, so that pass gathers all
 * their successors whatever the engine's pass mode, and its distances are
 * counted from that pass.  Every engine pass runs all resident requests of
 * its log2m at once (continuous batching); engines run on streams of their
 * own.  A request found converged is finalized, its outputs copied into the
 * caller's buffers, and its slot and memory are freed.
 *
 * Borrowing: the request's CSR arrays and output buffers must stay valid and
 * untouched from hb_serve_submit until the request reaches a final state.
 * Pinned host memory (hipHostMalloc) makes uploads and result copies
 * asynchronous; pageable memory works but stalls the serving thread on the
 * copy.  hb_serve_* calls may come from any thread. */
typedef struct hb_server hb_server;

typedef struct {
  int64_t budget_bytes;     /* admission cap on sum of 2*n*p (<= 0: 64 GiB) */
  int64_t max_nodes;        /* node pool per engine, padding included (<= 0: 2^25) */
  int64_t max_arcs;         /* arc pool per engine (<= 0: 2^29) */
  int32_t max_resident;     /* requests resident per engine (<= 0: 1024) */
  int32_t passes_per_tick;  /* engine passes enqueued per tick (<= 0: 1) */
  int32_t start_paused;     /* admit nothing until hb_serve_resume */
  hb_options opt;           /* row classes, frontier and mode thresholds, validate */
} hb_serve_config;

void hb_serve_default_config(hb_serve_config* cfg);

typedef struct {
  hb_csr graph;        /* host CSR (on_device must be 0); borrowed */
  int32_t log2m;       /* 4..8 */
  uint64_t seed;
  /* Host outputs, n entries each (registers: n*2^log2m bytes); any may be
   * NULL.  Written before the request becomes HB_REQ_DONE. */
  double* closeness;
  double* lin;
  double* harmonic;
  double* coreach;
  double* S;           /* sum_t t*(|B_t|-|B_{t-1}|) */
  double* H;           /* sum_t (|B_t|-|B_{t-1}|)/t */
  uint8_t* registers;
} hb_serve_request;

enum { HB_REQ_QUEUED = 0, HB_REQ_RUNNING = 1, HB_REQ_DONE = 2, HB_REQ_CANCELLED = 3, HB_REQ_FAILED = 4 };

typedef struct {
  int64_t id;
  int32_t state;       /* HB_REQ_* */
  int32_t passes;      /* pass count of the graph (DONE) */
  double t_submit;     /* seconds since hb_serve_start (steady clock) */
  double t_admit;      /* joined its engine (-1 while queued) */
  double t_done;       /* outputs written (-1 before) */
} hb_request_info;

typedef struct {
  int64_t submitted, admitted, completed, cancelled, failed;
  int64_t queued, resident;
  int64_t resident_bytes, peak_resident_bytes;  /* sum of 2*n*p */
  int64_t ticks, engine_passes;
  double busy_s;       /* wall time with at least one engine pass in flight */
  double elapsed_s;    /* since hb_serve_start */
} hb_serve_stats_t;

/* Starts the serving thread on the current device (cfg NULL: defaults). */
hb_status hb_serve_start(hb_server** out, const hb_serve_config* cfg);
/* Lets a server started with start_paused admit requests. */
hb_status hb_serve_resume(hb_server* s);
/* Enqueues a request and returns its id (> 0).  HB_EINVAL for a malformed
 * request (validated on the calling thread when opt.validate is set),
 * HB_ENOMEM for one that could never be admitted (over the budget or an
 * engine pool on its own), HB_ESTATE once the server failed or is stopping. */
hb_status hb_serve_submit(hb_server* s, const hb_serve_request* rq, int64_t* id);
/* Current state of a request, without waiting.  A final state (DONE,
 * CANCELLED, FAILED) is reported once; the id is forgotten afterwards. */
hb_status hb_serve_poll(hb_server* s, int64_t id, hb_request_info* info);
/* Waits up to timeout_s seconds (< 0: no limit) for a final state; returns
 * HB_ESTATE with info->state still QUEUED/RUNNING on a time-out and
 * HB_EDEVICE if the request failed. */
hb_status hb_serve_wait(hb_server* s, int64_t id, double timeout_s, hb_request_info* info);
/* Cancels a request that is still queued (HB_ESTATE once it was admitted). */
hb_status hb_serve_cancel(hb_server* s, int64_t id);
hb_status hb_serve_stats(hb_server* s, hb_serve_stats_t* st);
/* Finishes every submitted request (resuming a paused server), stops the
 * thread and frees everything; HB_EDEVICE if the server had failed. */
hb_status hb_serve_stop(hb_server* s);

/* ---- Weights, discounts and the neighbourhood function (single graphs) ----
 * Sec. 6: integer node weights w(x) >= 1 are simulated by w(x) replicas per
 * node: counter x starts as the HyperLogLog of the items x + j * 2^32,
 * j < w(x) (x itself for j = 0, so unit weights change nothing).  Sizes,
 * accumulators and centralities then count weighted nodes: S = sum_y w(y)
 * d(y,x), H = sum_y w(y)/d(y,x), coreachable size = sum of reachable
 * weights.  weights: n int32 (host or device, copied); NULL removes them.
 * The computation restarts from pass 0 with the current seed. */
hb_status hb_set_weights(hb_ctx* c, const int32_t* weights, int32_t on_device);

/* Sec. 7 discounted-gain centrality sum_{y != x, d(y,x) finite} w(y)
 * f(d(y,x)) for a discount table f(1..len) (host, copied; f(d) = f(len) for
 * d > len): pass t adds f(t+1) * delta to D[v].  NULL or len 0 turns it off.
 * Needs 2^log2m <= 256 and a single-graph, single-seed context.  The
 * computation restarts from pass 0. */
hb_status hb_set_discount(hb_ctx* c, const double* f, int32_t len);
/* The discount functions Sec. 7 names, f(1..len) into f (host, len >= 1),
 * logarithms in base 2 as everywhere in the paper:
 *   HB_DISCOUNT_HARMONIC     f(d) = 1/d (gives harmonic centrality),
 *   HB_DISCOUNT_QUADRATIC    f(d) = 1/d^2,
 *   HB_DISCOUNT_LOGARITHMIC  f(d) = 1/log2(d+1),
 *   HB_DISCOUNT_CONSTANT     f(d) = 1 (gives the coreachable-set size minus one).
 * HB_EINVAL for an unknown kind, a NULL output or len < 1.  Host arithmetic
 * only (no context, no device); pass the table to hb_set_discount. */
enum { HB_DISCOUNT_HARMONIC = 0, HB_DISCOUNT_QUADRATIC = 1, HB_DISCOUNT_LOGARITHMIC = 2, HB_DISCOUNT_CONSTANT = 3 };
hb_status hb_discount_table(int32_t kind, int32_t len, double* f);
/* The discounted sums (n doubles). */
hb_status hb_get_discounted(hb_ctx* c, double* D, int32_t dst_on_device);

/* Neighbourhood function (opt.neighbourhood = 1): N(t) = sum over nodes of
 * the size estimate after t passes, an estimate of the number of pairs
 * (x, y) with y in B(x, t) (weighted: sum of w(y)), for t = 0..passes.  Each
 * N(t) is the exact sum of the node estimates rounded once to double.
 * Copies min(cap, passes + 1) values; *len receives passes + 1. */
hb_status hb_neighbourhood(hb_ctx* c, double* N, int32_t cap, int32_t* len);

typedef struct {
  double pairs;              /* N(T) - N(0): pairs at distance >= 1 */
  double average_distance;   /* sum_{t>=1} t (N(t) - N(t-1)) / pairs */
  double effective_diameter; /* smallest t with N(t) >= alpha N(T), linearly interpolated */
} hb_distance_stats_t;

/* Distance statistics of a neighbourhood function N(0..len-1) (host
 * arithmetic, sums in t order; no context needed). */
hb_status hb_distance_stats(const double* N, int32_t len, double alpha, hb_distance_stats_t* out);

/* For callers that cannot allocate device memory (tight serving loops,
 * harnesses that forbid allocation): hb_init + hb_run + hb_centralities of
 * one graph in one call that allocates nothing.  All device state lives in
 * a fixed 64 MiB scratch array that the library holds on every GPU it runs
 * on until the process ends; a graph needs about n * (2 * 2^log2m + 29)
 * bytes of it (n up to about 1.1 M nodes at log2m 4, 120 k at log2m 8), and
 * a larger one is refused with HB_ENOMEM before any device work.
 *   g          device CSR (on_device must be 1), int32 or int64 offsets;
 *              read only.
 *   log2m      in [4, 8]; seed: the hash seed.
 *   closeness, lin, harmonic, coreach: device arrays of n doubles, each
 *              nullable; registers: device array of n * 2^log2m bytes
 *              (node-major final counters), nullable.
 *   passes     host int32 (nullable): the pass count, as hb_run reports it.
 *   stream     hipStream_t or NULL (default stream); the call synchronises it.
 * Results equal hb_init + hb_run + hb_centralities on the same graph, bit for
 * bit.  Every call on a GPU shares that GPU's scratch: calls that overlap on
 * one GPU (two threads, or two streams) race and give wrong results. */
hb_status hb_run_static(const hb_csr* g, int32_t log2m, uint64_t seed, double* closeness, double* lin,
                        double* harmonic, double* coreach, uint8_t* registers, int32_t* passes, void* stream);

/* Releases everything the context owns (never borrowed memory).  NULL-safe. */
void hb_free(hb_ctx* c);

/* Message for the last non-OK status returned on this thread. */
const char* hb_last_error(void);

/* Library ABI version (this header: 1). */
int32_t hb_version(void);

#ifdef __cplusplus
}
#endif

#endif /* HB_H */
