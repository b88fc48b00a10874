// Internal interface between the host side of libhb (hb_api.cpp) and its HIP
// kernels (hb_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hb {

// A row whose arcs are reduced by several workgroups: `nitems` consecutive
// chunk items starting at `item0` each write a partial counter that the merge
// kernel folds into the row.
struct HeavyRow {
  int64_t row;
  int64_t item0;
  int64_t nitems;
};

// One chunk of a heavy row: arcs [e0, e1).
struct HeavyItem {
  int64_t row;
  int64_t e0;
  int64_t e1;
};

// Number of slots the per-pass work counters are spread over (atomics to a
// single address would serialise); STAT_K counters per slot.
constexpr int STAT_SLOTS = 256;
// gathered successors, rows run, rows written, rows changed, arcs scanned,
// 16-byte slices gathered, 16-byte slices changed, arcs into changed rows
// (the number of successors the next pass would gather with edge skipping),
// and (OR, not a sum) the mask of ensemble seeds with a changed counter
constexpr int STAT_K = 9;
constexpr int STAT_SEEDS = 8;

// Reverse-CSR entries handled by one push item.
constexpr int PUSH_CHUNK = 2048;

// How a pass treats the previous pass's change bits.
enum PassMode : int32_t {
  MODE_FIRST = 0,   // pass 0: nothing changed before; every successor is gathered
  MODE_DENSE = 1,   // every listed row runs and gathers every successor
  MODE_SPARSE = 2,  // only rows with a changed successor (or a changed own
                    // counter) run, and they gather only changed successors
  MODE_SLICE = 3,   // every listed row runs and gathers only the 16-byte slices
                    // of its successors that changed in the previous pass
  MODE_EDGE = 4,    // every listed row runs and gathers only changed successors
};

// Per-graph state of a multi-graph context (batched or served graphs).
// Nodes node_base .. node_base+n-1 of the arena belong to the graph; the
// region is padded to a multiple of 64 with empty rows.
struct GraphDev {
  int64_t node_base;
  int64_t n;
  int64_t packed;     // first index of the graph in packed (unpadded) outputs
  uint64_t seed;
  int32_t t0;         // engine pass at which the graph's pass 0 runs
  int32_t done;       // 1 once one of its passes changed none of its counters
  int32_t passes;     // its pass count at convergence (the unchanged pass included)
  int32_t active;     // slot in use
};

// Device-resident pass control of a multi-graph context: every pass reads
// its mode, pass index and buffer parity here, and the bookkeeping kernels at
// the end of the pass write the next ones, so passes need no host round trip
// (and can be captured in a hipGraph).
struct PassCtl {
  int32_t t;                   // engine pass index
  int32_t mode;                // PassMode of the pass about to run
  int32_t parity;              // counter buffer holding the current counters
  int32_t n_done;              // graphs converged so far
  unsigned long long work;     // persistent work-queue cursor (tickets)
  // planning inputs (set by the host)
  int64_t listed_rows;         // non-empty rows of the resident graphs
  int64_t arcs;                // arcs of the resident graphs
  int32_t frontier, dense_pct, sparse_pct, has_reverse;
  int32_t n_graphs;
  int32_t pad;
  // changed rows and their in-arcs in the last pass, plus those of graphs
  // admitted since (every row of an admitted graph counts as changed)
  unsigned long long chg, pairs;
  // batched contexts: rows of the graphs converged so far (batch = 1 marks
  // such a context; served engines leave both 0)
  unsigned long long rows_done;
  int32_t batch;
  int32_t pad2;
};

// Everything one pass needs.  `cur` holds counters of radius t, `nxt`
// receives radius t+1.  mod_prev has bit v set if counter v changed in the
// previous pass; mod_cur (zeroed before the pass) receives this pass's bits.
struct PassArgs {
  const int64_t* off;
  const int32_t* idx;
  const uint8_t* cur;
  uint8_t* nxt;
  const uint64_t* mod_prev;
  uint64_t* mod_cur;
  const uint16_t* dmask_prev;        // changed 16-byte slices per node, previous pass
  uint16_t* dmask_cur;               // this pass (zeroed before the pass)
  double* S;
  double* H;
  double* E;
  const double* lc;                  // linear-counting table, entries 0..p
  const int32_t* light;              // rows with 1..light_max arcs, increasing
  const int32_t* medium;             // rows handled by a whole wavefront
  const HeavyItem* items;
  const HeavyRow* hrows;
  uint8_t* partial;                  // n_items * p bytes
  const int32_t* act;                // act[v] == epoch: v has a changed successor (sparse)
  const int64_t* roff;               // reverse CSR offsets (nullable): in-degrees for the stats
  const int32_t* ridx;               // reverse CSR indices (nullable)
  unsigned long long* stats;         // this pass: STAT_SLOTS * STAT_K
  unsigned long long* stats_next;    // zeroed by this pass for the next one
  double alpha_pp;                   // (alpha_p * p) * p
  double d;                          // t + 1
  int64_t n;
  int64_t n_blocks;                  // ceil(n / 64)
  int64_t n_light;
  int64_t n_medium;
  int64_t n_items;
  int64_t n_hrows;
  int32_t epoch;
  int32_t mode;                      // PassMode
  int32_t qdense;                    // dense passes use the queued gather too
  // Multi-seed ensembles: a row holds K = G / seg_lanes independent counters
  // (one per seed, seg_lanes * 16 bytes each) and E, S, H hold K values per
  // node.  0 means one counter per row.
  int32_t seg_lanes;
  // Discounted-gain accumulator (Sec. 7, nullable): D += disc_f * delta,
  // disc_f = f(t+1) for this pass.
  double* D;
  double disc_f;
  // First pass of an unweighted single-graph, single-seed context: nonzero
  // when every counter still holds only its own node's item, so a counter
  // can be recomputed from the node's hash with `seed`.
  int32_t singletons;
  uint64_t seed;
  // Multi-graph contexts (null otherwise): graph of each 64-node block, the
  // per-graph state, and the device pass control; with ctl set, cur/nxt,
  // mod_prev/mod_cur, mode, epoch and the stats halves are taken from ctl
  // (buffers cntb[], modb[], stats_base).
  const int32_t* blk_graph;
  // Batched contexts (nullable): graph of every 64-entry chunk of the light
  // list if all its rows belong to one graph, else -1 (lets a wavefront skip
  // a converged graph's chunk with one lookup).
  const int32_t* chunk_graph;
  GraphDev* graphs;
  PassCtl* ctl;
  uint8_t* cntb[2];
  uint64_t* modb[2];
  unsigned long long* stats_base;
  int32_t n_graphs;                  // graph slots (multi-graph contexts)
};

// Launchers (hb_kernels.hip).  All return the launch status.
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s);
// Singleton counters of nodes 0..n-1 in both buffers, S = H = 0, E their
// estimate.
hipError_t launch_init_nodes(int log2m, int64_t n, uint64_t seed, uint8_t* cur, uint8_t* nxt,
                             double* S, double* H, double* E, const double* lc, double alpha_pp,
                             hipStream_t s);
// Weighted initialisation (Sec. 6 replicas): counter v holds the HyperLogLog
// of items v + j * 2^32, j < w[v]; then E from the counters, S = H = 0, and
// D = 0 if D is set.
hipError_t launch_init_weighted(int log2m, int64_t n, uint64_t seed, const int32_t* w, uint8_t* cur, uint8_t* nxt,
                                double* S, double* H, double* D, double* E, const double* lc, double alpha_pp,
                                hipStream_t s);
// Sets *bad to 1 if some w[v] < 1.
hipError_t launch_check_weights(const int32_t* w, int64_t n, int* bad, hipStream_t s);
// Exact sum of E[0..n) as a 192-bit integer E * 2^52 (three words, low
// first) into out[0..2]; out[3] becomes 1 if an E is not a multiple of 2^-52
// (never for counter estimates).  partial holds 3 * max_blocks words of
// scratch; *inexact is a flag word that must be zero before the first sum
// (each sum leaves it zero).
hipError_t launch_esum(const double* E, int64_t n, uint64_t* partial, int max_blocks, uint64_t* out, int* inexact,
                       hipStream_t s);
// Ensemble initialisation: rows of K = 2^seg_log counters of p = 2^log2m
// registers, counter k of node v hashing v with seeds[k] (device array).
hipError_t launch_init_ensemble(int log2m, int seg_log, int64_t n, const uint64_t* seeds, uint8_t* cur, uint8_t* nxt,
                                double* S, double* H, double* E, const double* lc, double alpha_pp, hipStream_t s);
// Per node, the mean and empirical standard deviation over the K seeds of one
// centrality (0 closeness, 1 Lin, 2 harmonic, 3 coreachable size).
hipError_t launch_ensemble_summary(int64_t n, int k, int which, const double* S, const double* H, const double* E,
                                   double* mean, double* sd, hipStream_t s);
// Multi-graph initialisation of arena nodes [v0, v1): node v hashes its
// graph-local id with its graph's seed; padding rows get empty counters.
hipError_t launch_init_arena(int log2m, int64_t v0, int64_t v1, const int32_t* blk_graph,
                             const GraphDev* graphs, uint8_t* cur, uint8_t* nxt, double* S, double* H,
                             double* E, const double* lc, double alpha_pp, hipStream_t s);
// One device-driven pass of a multi-graph context: push (sparse passes
// only), persistent expand, merge, per-graph convergence, next-pass planning
// and clearing of the next change bitmap.  Enqueues only (capturable).
hipError_t launch_device_pass(int log2m, const PassArgs& a, int persist_wgs, uint2* push_items,
                              unsigned long long* push_count, int64_t n_arena, hipStream_t s);
// Copies arena-layout values of graph nodes into packed graph-order arrays.
hipError_t launch_pack(const double* src, double* dst, int64_t n_arena, const int32_t* blk_graph,
                       const GraphDev* graphs, hipStream_t s);
// Serving: CSR of one graph into its pool regions (indices already copied
// to arc_base.. and rebased in place), slot admission at the next engine
// pass, planning totals, and a whole slot record.
hipError_t launch_rebase_csr(const void* off_l, int bits, int64_t n, int64_t m, int64_t node_base, int64_t arc_base,
                             int64_t* off, int32_t* idx, hipStream_t s);
hipError_t launch_admit(PassCtl* ctl, GraphDev* graphs, int32_t slot, const GraphDev& val, int64_t m,
                        int32_t* blk_graph, uint64_t* mod0, uint64_t* mod1, int64_t b0, int64_t b1, hipStream_t s);
hipError_t launch_set_plan(PassCtl* ctl, int64_t listed_rows, int64_t arcs, hipStream_t s);
// chunk_graph[j] for the 64-entry chunks j of a light list (see PassArgs).
hipError_t launch_chunk_graph(const int32_t* light, int64_t n_light, const int32_t* blk_graph, int32_t* chunk_graph,
                              hipStream_t s);
hipError_t launch_set_slot(GraphDev* graphs, int32_t slot, const GraphDev& val, hipStream_t s);
hipError_t launch_pack_u8(const uint8_t* src, uint8_t* dst, int64_t n_arena, int p, const int32_t* blk_graph,
                          const GraphDev* graphs, hipStream_t s);
// Streamed graphs: sets bit `bit` of mask[w] for every successor w in
// idx[0..count) (one chunk's arcs).
hipError_t launch_pred_masks(const int32_t* idx, int64_t count, uint32_t bit, uint32_t* mask, hipStream_t s);
// *act (zeroed here) receives the OR over the nodes whose bit is set in
// mod_prev of mask[node] and the bit (chunk % 32) of the chunk holding the
// node's own row; chunk_rows holds the first row of each of the n_chunks
// chunks.
hipError_t launch_chunk_activity(const uint64_t* mod_prev, int64_t n_words, const uint32_t* mask,
                                 const int64_t* chunk_rows, int32_t n_chunks, uint32_t* act, hipStream_t s);
// Compressed streamed chunks: arcs in blocks of STREAM_BLOCK_ARCS, each
// block its first id then zigzag differences, all as 7-bit variable-length
// integers; boff (blocks + 1 entries) gives each block's first byte.  Decodes
// n_arcs ids into ids.  The byte buffer must be readable up to boff[blocks]
// rounded up to 4 bytes.
constexpr int STREAM_BLOCK_ARCS = 32;
hipError_t launch_decode_chunk(const uint32_t* boff, const uint8_t* bytes, int64_t n_arcs, int32_t* ids, hipStream_t s);
// ev_mid (nullable) is recorded between the expand and merge kernels.
hipError_t launch_pass(int log2m, const PassArgs& a, hipStream_t s, hipEvent_t ev_mid);
hipError_t launch_finalize(int64_t n, const double* S, const double* H, const double* E,
                           double* clo, double* lin, double* harm, double* core, hipStream_t s);
hipError_t launch_widen_offsets(const int32_t* in, int64_t* out, int64_t count, hipStream_t s);
// Writes 1 to *bad if the CSR is malformed (bad must be zeroed first).
hipError_t launch_validate(const int64_t* off, const int32_t* idx, int64_t n, int64_t m,
                           int* bad, hipStream_t s);

// Stream compaction of the rows whose degree lies in [lo, hi], in increasing
// order, into out; *count (device) receives their number.  With tmp NULL,
// *tmp_bytes receives the scratch size (hipcub DeviceSelect).
hipError_t select_rows(const int64_t* off, int64_t n, int64_t lo, int64_t hi, int32_t* out, int* count, void* tmp,
                       size_t* tmp_bytes, hipStream_t s);
// out[2i], out[2i+1] = off[rows[i]], off[rows[i] + 1].
hipError_t launch_take_offsets(const int32_t* rows, int64_t count, const int64_t* off, int64_t* out, hipStream_t s);
// Reverse CSR (row w lists every v with an arc v->w, in increasing v).
// roff: n+1 entries, ridx: m entries.  Radix-sorts the arcs by target; the
// sort's scratch (2m int32 and hipcub storage) is allocated and freed inside.
hipError_t build_reverse(const int64_t* off, const int32_t* idx, int64_t n, int64_t m, int64_t* roff,
                         int32_t* ridx, hipStream_t s);
// Marks act[v] = epoch for every v with an arc to a node whose bit is set in
// mod_prev.  items/count are scratch (capacity `cap` items; count zeroed here).
hipError_t launch_push(const uint64_t* mod_prev, int64_t n_words, int64_t n, const int64_t* roff,
                       const int32_t* ridx, uint2* items, unsigned long long* count, int32_t* act,
                       int32_t epoch, hipStream_t s);

// ---- sparse passes from pair lists (single-graph contexts) ----------------
// Every arc v -> u whose successor u changed in the previous pass becomes a
// pair (v, u), every changed u also (u, -1) (its own write-back); the pairs
// are sorted by v, and each run of equal v is one row's work, cut into items
// of at most RUN_CHUNK pairs (runs of several items leave partial counters
// that a merge kernel folds).
constexpr int RUN_CHUNK = 64;

struct PairItem {
  int64_t start;   // first sorted pair
  int32_t len;     // pairs
  int32_t row;
  int32_t nparts;  // items of the row's run
  int32_t slot;    // partial slot (nparts > 1), else -1
  int32_t pad[2];
};

// Device buffers of the pair path, sized for `cap` pairs at init.
struct PairBufs {
  int64_t cap = 0;                 // pairs
  int64_t items_cap = 0;           // cap + cap / RUN_CHUNK + 1
  int64_t slots_cap = 0;           // cap / (RUN_CHUNK / 2) + 2
  int64_t multi_cap = 0;           // cap / (RUN_CHUNK + 1) + 1
  int end_bit = 1;                 // key bits of the sort
  uint32_t* keys[2] = {nullptr, nullptr};  // row of each pair: emitted, sorted
  int32_t* vals[2] = {nullptr, nullptr};   // successor (-1: own write-back)
  uint32_t* uniq = nullptr;        // per run: row
  uint32_t* cnt = nullptr;         // per run: pairs
  uint32_t* rstart = nullptr;      // per run: first sorted pair
  uint32_t* ni = nullptr;          // per run: items
  uint32_t* ioff = nullptr;        // per run: first item
  uint32_t* mp = nullptr;          // per run: partial slots needed
  uint32_t* pbase = nullptr;       // per run: first partial slot
  int32_t* num_runs = nullptr;     // device scalars: runs, items, multi-item runs
  uint32_t* num_items = nullptr;
  uint32_t* num_multi = nullptr;
  uint32_t* multi = nullptr;       // first item of each multi-item run
  unsigned long long* npairs = nullptr;  // pairs reserved (checked against the plan)
  uint32_t* ppos = nullptr;        // first pair of each push item (push item capacity)
  PairItem* items = nullptr;
  uint8_t* partial = nullptr;      // slots_cap x p bytes
  void* tmp = nullptr;
  size_t tmp_bytes = 0;
};
// hipcub scratch the pair path needs for `cap` pairs and `end_bit` key bits.
size_t pair_tmp_bytes(int64_t cap, int end_bit);
// Builds the sorted pair list and work items of a sparse pass (total = the
// exact number of pairs: arcs into changed counters plus changed rows, at
// most pb.cap); items/count are the push item scratch.  Enqueues only.
hipError_t launch_pair_build(const PassArgs& a, const PairBufs& pb, int64_t total, uint2* items,
                             unsigned long long* count, hipStream_t s);
// Runs the pass over the pair items (expand, then the merge of multi-item
// runs); ev_mid, if set, is recorded between the two.
hipError_t launch_pair_pass(int log2m, const PassArgs& a, const PairBufs& pb, int64_t total, hipStream_t s,
                            hipEvent_t ev_mid);

}  // namespace hb
