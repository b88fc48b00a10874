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
// (the number of successors the next pass would gather with edge skipping)
constexpr int STAT_K = 8;

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
};

// Launchers (hb_kernels.hip).  All return the launch status.
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t s);
hipError_t launch_init_nodes(int log2m, int64_t n, uint64_t seed, uint8_t* cur, uint8_t* nxt,
                             double* S, double* H, double* E, const double* lc, double alpha_pp,
                             hipStream_t s);
// ev_mid (nullable) is recorded between the expand and merge kernels.
hipError_t launch_pass(int log2m, const PassArgs& a, hipStream_t s, hipEvent_t ev_mid);
hipError_t launch_finalize(int64_t n, const double* S, const double* H, const double* E,
                           double* clo, double* lin, double* harm, double* core, hipStream_t s);
hipError_t launch_widen_offsets(const int32_t* in, int64_t* out, int64_t count, hipStream_t s);
// Writes 1 to *bad if the CSR is malformed (bad must be zeroed first).
hipError_t launch_validate(const int64_t* off, const int32_t* idx, int64_t n, int64_t m,
                           int* bad, hipStream_t s);

// Reverse CSR (row w lists every v with an arc v->w).  roff: n+1 entries,
// ridx: m entries.  Needs n+1 scratch counters (zeroed here) and hipcub scan
// storage; both are allocated and freed inside.
hipError_t build_reverse(const int64_t* off, const int32_t* idx, int64_t n, int64_t m, int64_t* roff,
                         int32_t* ridx, hipStream_t s);
// Marks act[v] = epoch for every v with an arc to a node whose bit is set in
// mod_prev.  items/count are scratch (capacity `cap` items; count zeroed here).
hipError_t launch_push(const uint64_t* mod_prev, int64_t n_words, int64_t n, const int64_t* roff,
                       const int32_t* ridx, uint2* items, unsigned long long* count, int32_t* act,
                       int32_t epoch, hipStream_t s);

}  // namespace hb
