// Host-side context shared by the C-ABI entry points (hb_api.cpp) and the
// serving loop (hb_serve.cpp).  Not part of the public ABI.
#pragma once

#include <string>
#include <vector>

#include "../../include/hb.h"
#include "hb_internal.h"

namespace hbh {

// Message of the last failure on this thread (hb_last_error).
extern thread_local std::string g_err;

inline hb_status fail(hb_status st, const std::string& msg) {
  g_err = msg;
  return st;
}

#define HB_HIP(call)                                                                                   \
  do {                                                                                                 \
    hipError_t e_ = (call);                                                                            \
    if (e_ != hipSuccess) return hbh::fail(HB_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
  } while (0)

template <class T>
hipError_t dmalloc(T** p, size_t count) {
  *p = nullptr;
  if (count == 0) count = 1;
  return hipMalloc(reinterpret_cast<void**>(p), count * sizeof(T));
}

// Row classes of the degree-aware schedule, on the host, for offsets of type
// T (int32 or int64): rows with 1..light_max arcs, rows below heavy_min arcs,
// and heavy rows cut into chunks of `chunk` arcs (item offsets are the CSR's
// own); empty rows never change and are left out.
template <class T>
void plan_rows_host(const T* off, int64_t n, int64_t light_max, int64_t heavy_min, int64_t chunk,
                    std::vector<int32_t>& light, std::vector<int32_t>& medium, std::vector<hb::HeavyItem>& items,
                    std::vector<hb::HeavyRow>& hrows) {
  for (int64_t v = 0; v < n; ++v) {
    const int64_t s = (int64_t)off[v], e = (int64_t)off[v + 1], deg = e - s;
    if (deg == 0) continue;
    if (deg <= light_max) {
      light.push_back((int32_t)v);
    } else if (deg < heavy_min) {
      medium.push_back((int32_t)v);
    } else {
      hb::HeavyRow hr;
      hr.row = v;
      hr.item0 = (int64_t)items.size();
      for (int64_t k = s; k < e; k += chunk) {
        hb::HeavyItem it;
        it.row = v;
        it.e0 = k;
        it.e1 = k + chunk < e ? k + chunk : e;
        items.push_back(it);
      }
      hr.nitems = (int64_t)items.size() - hr.item0;
      hrows.push_back(hr);
    }
  }
}

// alpha_p of Flajolet-Fusy-Gandouet-Meunier 2007 (Algorithm 1 defers to it).
inline double alpha_for(int p) {
  if (p == 16) return 0.673;
  if (p == 32) return 0.697;
  if (p == 64) return 0.709;
  return 0.7213 / (1.0 + 1.079 / (double)p);
}

}  // namespace hbh

// One row chunk of a streamed graph: rows [r0, r1), arcs [e0, e1), and its
// entries of the row lists (light [l0, l1), medium [m0, m1), heavy items
// [i0, i1), heavy rows [h0, h1); the lists are sorted by row, so a chunk's
// entries are contiguous).
struct StreamChunk {
  int64_t r0, r1, e0, e1;
  int64_t l0, l1, m0, m1, i0, i1, h0, h1;
  // compressed chunks (opt.stream_compress): blocks, and where the chunk's
  // block offsets and bytes start in the pinned host arrays
  int64_t nb, bo_at, cb_at, cb_len;
};

struct hb_ctx {
  int64_t n = 0, m = 0;
  int b = 0, p = 0;              // row width: p = 2^b bytes
  // Multi-seed ensembles: a row holds n_seeds = 2^seg_log counters of
  // 2^b_seed registers each (otherwise n_seeds = 1 and b_seed = b).
  int32_t n_seeds = 1;
  int seg_log = 0;
  int b_seed = 0;
  std::vector<uint64_t> seeds;
  uint64_t* seeds_dev = nullptr;
  std::vector<int32_t> seed_passes;  // pass count of each seed once converged, else -1
  // Sec. 6 node weights (device, n entries; null: every weight 1).
  int32_t* weights = nullptr;
  // The counters hold singletons (an unweighted single-graph, single-seed
  // reset): the first pass recomputes successor counters from node hashes.
  bool singletons = false;
  // Sec. 7 discounted-gain accumulator and its table f(1..L) (empty: off).
  double* D = nullptr;
  std::vector<double> disc;
  // Neighbourhood function N(0..t) (opt.neighbourhood) and its exact-sum scratch.
  std::vector<double> nf;
  uint64_t* esum_part = nullptr;
  uint64_t* esum_out = nullptr;  // 3 sum words, the reported inexact flag, the kernels' flag word
  uint64_t* esum_host = nullptr; // pinned copy of esum_out
  uint64_t seed = 0;
  hb_options opt{};
  hipStream_t stream = nullptr;
  int64_t* off = nullptr;
  bool own_off = false;
  const int32_t* idx = nullptr;
  int32_t* idx_owned = nullptr;
  uint8_t* cnt[2] = {nullptr, nullptr};
  uint64_t* mod[2] = {nullptr, nullptr};
  uint16_t* dmask[2] = {nullptr, nullptr};
  int64_t n_blocks = 0;
  double* S = nullptr;
  double* H = nullptr;
  double* E = nullptr;
  double* lc = nullptr;
  double alpha_pp = 0.0;
  hb::HeavyItem* items = nullptr;
  int64_t n_items = 0;
  hb::HeavyRow* hrows = nullptr;
  int64_t n_hrows = 0;
  int64_t n_medium = 0;
  int32_t* light = nullptr;
  int32_t* medium = nullptr;
  int64_t n_light = 0;
  int64_t n_nonempty = 0;
  int64_t* roff = nullptr;      // reverse CSR (push activation)
  int32_t* ridx = nullptr;
  int32_t* act = nullptr;
  uint2* push_items = nullptr;
  unsigned long long* push_count = nullptr;
  hb::PairBufs pb;              // pair lists of sparse passes (pb.cap = 0: none)
  int32_t* chunk_graph = nullptr;  // batched contexts: graph of each 64-entry light-list chunk
  unsigned long long* npairs_host = nullptr;  // pinned: pairs the last pair pass emitted
  uint8_t* partial = nullptr;
  unsigned long long* stats = nullptr;       // 2 halves of STAT_SLOTS * STAT_K
  unsigned long long* stats_host = nullptr;  // pinned
  double* out_tmp = nullptr;                 // 4n doubles for host-destination finalize
  int* bad = nullptr;
  int cur = 0;
  int32_t t = 0;
  bool converged = false;
  int64_t last_nmod = -1;
  int64_t last_slices = -1;
  int64_t last_pairs = -1;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  // Multi-graph (batched) contexts.
  int32_t n_graphs = 0;
  std::vector<hb::GraphDev> graphs_host;
  hb::GraphDev* graphs = nullptr;
  int32_t* blk_graph = nullptr;
  hb::PassCtl* ctl = nullptr;
  hb::PassCtl* ctl_host = nullptr;  // pinned
  int64_t n_packed = 0;
  int persist_wgs = 0;
  int graph_passes = 0;              // passes per hipGraph replay
  hipGraphExec_t gexec = nullptr;
  bool own_stream = false;
  double* arena_tmp = nullptr;       // n doubles, arena layout staging for packed outputs
  std::vector<hb_pass_info> hist;
  double total_ms = 0.0;
  bool failed = false;
  // Streamed graphs (opt.stream_graph): the CSR stays in pinned host memory
  // and is uploaded chunk by chunk into two staging buffers every pass.
  bool streamed = false;
  int64_t* host_off = nullptr;   // pinned, n+1
  int32_t* host_idx = nullptr;   // pinned, m
  std::vector<StreamChunk> chunks;
  int64_t chunk_bytes = 0;       // capacity of each staging buffer
  uint8_t* stage[2] = {nullptr, nullptr};
  hipStream_t copy_stream = nullptr;
  hipEvent_t up_ev[2] = {nullptr, nullptr};
  hipEvent_t done_ev[2] = {nullptr, nullptr};
  uint32_t* pred_mask = nullptr;      // n words: chunks (mod 32) holding an arc into the node
  int64_t* chunk_rows = nullptr;      // first row of every chunk (device)
  uint32_t* chunk_act = nullptr;      // chunk selection of a pass (device word)
  uint32_t* chunk_act_host = nullptr; // pinned
  bool masks_ready = false;
  // Compressed streamed arcs (opt.stream_compress): per chunk, blocks of
  // STREAM_BLOCK_ARCS arcs coded as variable-length deltas, decoded on the
  // device after the upload.
  bool compressed = false;
  uint8_t* host_cbytes = nullptr;   // pinned: every chunk's bytes, each 4-byte aligned
  uint32_t* host_boff = nullptr;    // pinned: every chunk's block offsets (blocks + 1 each)
  int64_t cstage_bytes = 0;         // capacity of each compressed staging buffer
  uint8_t* cstage[2] = {nullptr, nullptr};
  int64_t host_graph_bytes = 0;     // pinned bytes holding the streamed graph
};

namespace hbh {

void release(hb_ctx* c);
hb_status plan_rows_device(hb_ctx* c);
hb_status upload_plan(hb_ctx* c, const std::vector<int32_t>& light, const std::vector<int32_t>& medium,
                      const std::vector<hb::HeavyItem>& items, const std::vector<hb::HeavyRow>& hrows);
hb::PassArgs device_args(hb_ctx* c);
hb_status read_ctl(hb_ctx* c);

}  // namespace hbh
