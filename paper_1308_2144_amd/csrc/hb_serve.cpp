// Serving form of libhb: a thread that admits centrality requests into
// resident multi-graph engines (one per log2m) and runs them with continuous
// batching.  See include/hb.h for the contract.
//
// Engine layout.  An engine is a multi-graph context whose arena is a pool:
// graphs occupy first-fit regions of the node pool (64-aligned, at least one
// padding row so that offsets[base + n] is private to the region) and of the
// arc pool, and contiguous segments of the row-class lists.  Node block 0 is a
// dead block mapped to slot 0, a permanently converged graph; list entries of
// retired graphs are zeroed, so they name row 0 and are skipped by every
// kernel.  Passes are the device-driven passes of the batched form; the pass
// index, mode and buffer parity live on the device, so admission and
// retirement are stream-ordered kernels and need no host round trip.
//
// Exactness of mid-flight admission.  A graph admitted before engine pass T
// starts from its singleton counters in both buffers with zero accumulators,
// and has every change bit set in the bitmap pass T reads.  In every pass
// mode a row whose successors all count as changed gathers all of them, so
// pass T computes the graph's pass 0 exactly; its distance weight is T+1-t0 =
// 1 with t0 = T.  From then on the graph's rows only ever read its own rows
// (arcs never leave a region), so the rest of the engine cannot affect it;
// the pass modes differ only in the work they skip (all are exact).  A
// converged graph is never run again, and both of its counter buffers hold
// its final counters.
#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <set>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>
#include <cmath>

#include "hb_ctx.h"

using namespace hbh;

namespace {

using Clock = std::chrono::steady_clock;

constexpr int64_t DEFAULT_BUDGET = 64ll << 30;
constexpr int64_t DEFAULT_MAX_NODES = 1ll << 25;
constexpr int64_t DEFAULT_MAX_ARCS = 1ll << 29;
constexpr int32_t DEFAULT_MAX_RESIDENT = 1024;
constexpr int TICK_DEPTH = 2;  // ticks in flight per engine

// First-fit allocator of index ranges [0, cap).
class RangePool {
 public:
  void reset(int64_t cap) {
    cap_ = cap;
    free_.clear();
    if (cap > 0) free_[0] = cap;
  }
  int64_t cap() const { return cap_; }
  // A range of `len` entries whose start is a multiple of `align`; len 0
  // always succeeds with start 0 and owns nothing.
  bool alloc(int64_t len, int64_t align, int64_t* start) {
    *start = 0;
    if (len == 0) return true;
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      const int64_t s = it->first, e = it->first + it->second;
      const int64_t a = (s + align - 1) / align * align;
      if (a + len > e) continue;
      free_.erase(it);
      if (a > s) free_[s] = a - s;
      if (a + len < e) free_[a + len] = e - (a + len);
      *start = a;
      return true;
    }
    return false;
  }
  void release(int64_t start, int64_t len) {
    if (len == 0) return;
    int64_t s = start, e = start + len;
    auto nx = free_.lower_bound(s);
    if (nx != free_.end() && nx->first == e) {
      e += nx->second;
      nx = free_.erase(nx);
    }
    if (nx != free_.begin()) {
      auto pv = std::prev(nx);
      if (pv->first + pv->second == s) {
        s = pv->first;
        free_.erase(pv);
      }
    }
    free_[s] = e - s;
  }
  // End of the last allocated range.
  int64_t high_water() const {
    if (free_.empty()) return cap_;
    const auto last = std::prev(free_.end());
    return last->first + last->second == cap_ ? last->first : cap_;
  }

 private:
  int64_t cap_ = 0;
  std::map<int64_t, int64_t> free_;
};

struct Seg {
  int64_t start = 0, len = 0;
};

struct Engine;

struct Req {
  int64_t id = 0;
  hb_serve_request rq{};
  int64_t n = 0, m = 0, npad = 0, bytes = 0;
  int b = 0;
  // Visible to callers (guarded by the server mutex).
  int32_t state = HB_REQ_QUEUED;
  int32_t passes = 0;
  double t_submit = 0.0, t_admit = -1.0, t_done = -1.0;
  bool reported = false;        // final state handed to a caller
  bool server_released = false; // the serving thread holds no reference
  std::string err;
  // Serving-thread state.
  Engine* eng = nullptr;
  int32_t slot = -1;
  int64_t node_base = 0, arc_base = 0;
  Seg light, medium, items, hrows;
  std::vector<int32_t> light_v, medium_v;
  std::vector<hb::HeavyItem> items_v;
  std::vector<hb::HeavyRow> hrows_v;
  int64_t admit_seq = 0;  // first tick whose snapshot describes this request
  bool seen_done = false;
  bool planned = false;
  bool admitting = false;  // guarded by the mutex: placement under way, no cancel
};

struct Tick {
  hipEvent_t ev = nullptr;
  hb::GraphDev* snap = nullptr;  // pinned copy of the slot table after the tick
  int64_t seq = 0;
  int32_t n_slots = 0;
};

struct Engine {
  int b = 0, p = 0;
  hb_ctx* c = nullptr;
  RangePool nodes, arcs, light, medium, items, hrows;
  int32_t n_slots = 0;
  std::set<int32_t> free_slots;
  std::vector<Req*> slot_req;
  int64_t listed = 0, arcs_res = 0;
  bool plan_dirty = true;
  int64_t running = 0;  // admitted and not yet seen converged
  std::deque<Tick> inflight;
  std::vector<Tick> spare;
  int64_t seq = 0;
  uint8_t* stage = nullptr;
  size_t stage_bytes = 0;
};

struct RetireBatch {
  hipEvent_t ev = nullptr;
  std::vector<Req*> reqs;
};

}  // namespace

struct hb_server {
  hb_serve_config cfg{};
  int device = 0;
  Clock::time_point t0;
  std::thread th;
  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  // Guarded by mu.
  std::deque<Req*> incoming;
  std::unordered_map<int64_t, Req*> reqs;
  int64_t next_id = 1;
  bool stop = false;
  bool paused = false;
  bool failed = false;
  bool exited = false;
  std::string fail_msg;
  hb_serve_stats_t st{};
  // Serving thread only.
  std::deque<Req*> pending;
  Engine* eng[9] = {};
  std::deque<RetireBatch> retiring;
  std::vector<hipEvent_t> free_events;
  int64_t resident_bytes = 0;
  int64_t inflight_ticks = 0;
  Clock::time_point busy_since;
};

namespace {

double now_s(const hb_server* s) {
  return std::chrono::duration<double>(Clock::now() - s->t0).count();
}

// Must hold s->mu.  Frees a request once it was reported and the serving
// thread let go of it.
void maybe_delete(hb_server* s, Req* r) {
  if (r->reported && r->server_released) {
    s->reqs.erase(r->id);
    delete r;
  }
}

void fill_defaults(hb_serve_config* cfg) {
  if (cfg->budget_bytes <= 0) cfg->budget_bytes = DEFAULT_BUDGET;
  if (cfg->max_nodes <= 0) cfg->max_nodes = DEFAULT_MAX_NODES;
  cfg->max_nodes = std::max<int64_t>(cfg->max_nodes / 64 * 64, 128);
  if (cfg->max_nodes > 0x7fffffc0LL) cfg->max_nodes = 0x7fffffc0LL;
  if (cfg->max_arcs <= 0) cfg->max_arcs = DEFAULT_MAX_ARCS;
  if (cfg->max_resident <= 0) cfg->max_resident = DEFAULT_MAX_RESIDENT;
  if (cfg->passes_per_tick <= 0) cfg->passes_per_tick = 1;
  hb_options& o = cfg->opt;
  hb_options d;
  hb_default_options(&d);
  if (o.light_max <= 0) o.light_max = d.light_max;
  if (o.heavy_min <= 0) o.heavy_min = d.heavy_min;
  if (o.chunk <= 0) o.chunk = d.chunk;
  if (o.dense_pct < 0) o.dense_pct = d.dense_pct;
  if (o.sparse_pct < 0) o.sparse_pct = d.sparse_pct;
  if (o.heavy_min <= o.light_max) o.heavy_min = o.light_max + 1;
}

// Pool capacities of the row-class lists: every row is in at most one list,
// a medium row has more than light_max arcs, a heavy row at least heavy_min
// arcs cut into chunks of `chunk`.
int64_t medium_cap(const hb_serve_config& c) { return c.max_arcs / (c.opt.light_max + 1) + 64; }
int64_t hrows_cap(const hb_serve_config& c) { return c.max_arcs / c.opt.heavy_min + 64; }
int64_t items_cap(const hb_serve_config& c) {
  return c.max_arcs / c.opt.chunk + c.max_arcs / c.opt.heavy_min + 64;
}

template <class T>
bool csr_ok(const T* off, const int32_t* idx, int64_t n, int64_t m) {
  if (off[0] != 0 || (int64_t)off[n] != m) return false;
  for (int64_t v = 0; v < n; ++v)
    if (off[v + 1] < off[v]) return false;
  for (int64_t e = 0; e < m; ++e)
    if (idx[e] < 0 || idx[e] >= n) return false;
  return true;
}

void release_engine(Engine* e) {
  if (!e) return;
  if (e->c && e->c->stream) (void)hipStreamSynchronize(e->c->stream);
  for (Tick& t : e->spare) {
    if (t.ev) (void)hipEventDestroy(t.ev);
    if (t.snap) (void)hipHostFree(t.snap);
  }
  for (Tick& t : e->inflight) {
    if (t.ev) (void)hipEventDestroy(t.ev);
    if (t.snap) (void)hipHostFree(t.snap);
  }
  if (e->stage) (void)hipFree(e->stage);  // the stream was synchronised above
  if (e->c) release(e->c);
  delete e;
}

hb_status make_engine(hb_server* s, int b, Engine** out) {
  *out = nullptr;
  Engine* e = new (std::nothrow) Engine();
  if (!e) return fail(HB_ENOMEM, "cannot allocate an engine");
  hb_ctx* c = new (std::nothrow) hb_ctx();
  if (!c) {
    delete e;
    return fail(HB_ENOMEM, "cannot allocate an engine context");
  }
  e->c = c;
  e->b = b;
  e->p = 1 << b;
  const hb_serve_config& cfg = s->cfg;
  const int64_t N = cfg.max_nodes, M = cfg.max_arcs;
  c->b = b;
  c->p = e->p;
  c->opt = cfg.opt;
  c->n = 0;
  c->m = 0;
  c->n_blocks = 0;
  e->n_slots = cfg.max_resident + 1;
  c->n_graphs = e->n_slots;
  auto bail = [&](hb_status st) {
    const std::string msg = g_err;
    release_engine(e);
    g_err = msg;
    return st;
  };
#define ENG_HIP(call)                                                                         \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      return bail(fail(HB_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)));       \
  } while (0)
#define ENG_ALLOC(ptr, count)                                                                 \
  do {                                                                                        \
    if (dmalloc(&(ptr), (size_t)(count)) != hipSuccess)                                       \
      return bail(fail(HB_ENOMEM, std::string("engine pool allocation failed: ") + #ptr));    \
  } while (0)
  ENG_HIP(hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking));
  c->own_stream = true;
  ENG_ALLOC(c->off, N + 1);
  c->own_off = true;
  ENG_ALLOC(c->idx_owned, M);
  c->idx = c->idx_owned;
  for (int i = 0; i < 2; ++i) {
    ENG_ALLOC(c->cnt[i], (size_t)N * (size_t)e->p);
    ENG_ALLOC(c->mod[i], N / 64);
  }
  ENG_ALLOC(c->S, N);
  ENG_ALLOC(c->H, N);
  ENG_ALLOC(c->E, N);
  ENG_ALLOC(c->lc, e->p + 1);
  ENG_ALLOC(c->light, N);
  ENG_ALLOC(c->medium, medium_cap(cfg));
  ENG_ALLOC(c->items, items_cap(cfg));
  ENG_ALLOC(c->hrows, hrows_cap(cfg));
  ENG_ALLOC(c->partial, (size_t)items_cap(cfg) * (size_t)e->p);
  ENG_ALLOC(c->stats, (size_t)2 * hb::STAT_SLOTS * hb::STAT_K);
  ENG_ALLOC(c->graphs, e->n_slots);
  ENG_ALLOC(c->blk_graph, N / 64);
  ENG_ALLOC(c->ctl, 1);
  // Staging for one request at a time, in stream order on the engine stream:
  // its offsets before the rebase (<= 8 (N+1) bytes) and its four finalized
  // outputs before their copies to the host (32 N bytes).  Allocated once,
  // here, so that no allocation or free is ever ordered on a stream.
  e->stage_bytes = std::max((size_t)8 * (size_t)(N + 1), (size_t)32 * (size_t)N);
  ENG_ALLOC(e->stage, e->stage_bytes);

  hipStream_t st = c->stream;
  ENG_HIP(hb::launch_fill_zero(c->off, sizeof(int64_t) * (size_t)(N + 1), st));
  for (int i = 0; i < 2; ++i) ENG_HIP(hb::launch_fill_zero(c->mod[i], sizeof(uint64_t) * (size_t)(N / 64), st));
  ENG_HIP(hb::launch_fill_zero(c->light, sizeof(int32_t) * (size_t)N, st));
  ENG_HIP(hb::launch_fill_zero(c->medium, sizeof(int32_t) * (size_t)medium_cap(cfg), st));
  ENG_HIP(hb::launch_fill_zero(c->items, sizeof(hb::HeavyItem) * (size_t)items_cap(cfg), st));
  ENG_HIP(hb::launch_fill_zero(c->hrows, sizeof(hb::HeavyRow) * (size_t)hrows_cap(cfg), st));
  ENG_HIP(hb::launch_fill_zero(c->stats, sizeof(unsigned long long) * 2 * hb::STAT_SLOTS * hb::STAT_K, st));
  ENG_HIP(hb::launch_fill_zero(c->graphs, sizeof(hb::GraphDev) * (size_t)e->n_slots, st));
  ENG_HIP(hb::launch_fill_zero(c->blk_graph, sizeof(int32_t) * (size_t)(N / 64), st));
  hb::GraphDev dead{};
  dead.done = 1;
  ENG_HIP(hb::launch_set_slot(c->graphs, 0, dead, st));
  c->alpha_pp = (alpha_for(e->p) * (double)e->p) * (double)e->p;
  std::vector<double> lc((size_t)e->p + 1, 0.0);
  for (int V = 1; V <= e->p; ++V) lc[(size_t)V] = (double)e->p * std::log((double)e->p / (double)V);
  ENG_HIP(hipMemcpyAsync(c->lc, lc.data(), sizeof(double) * lc.size(), hipMemcpyHostToDevice, st));
  hb::PassCtl k{};
  k.mode = hb::MODE_DENSE;
  k.frontier = cfg.opt.frontier;
  k.dense_pct = cfg.opt.dense_pct;
  k.sparse_pct = cfg.opt.sparse_pct;
  k.has_reverse = 0;
  k.n_graphs = e->n_slots;
  ENG_HIP(hipMemcpyAsync(c->ctl, &k, sizeof(k), hipMemcpyHostToDevice, st));
  ENG_HIP(hipStreamSynchronize(st));  // host staging above dies here
  int dev = 0;
  ENG_HIP(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  ENG_HIP(hipGetDeviceProperties(&prop, dev));
  c->persist_wgs = prop.multiProcessorCount * (cfg.opt.wgs_per_cu > 0 ? cfg.opt.wgs_per_cu : 5);
  for (int i = 0; i < TICK_DEPTH; ++i) {
    Tick t;
    ENG_HIP(hipEventCreateWithFlags(&t.ev, hipEventDisableTiming));
    ENG_HIP(hipHostMalloc(reinterpret_cast<void**>(&t.snap), sizeof(hb::GraphDev) * (size_t)e->n_slots,
                          hipHostMallocDefault));
    e->spare.push_back(t);
  }
#undef ENG_HIP
#undef ENG_ALLOC
  e->nodes.reset(N);
  int64_t dead_block = 0;
  (void)e->nodes.alloc(64, 64, &dead_block);  // block 0: the dead rows
  e->arcs.reset(M);
  e->light.reset(N);
  e->medium.reset(medium_cap(cfg));
  e->items.reset(items_cap(cfg));
  e->hrows.reset(hrows_cap(cfg));
  e->slot_req.assign((size_t)e->n_slots, nullptr);
  for (int32_t i = 1; i < e->n_slots; ++i) e->free_slots.insert(i);
  *out = e;
  return HB_OK;
}

// The engine's stage holds what one request needs (sized in make_engine for
// the largest request the node pool admits).
hb_status ensure_stage(Engine* e, size_t bytes) {
  if (bytes > e->stage_bytes) return fail(HB_EINVAL, "request larger than the engine's staging buffer");
  return HB_OK;
}

void release_regions(Engine* e, Req* r) {
  e->nodes.release(r->node_base, r->npad);
  e->arcs.release(r->arc_base, r->m);
  e->light.release(r->light.start, r->light.len);
  e->medium.release(r->medium.start, r->medium.len);
  e->items.release(r->items.start, r->items.len);
  e->hrows.release(r->hrows.start, r->hrows.len);
}

// Places a request in its engine if everything it needs is free now; false
// (and nothing taken) otherwise.
bool place(Engine* e, Req* r) {
  if (e->free_slots.empty()) return false;
  r->light.len = (int64_t)r->light_v.size();
  r->medium.len = (int64_t)r->medium_v.size();
  r->items.len = (int64_t)r->items_v.size();
  r->hrows.len = (int64_t)r->hrows_v.size();
  RangePool* pools[6] = {&e->nodes, &e->arcs, &e->light, &e->medium, &e->items, &e->hrows};
  int64_t* starts[6] = {&r->node_base, &r->arc_base, &r->light.start, &r->medium.start, &r->items.start,
                        &r->hrows.start};
  const int64_t lens[6] = {r->npad, r->m, r->light.len, r->medium.len, r->items.len, r->hrows.len};
  const int64_t aligns[6] = {64, 1, 1, 1, 1, 1};
  for (int i = 0; i < 6; ++i) {
    if (pools[i]->alloc(lens[i], aligns[i], starts[i])) continue;
    for (int j = i - 1; j >= 0; --j) pools[j]->release(*starts[j], lens[j]);
    return false;
  }
  r->slot = *e->free_slots.begin();
  e->free_slots.erase(e->free_slots.begin());
  return true;
}

}  // namespace

namespace {

// ---- the serving thread ------------------------------------------------------

hb_status get_engine(hb_server* s, int b, Engine** out) {
  if (!s->eng[b]) {
    hb_status st = make_engine(s, b, &s->eng[b]);
    if (st != HB_OK) return st;
  }
  *out = s->eng[b];
  return HB_OK;
}

// Enqueues the upload and admission of a placed request.
hb_status enqueue_admit(Engine* e, Req* r) {
  hb_ctx* c = e->c;
  hipStream_t st = c->stream;
  const hb_csr& g = r->rq.graph;
  const size_t ob = g.offsets_bits == 64 ? 8 : 4;
  hb_status hs = ensure_stage(e, std::max(ob * (size_t)(r->n + 1), (size_t)32 * (size_t)r->n));
  if (hs != HB_OK) return hs;
  HB_HIP(hipMemcpyAsync(e->stage, g.offsets, ob * (size_t)(r->n + 1), hipMemcpyHostToDevice, st));
  if (r->m > 0)
    HB_HIP(hipMemcpyAsync(const_cast<int32_t*>(c->idx) + r->arc_base, g.indices, sizeof(int32_t) * (size_t)r->m,
                          hipMemcpyHostToDevice, st));
  HB_HIP(hb::launch_rebase_csr(e->stage, g.offsets_bits, r->n, r->m, r->node_base, r->arc_base, c->off,
                               const_cast<int32_t*>(c->idx), st));
  // Row lists in engine ids (host copies live until the request retires).
  for (auto& v : r->light_v) v += (int32_t)r->node_base;
  for (auto& v : r->medium_v) v += (int32_t)r->node_base;
  for (auto& it : r->items_v) {
    it.row += r->node_base;
    it.e0 += r->arc_base;
    it.e1 += r->arc_base;
  }
  for (auto& h : r->hrows_v) {
    h.row += r->node_base;
    h.item0 += r->items.start;
  }
  if (r->light.len)
    HB_HIP(hipMemcpyAsync(c->light + r->light.start, r->light_v.data(), sizeof(int32_t) * (size_t)r->light.len,
                          hipMemcpyHostToDevice, st));
  if (r->medium.len)
    HB_HIP(hipMemcpyAsync(c->medium + r->medium.start, r->medium_v.data(), sizeof(int32_t) * (size_t)r->medium.len,
                          hipMemcpyHostToDevice, st));
  if (r->items.len)
    HB_HIP(hipMemcpyAsync(c->items + r->items.start, r->items_v.data(), sizeof(hb::HeavyItem) * (size_t)r->items.len,
                          hipMemcpyHostToDevice, st));
  if (r->hrows.len)
    HB_HIP(hipMemcpyAsync(c->hrows + r->hrows.start, r->hrows_v.data(), sizeof(hb::HeavyRow) * (size_t)r->hrows.len,
                          hipMemcpyHostToDevice, st));
  hb::GraphDev gd{};
  gd.node_base = r->node_base;
  gd.n = r->n;
  gd.packed = 0;
  gd.seed = r->rq.seed;
  HB_HIP(hb::launch_admit(c->ctl, c->graphs, r->slot, gd, r->m, c->blk_graph, c->mod[0], c->mod[1],
                          r->node_base / 64, (r->node_base + r->npad) / 64, st));
  HB_HIP(hb::launch_init_arena(e->b, r->node_base, r->node_base + r->npad, c->blk_graph, c->graphs, c->cnt[0],
                               c->cnt[1], c->S, c->H, c->E, c->lc, c->alpha_pp, st));
  e->slot_req[(size_t)r->slot] = r;
  e->listed += r->light.len + r->medium.len + r->hrows.len;
  e->arcs_res += r->m;
  e->plan_dirty = true;
  e->running += 1;
  r->eng = e;
  r->admit_seq = e->seq;
  return HB_OK;
}

// Enqueues the outputs of a converged request and frees its place.
hb_status enqueue_retire(hb_server* s, Engine* e, Req* r) {
  hb_ctx* c = e->c;
  hipStream_t st = c->stream;
  const hb_serve_request& q = r->rq;
  const int64_t base = r->node_base, n = r->n;
  if (n > 0) {
    if (q.closeness || q.lin || q.harmonic || q.coreach) {
      const hb_status hs = ensure_stage(e, (size_t)32 * (size_t)n);
      if (hs != HB_OK) return hs;
      double* o = reinterpret_cast<double*>(e->stage);
      HB_HIP(hb::launch_finalize(n, c->S + base, c->H + base, c->E + base, o, o + n, o + 2 * n, o + 3 * n, st));
      double* dst[4] = {q.closeness, q.lin, q.harmonic, q.coreach};
      for (int i = 0; i < 4; ++i)
        if (dst[i])
          HB_HIP(hipMemcpyAsync(dst[i], o + (size_t)i * (size_t)n, sizeof(double) * (size_t)n, hipMemcpyDeviceToHost,
                                st));
    }
    if (q.S) HB_HIP(hipMemcpyAsync(q.S, c->S + base, sizeof(double) * (size_t)n, hipMemcpyDeviceToHost, st));
    if (q.H) HB_HIP(hipMemcpyAsync(q.H, c->H + base, sizeof(double) * (size_t)n, hipMemcpyDeviceToHost, st));
    if (q.registers)
      HB_HIP(hipMemcpyAsync(q.registers, c->cnt[0] + (size_t)base * (size_t)e->p, (size_t)n * (size_t)e->p,
                            hipMemcpyDeviceToHost, st));
  }
  hb::GraphDev dead{};
  dead.done = 1;
  HB_HIP(hb::launch_set_slot(c->graphs, r->slot, dead, st));
  if (r->light.len) HB_HIP(hb::launch_fill_zero(c->light + r->light.start, sizeof(int32_t) * (size_t)r->light.len, st));
  if (r->medium.len)
    HB_HIP(hb::launch_fill_zero(c->medium + r->medium.start, sizeof(int32_t) * (size_t)r->medium.len, st));
  if (r->items.len)
    HB_HIP(hb::launch_fill_zero(c->items + r->items.start, sizeof(hb::HeavyItem) * (size_t)r->items.len, st));
  if (r->hrows.len)
    HB_HIP(hb::launch_fill_zero(c->hrows + r->hrows.start, sizeof(hb::HeavyRow) * (size_t)r->hrows.len, st));
  release_regions(e, r);
  e->slot_req[(size_t)r->slot] = nullptr;
  e->free_slots.insert(r->slot);
  e->listed -= r->light.len + r->medium.len + r->hrows.len;
  e->arcs_res -= r->m;
  e->plan_dirty = true;
  s->resident_bytes -= r->bytes;
  return HB_OK;
}

hb_status enqueue_tick(hb_server* s, Engine* e) {
  hb_ctx* c = e->c;
  hipStream_t st = c->stream;
  if (e->plan_dirty) {
    HB_HIP(hb::launch_set_plan(c->ctl, e->listed, e->arcs_res, st));
    e->plan_dirty = false;
  }
  c->n = e->nodes.high_water();
  c->n_blocks = c->n / 64;
  c->n_light = e->light.high_water();
  c->n_medium = e->medium.high_water();
  c->n_items = e->items.high_water();
  c->n_hrows = e->hrows.high_water();
  const hb::PassArgs a = device_args(c);
  for (int k = 0; k < s->cfg.passes_per_tick; ++k)
    HB_HIP(hb::launch_device_pass(e->b, a, c->persist_wgs, nullptr, nullptr, c->n, st));
  Tick t = e->spare.back();
  e->spare.pop_back();
  // The snapshot covers slots up to the highest one in use.
  int32_t used_hw = 1;
  for (int32_t i = e->n_slots - 1; i > 0; --i)
    if (e->slot_req[(size_t)i]) {
      used_hw = i + 1;
      break;
    }
  t.n_slots = used_hw;
  t.seq = e->seq++;
  HB_HIP(hipMemcpyAsync(t.snap, c->graphs, sizeof(hb::GraphDev) * (size_t)used_hw, hipMemcpyDeviceToHost, st));
  HB_HIP(hipEventRecord(t.ev, st));
  e->inflight.push_back(t);
  if (s->inflight_ticks++ == 0) s->busy_since = Clock::now();
  std::lock_guard<std::mutex> lk(s->mu);
  s->st.ticks += 1;
  s->st.engine_passes += s->cfg.passes_per_tick;
  return HB_OK;
}

hb_status get_event(hb_server* s, hipEvent_t* ev) {
  if (!s->free_events.empty()) {
    *ev = s->free_events.back();
    s->free_events.pop_back();
    return HB_OK;
  }
  HB_HIP(hipEventCreateWithFlags(ev, hipEventDisableTiming));
  return HB_OK;
}

// One round of the serving loop; *progress tells whether anything happened.
hb_status serve_step(hb_server* s, bool* progress) {
  *progress = false;
  // 1. Finished result copies.
  while (!s->retiring.empty()) {
    RetireBatch& rb = s->retiring.front();
    const hipError_t q = hipEventQuery(rb.ev);
    if (q == hipErrorNotReady) break;
    if (q != hipSuccess) return fail(HB_EDEVICE, std::string("result copy: ") + hipGetErrorString(q));
    {
      std::lock_guard<std::mutex> lk(s->mu);
      const double t = now_s(s);
      for (Req* r : rb.reqs) {
        r->state = HB_REQ_DONE;
        r->t_done = t;
        r->server_released = true;
        s->st.completed += 1;
        s->st.resident -= 1;
        s->st.resident_bytes = s->resident_bytes;
        maybe_delete(s, r);
      }
    }
    s->cv_done.notify_all();
    s->free_events.push_back(rb.ev);
    s->retiring.pop_front();
    *progress = true;
  }
  // 2. Finished ticks: converged requests retire.
  for (int b = 4; b <= 8; ++b) {
    Engine* e = s->eng[b];
    if (!e) continue;
    std::vector<Req*> done;
    while (!e->inflight.empty()) {
      Tick& t = e->inflight.front();
      const hipError_t q = hipEventQuery(t.ev);
      if (q == hipErrorNotReady) break;
      if (q != hipSuccess) return fail(HB_EDEVICE, std::string("engine pass: ") + hipGetErrorString(q));
      for (int32_t i = 1; i < t.n_slots; ++i) {
        Req* r = e->slot_req[(size_t)i];
        if (!r || r->seen_done || t.seq < r->admit_seq || !t.snap[i].done) continue;
        r->seen_done = true;
        r->passes = t.snap[i].passes;
        e->running -= 1;
        done.push_back(r);
      }
      e->spare.push_back(t);
      e->inflight.pop_front();
      if (--s->inflight_ticks == 0) {
        const double busy = std::chrono::duration<double>(Clock::now() - s->busy_since).count();
        std::lock_guard<std::mutex> lk(s->mu);
        s->st.busy_s += busy;
      }
      *progress = true;
    }
    if (!done.empty()) {
      for (Req* r : done) {
        hb_status st = enqueue_retire(s, e, r);
        if (st != HB_OK) return st;
      }
      RetireBatch rb;
      hb_status st = get_event(s, &rb.ev);
      if (st != HB_OK) return st;
      HB_HIP(hipEventRecord(rb.ev, e->c->stream));
      rb.reqs = std::move(done);
      s->retiring.push_back(std::move(rb));
    }
  }
  // 3. Admission in submission order.
  while (!s->pending.empty()) {
    Req* r = s->pending.front();
    {
      std::lock_guard<std::mutex> lk(s->mu);
      if (r->state == HB_REQ_CANCELLED) {
        s->pending.pop_front();
        r->server_released = true;
        maybe_delete(s, r);
        *progress = true;
        continue;
      }
    }
    if (s->resident_bytes + r->bytes > s->cfg.budget_bytes) break;
    Engine* e = nullptr;
    hb_status st = get_engine(s, r->b, &e);
    if (st != HB_OK) return st;
    if (!r->planned) {
      const hb_csr& g = r->rq.graph;
      const hb_options& o = s->cfg.opt;
      if (g.offsets_bits == 64)
        plan_rows_host(static_cast<const int64_t*>(g.offsets), r->n, o.light_max, o.heavy_min, o.chunk, r->light_v,
                       r->medium_v, r->items_v, r->hrows_v);
      else
        plan_rows_host(static_cast<const int32_t*>(g.offsets), r->n, o.light_max, o.heavy_min, o.chunk, r->light_v,
                       r->medium_v, r->items_v, r->hrows_v);
      r->planned = true;
    }
    {
      std::lock_guard<std::mutex> lk(s->mu);
      if (r->state == HB_REQ_CANCELLED) continue;  // dropped on the next round
      r->admitting = true;
    }
    if (!place(e, r)) {
      std::lock_guard<std::mutex> lk(s->mu);
      r->admitting = false;
      break;
    }
    st = enqueue_admit(e, r);
    if (st != HB_OK) return st;
    s->pending.pop_front();
    s->resident_bytes += r->bytes;
    {
      std::lock_guard<std::mutex> lk(s->mu);
      r->state = HB_REQ_RUNNING;
      r->admitting = false;
      r->t_admit = now_s(s);
      s->st.admitted += 1;
      s->st.queued -= 1;
      s->st.resident += 1;
      s->st.resident_bytes = s->resident_bytes;
      s->st.peak_resident_bytes = std::max(s->st.peak_resident_bytes, s->resident_bytes);
    }
    *progress = true;
  }
  // 4. Keep every engine with running requests TICK_DEPTH ticks ahead.
  for (int b = 4; b <= 8; ++b) {
    Engine* e = s->eng[b];
    if (!e) continue;
    while (e->running > 0 && (int)e->inflight.size() < TICK_DEPTH) {
      hb_status st = enqueue_tick(s, e);
      if (st != HB_OK) return st;
      *progress = true;
    }
  }
  return HB_OK;
}

bool server_idle(const hb_server* s) {
  if (!s->pending.empty() || !s->retiring.empty()) return false;
  for (int b = 4; b <= 8; ++b)
    if (s->eng[b] && (s->eng[b]->running > 0 || !s->eng[b]->inflight.empty())) return false;
  return true;
}

void fail_all(hb_server* s, const std::string& msg) {
  std::lock_guard<std::mutex> lk(s->mu);
  s->failed = true;
  s->fail_msg = msg;
  for (auto& kv : s->reqs) {
    Req* r = kv.second;
    if (r->state == HB_REQ_QUEUED || r->state == HB_REQ_RUNNING) {
      r->state = HB_REQ_FAILED;
      r->err = msg;
      s->st.failed += 1;
    }
  }
  while (!s->incoming.empty()) s->incoming.pop_front();
}

void serve_main(hb_server* s) {
  (void)hipSetDevice(s->device);
  for (;;) {
    {
      std::unique_lock<std::mutex> lk(s->mu);
      while (!s->incoming.empty()) {
        s->pending.push_back(s->incoming.front());
        s->incoming.pop_front();
      }
      if (s->paused || server_idle(s)) {
        if (s->stop && !s->paused) break;
        s->cv_work.wait(lk, [s] { return (!s->paused && !s->incoming.empty()) || s->stop || (!s->paused && !server_idle(s)); });
        continue;
      }
    }
    bool progress = false;
    const hb_status st = serve_step(s, &progress);
    if (st != HB_OK) {
      fail_all(s, g_err);
      break;
    }
    if (!progress) std::this_thread::sleep_for(std::chrono::microseconds(20));
  }
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->exited = true;
  }
  s->cv_done.notify_all();
}

void fill_info(const Req* r, hb_request_info* info) {
  info->id = r->id;
  info->state = r->state;
  info->passes = r->passes;
  info->t_submit = r->t_submit;
  info->t_admit = r->t_admit;
  info->t_done = r->t_done;
}

bool is_final(int32_t state) {
  return state == HB_REQ_DONE || state == HB_REQ_CANCELLED || state == HB_REQ_FAILED;
}

}  // namespace

extern "C" {

void hb_serve_default_config(hb_serve_config* cfg) {
  if (!cfg) return;
  std::memset(cfg, 0, sizeof(*cfg));
  cfg->budget_bytes = DEFAULT_BUDGET;
  cfg->max_nodes = DEFAULT_MAX_NODES;
  cfg->max_arcs = DEFAULT_MAX_ARCS;
  cfg->max_resident = DEFAULT_MAX_RESIDENT;
  cfg->passes_per_tick = 1;
  hb_default_options(&cfg->opt);
}

hb_status hb_serve_start(hb_server** out, const hb_serve_config* cfg) {
  if (!out) return fail(HB_EINVAL, "out is NULL");
  *out = nullptr;
  hb_server* s = new (std::nothrow) hb_server();
  if (!s) return fail(HB_ENOMEM, "cannot allocate a server");
  if (cfg)
    s->cfg = *cfg;
  else
    hb_serve_default_config(&s->cfg);
  fill_defaults(&s->cfg);
  // The device is first used by the serving thread, when the first request
  // is admitted.
  if (hipGetDevice(&s->device) != hipSuccess) s->device = 0;
  s->paused = s->cfg.start_paused != 0;
  s->t0 = Clock::now();
  try {
    s->th = std::thread(serve_main, s);
  } catch (...) {
    delete s;
    return fail(HB_ENOMEM, "cannot start the serving thread");
  }
  *out = s;
  return HB_OK;
}

hb_status hb_serve_resume(hb_server* s) {
  if (!s) return fail(HB_EINVAL, "NULL server");
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->paused = false;
  }
  s->cv_work.notify_all();
  return HB_OK;
}

hb_status hb_serve_submit(hb_server* s, const hb_serve_request* rq, int64_t* id) {
  if (!s || !rq || !id) return fail(HB_EINVAL, "NULL argument");
  *id = 0;
  const hb_csr& g = rq->graph;
  if (g.on_device) return fail(HB_EINVAL, "served graphs must be host CSRs");
  if (rq->log2m < 4 || rq->log2m > 8) return fail(HB_EINVAL, "served requests need log2m in [4, 8]");
  if (g.n < 0 || g.m < 0 || (g.offsets_bits != 32 && g.offsets_bits != 64) || !g.offsets ||
      (g.m > 0 && !g.indices))
    return fail(HB_EINVAL, "malformed CSR description");
  if (g.offsets_bits == 32 && g.m > 0x7fffffffLL) return fail(HB_EINVAL, "m too large for int32 offsets");
  const hb_serve_config& cfg = s->cfg;
  const int64_t p = 1ll << rq->log2m;
  const int64_t npad = (g.n + 1 + 63) / 64 * 64;
  const int64_t bytes = 2 * g.n * p;
  if (bytes > cfg.budget_bytes) return fail(HB_ENOMEM, "request needs more counter memory than the budget");
  if (npad > cfg.max_nodes - 64 || g.m > cfg.max_arcs)
    return fail(HB_ENOMEM, "request larger than an engine's node or arc pool");
  if (cfg.opt.validate) {
    const bool ok = g.offsets_bits == 64 ? csr_ok(static_cast<const int64_t*>(g.offsets), g.indices, g.n, g.m)
                                         : csr_ok(static_cast<const int32_t*>(g.offsets), g.indices, g.n, g.m);
    if (!ok) return fail(HB_EINVAL, "malformed CSR (offsets or an index outside [0, n))");
  }
  Req* r = new (std::nothrow) Req();
  if (!r) return fail(HB_ENOMEM, "cannot allocate a request");
  r->rq = *rq;
  r->n = g.n;
  r->m = g.m;
  r->npad = npad;
  r->bytes = bytes;
  r->b = rq->log2m;
  {
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->failed || s->exited || s->stop) {
      delete r;
      return fail(HB_ESTATE, s->failed ? "server failed: " + s->fail_msg : std::string("server is stopping"));
    }
    r->id = s->next_id++;
    r->t_submit = now_s(s);
    s->reqs[r->id] = r;
    s->incoming.push_back(r);
    s->st.submitted += 1;
    s->st.queued += 1;
  }
  s->cv_work.notify_one();
  *id = r->id;
  return HB_OK;
}

hb_status hb_serve_poll(hb_server* s, int64_t id, hb_request_info* info) {
  if (!s || !info) return fail(HB_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  auto it = s->reqs.find(id);
  if (it == s->reqs.end() || it->second->reported) return fail(HB_EINVAL, "unknown request id");
  Req* r = it->second;
  fill_info(r, info);
  if (is_final(r->state)) {
    const bool bad = r->state == HB_REQ_FAILED;
    const std::string err = r->err;
    r->reported = true;
    maybe_delete(s, r);
    if (bad) return fail(HB_EDEVICE, "request failed: " + err);
  }
  return HB_OK;
}

hb_status hb_serve_wait(hb_server* s, int64_t id, double timeout_s, hb_request_info* info) {
  if (!s || !info) return fail(HB_EINVAL, "NULL argument");
  std::unique_lock<std::mutex> lk(s->mu);
  auto it = s->reqs.find(id);
  if (it == s->reqs.end() || it->second->reported) return fail(HB_EINVAL, "unknown request id");
  Req* r = it->second;
  auto ready = [&] { return is_final(r->state) || s->exited; };
  if (timeout_s < 0)
    s->cv_done.wait(lk, ready);
  else
    s->cv_done.wait_for(lk, std::chrono::duration<double>(timeout_s), ready);
  fill_info(r, info);
  if (!is_final(r->state)) {
    if (s->exited) return fail(HB_ESTATE, "serving thread ended: " + s->fail_msg);
    return fail(HB_ESTATE, "timed out");
  }
  const bool bad = r->state == HB_REQ_FAILED;
  const std::string err = r->err;
  r->reported = true;
  maybe_delete(s, r);
  if (bad) return fail(HB_EDEVICE, "request failed: " + err);
  return HB_OK;
}

hb_status hb_serve_cancel(hb_server* s, int64_t id) {
  if (!s) return fail(HB_EINVAL, "NULL server");
  {
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->reqs.find(id);
    if (it == s->reqs.end() || it->second->reported) return fail(HB_EINVAL, "unknown request id");
    Req* r = it->second;
    if (r->state != HB_REQ_QUEUED || r->admitting) return fail(HB_ESTATE, "request is no longer queued");
    r->state = HB_REQ_CANCELLED;
    s->st.cancelled += 1;
    s->st.queued -= 1;
  }
  s->cv_done.notify_all();
  s->cv_work.notify_one();
  return HB_OK;
}

hb_status hb_serve_stats(hb_server* s, hb_serve_stats_t* out) {
  if (!s || !out) return fail(HB_EINVAL, "NULL argument");
  std::lock_guard<std::mutex> lk(s->mu);
  *out = s->st;
  out->elapsed_s = now_s(s);
  return HB_OK;
}

hb_status hb_serve_stop(hb_server* s) {
  if (!s) return fail(HB_EINVAL, "NULL server");
  {
    std::lock_guard<std::mutex> lk(s->mu);
    s->stop = true;
    s->paused = false;
  }
  s->cv_work.notify_all();
  if (s->th.joinable()) s->th.join();
  const bool failed = s->failed;
  const std::string msg = s->fail_msg;
  for (int b = 4; b <= 8; ++b) release_engine(s->eng[b]);
  for (hipEvent_t ev : s->free_events) (void)hipEventDestroy(ev);
  for (RetireBatch& rb : s->retiring) (void)hipEventDestroy(rb.ev);
  for (auto& kv : s->reqs) delete kv.second;
  delete s;
  if (failed) return fail(HB_EDEVICE, "server failed: " + msg);
  return HB_OK;
}

}  // extern "C"
