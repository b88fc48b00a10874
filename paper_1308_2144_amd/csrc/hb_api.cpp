// Host side of libhb: context management, validation, allocation and the
// per-pass driver loop.  See include/hb.h for the contract of every entry
// point.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <sys/mman.h>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "hb_ctx.h"
#include "hb_stream_codes.h"

namespace hbh {
thread_local std::string g_err;
}  // namespace hbh

using namespace hbh;

namespace {

constexpr int DEFAULT_LIGHT_MAX = 64;
constexpr int DEFAULT_HEAVY_MIN = 8192;
constexpr int DEFAULT_CHUNK = 4096;
constexpr int DEFAULT_DENSE_PCT = 60;
constexpr int DEFAULT_SPARSE_PCT = 20;

// Anonymous host mapping for the batch arena: uninitialised, released on
// scope exit, huge pages advised.
template <class T>
struct HostArena {
  T* p = nullptr;
  size_t bytes = 0;
  explicit HostArena(size_t count) : bytes(count * sizeof(T)) {
    void* m = mmap(nullptr, bytes, PROT_READ | PROT_WRITE, MAP_PRIVATE | MAP_ANONYMOUS, -1, 0);
    if (m == MAP_FAILED) return;
    (void)madvise(m, bytes, MADV_HUGEPAGE);
    p = static_cast<T*>(m);
  }
  ~HostArena() {
    if (p) (void)munmap(p, bytes);
  }
  HostArena(const HostArena&) = delete;
  HostArena& operator=(const HostArena&) = delete;
  explicit operator bool() const { return p != nullptr; }
  T& operator[](size_t i) { return p[i]; }
  T* get() { return p; }
};

}  // namespace


namespace hbh {

void release(hb_ctx* c) {
  if (!c) return;
  if (c->copy_stream) {
    (void)hipStreamSynchronize(c->copy_stream);
    (void)hipStreamDestroy(c->copy_stream);
  }
  for (int i = 0; i < 2; ++i) {
    if (c->up_ev[i]) (void)hipEventDestroy(c->up_ev[i]);
    if (c->done_ev[i]) (void)hipEventDestroy(c->done_ev[i]);
    (void)hipFree(c->stage[i]);
  }
  for (int i = 0; i < 2; ++i) (void)hipFree(c->cstage[i]);
  if (c->host_cbytes) (void)hipHostFree(c->host_cbytes);
  if (c->host_boff) (void)hipHostFree(c->host_boff);
  if (c->host_off) (void)hipHostFree(c->host_off);
  if (c->host_idx) (void)hipHostFree(c->host_idx);
  if (c->chunk_act_host) (void)hipHostFree(c->chunk_act_host);
  (void)hipFree(c->pred_mask);
  (void)hipFree(c->chunk_rows);
  (void)hipFree(c->chunk_act);
  if (c->own_off) (void)hipFree(c->off);
  (void)hipFree(c->idx_owned);
  for (int i = 0; i < 2; ++i) {
    (void)hipFree(c->cnt[i]);
    (void)hipFree(c->mod[i]);
    (void)hipFree(c->dmask[i]);
  }
  (void)hipFree(c->S);
  (void)hipFree(c->H);
  (void)hipFree(c->E);
  (void)hipFree(c->lc);
  (void)hipFree(c->light);
  (void)hipFree(c->medium);
  (void)hipFree(c->roff);
  (void)hipFree(c->ridx);
  (void)hipFree(c->act);
  (void)hipFree(c->push_items);
  (void)hipFree(c->push_count);
  {
    hb::PairBufs& pb = c->pb;
    for (int i = 0; i < 2; ++i) {
      (void)hipFree(pb.keys[i]);
      (void)hipFree(pb.vals[i]);
    }
    void* bufs[] = {pb.uniq, pb.cnt, pb.rstart, pb.ni, pb.ioff, pb.mp, pb.pbase, pb.num_runs, pb.num_items,
                    pb.num_multi, pb.multi, pb.npairs, pb.ppos, pb.items, pb.partial, pb.tmp};
    for (void* b : bufs) (void)hipFree(b);
    if (c->npairs_host) (void)hipHostFree(c->npairs_host);
  }
  (void)hipFree(c->items);
  (void)hipFree(c->hrows);
  (void)hipFree(c->partial);
  (void)hipFree(c->stats);
  (void)hipFree(c->out_tmp);
  (void)hipFree(c->bad);
  (void)hipFree(c->graphs);
  (void)hipFree(c->blk_graph);
  (void)hipFree(c->chunk_graph);
  (void)hipFree(c->ctl);
  (void)hipFree(c->arena_tmp);
  (void)hipFree(c->seeds_dev);
  (void)hipFree(c->weights);
  (void)hipFree(c->D);
  (void)hipFree(c->esum_part);
  (void)hipFree(c->esum_out);
  if (c->esum_host) (void)hipHostFree(c->esum_host);
  if (c->ctl_host) (void)hipHostFree(c->ctl_host);
  if (c->gexec) (void)hipGraphExecDestroy(c->gexec);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
  if (c->stats_host) (void)hipHostFree(c->stats_host);
  for (int i = 0; i < 4; ++i)
    if (c->ev[i]) (void)hipEventDestroy(c->ev[i]);
  delete c;
}

}  // namespace hbh

namespace {

hb_status check_ctx(hb_ctx* c) {
  if (!c) return fail(HB_EINVAL, "NULL context");
  if (c->failed) return fail(HB_ESTATE, "context is in a failed state");
  return HB_OK;
}

}  // namespace

namespace hbh {

// Row classes of the degree-aware schedule (empty rows never change and are
// left out of every pass): rows with 1..light_max arcs, rows up to heavy_min
// arcs, and heavy rows cut into chunks of `chunk` arcs.  Light and medium
// lists by stream compaction on the device (row order kept); the few heavy
// rows are copied back with their offsets and cut into chunks on the host.
hb_status plan_rows_device(hb_ctx* c) {
  const int64_t n = c->n, m = c->m;
  if (n == 0) {
    c->n_light = c->n_medium = c->n_items = c->n_hrows = 0;
    return HB_OK;
  }
  const int64_t lmax = c->opt.light_max, hmin = c->opt.heavy_min, chunk = c->opt.chunk;
  const int64_t med_cap = std::min<int64_t>(n, m / (lmax + 1) + 1);
  const int64_t heavy_cap = std::min<int64_t>(n, m / hmin + 1);
  int32_t* heavy = nullptr;
  int* counts = nullptr;
  void* tmp = nullptr;
  size_t tmp_bytes = 0, b1 = 0;
  HB_HIP(dmalloc(&c->light, (size_t)n));
  HB_HIP(dmalloc(&c->medium, (size_t)med_cap));
  HB_HIP(dmalloc(&heavy, (size_t)heavy_cap));
  HB_HIP(dmalloc(&counts, 3));
  hipError_t e = hb::select_rows(c->off, n, 1, lmax, c->light, counts, nullptr, &tmp_bytes, c->stream);
  if (e == hipSuccess) e = hb::select_rows(c->off, n, lmax + 1, hmin - 1, c->medium, counts + 1, nullptr, &b1, c->stream);
  tmp_bytes = std::max(tmp_bytes, b1);
  if (e == hipSuccess) e = hb::select_rows(c->off, n, hmin, INT64_MAX, heavy, counts + 2, nullptr, &b1, c->stream);
  tmp_bytes = std::max(tmp_bytes, b1);
  if (e == hipSuccess) e = hipMalloc(&tmp, tmp_bytes > 0 ? tmp_bytes : 1);
  if (e == hipSuccess) e = hb::select_rows(c->off, n, 1, lmax, c->light, counts, tmp, &tmp_bytes, c->stream);
  if (e == hipSuccess) e = hb::select_rows(c->off, n, lmax + 1, hmin - 1, c->medium, counts + 1, tmp, &tmp_bytes, c->stream);
  if (e == hipSuccess) e = hb::select_rows(c->off, n, hmin, INT64_MAX, heavy, counts + 2, tmp, &tmp_bytes, c->stream);
  int cnt[3] = {0, 0, 0};
  if (e == hipSuccess) e = hipMemcpyAsync(cnt, counts, sizeof(cnt), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  std::vector<int32_t> hrow_ids;
  std::vector<int64_t> hoff;
  int64_t* hoff_dev = nullptr;
  if (e == hipSuccess && cnt[2] > 0) {
    hrow_ids.resize((size_t)cnt[2]);
    hoff.resize(2 * (size_t)cnt[2]);
    e = dmalloc(&hoff_dev, 2 * (size_t)cnt[2]);
    if (e == hipSuccess) e = hb::launch_take_offsets(heavy, cnt[2], c->off, hoff_dev, c->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(hrow_ids.data(), heavy, sizeof(int32_t) * hrow_ids.size(), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(hoff.data(), hoff_dev, sizeof(int64_t) * hoff.size(), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  }
  (void)hipFree(tmp);
  (void)hipFree(counts);
  (void)hipFree(heavy);
  (void)hipFree(hoff_dev);
  if (e != hipSuccess) return fail(HB_EDEVICE, std::string("row classification: ") + hipGetErrorString(e));
  c->n_light = cnt[0];
  c->n_medium = cnt[1];
  std::vector<hb::HeavyItem> items;
  std::vector<hb::HeavyRow> hrows;
  for (size_t h = 0; h < hrow_ids.size(); ++h) {
    const int64_t v = hrow_ids[h], s0 = hoff[2 * h], e0 = hoff[2 * h + 1];
    hb::HeavyRow hr;
    hr.row = v;
    hr.item0 = (int64_t)items.size();
    for (int64_t k = s0; k < e0; k += chunk) {
      hb::HeavyItem it;
      it.row = v;
      it.e0 = k;
      it.e1 = k + chunk < e0 ? k + chunk : e0;
      items.push_back(it);
    }
    hr.nitems = (int64_t)items.size() - hr.item0;
    hrows.push_back(hr);
  }
  return upload_plan(c, {}, {}, items, hrows);
}

// Copies host-made row lists to the device (light / medium only when given:
// the device planner fills those itself).
hb_status upload_plan(hb_ctx* c, const std::vector<int32_t>& light, const std::vector<int32_t>& medium,
                      const std::vector<hb::HeavyItem>& items, const std::vector<hb::HeavyRow>& hrows) {
  if (!c->light) {
    c->n_light = (int64_t)light.size();
    c->n_medium = (int64_t)medium.size();
    HB_HIP(dmalloc(&c->light, light.size()));
    HB_HIP(dmalloc(&c->medium, medium.size()));
    if (!light.empty())
      HB_HIP(hipMemcpyAsync(c->light, light.data(), sizeof(int32_t) * light.size(), hipMemcpyHostToDevice,
                            c->stream));
    if (!medium.empty())
      HB_HIP(hipMemcpyAsync(c->medium, medium.data(), sizeof(int32_t) * medium.size(), hipMemcpyHostToDevice,
                            c->stream));
  }
  c->n_items = (int64_t)items.size();
  c->n_hrows = (int64_t)hrows.size();
  HB_HIP(dmalloc(&c->items, items.size()));
  HB_HIP(dmalloc(&c->hrows, hrows.size()));
  if (!items.empty())
    HB_HIP(hipMemcpyAsync(c->items, items.data(), sizeof(hb::HeavyItem) * items.size(), hipMemcpyHostToDevice,
                          c->stream));
  if (!hrows.empty())
    HB_HIP(hipMemcpyAsync(c->hrows, hrows.data(), sizeof(hb::HeavyRow) * hrows.size(), hipMemcpyHostToDevice,
                          c->stream));
  HB_HIP(hipStreamSynchronize(c->stream));  // host staging dies here
  return HB_OK;
}

}  // namespace hbh

namespace {

constexpr int ESUM_BLOCKS = 1024;
constexpr int64_t HOST_PLAN_MAX = 1 << 20;  // graphs up to this many nodes are classified on the host

// X * 2^-52 rounded to the nearest double (ties to even), X the 192-bit
// integer w[0] + w[1] 2^64 + w[2] 2^128 of an exact sum of estimates.
double fix_to_double(const uint64_t* w) {
  int top = -1;
  for (int i = 2; i >= 0 && top < 0; --i)
    if (w[i]) top = 64 * i + 63 - __builtin_clzll(w[i]);
  if (top < 0) return 0.0;
  if (top <= 52) return std::ldexp((double)w[0], -52);  // below 2^53: exact
  auto bit = [&](int k) -> uint64_t { return (w[k >> 6] >> (k & 63)) & 1ull; };
  const int shift = top - 52;
  uint64_t mant = 0;
  for (int k = 52; k >= 0; --k) mant = (mant << 1) | bit(shift + k);
  const uint64_t guard = bit(shift - 1);
  bool sticky = false;
  for (int k = 0; k < shift - 1 && !sticky; ++k) sticky = bit(k) != 0;
  int e = shift - 52;
  if (guard && (sticky || (mant & 1ull))) ++mant;
  if (mant == (1ull << 53)) {
    mant >>= 1;
    ++e;
  }
  return std::ldexp((double)mant, e);
}

// Enqueues the exact sum of the current estimates and its readback
// (esum_out: 3 sum words, the inexact flag, and the zeroed flag word the
// kernels use).
hipError_t enqueue_esum(hb_ctx* c) {
  hipError_t e = hb::launch_esum(c->E, c->n, c->esum_part, ESUM_BLOCKS, c->esum_out,
                                 reinterpret_cast<int*>(c->esum_out + 4), c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->esum_host, c->esum_out, 4 * sizeof(uint64_t), hipMemcpyDeviceToHost, c->stream);
  return e;
}

// After the stream synchronised: appends N(t).
hb_status take_esum(hb_ctx* c) {
  if ((uint32_t)c->esum_host[3] != 0u) return fail(HB_EDEVICE, "neighbourhood sum: an estimate is not a multiple of 2^-52");
  c->nf.push_back(fix_to_double(c->esum_host));
  return HB_OK;
}

hb_status do_reset(hb_ctx* c, uint64_t seed) {
  c->seed = seed;
  c->t = 0;
  c->cur = 0;
  c->converged = false;
  c->last_nmod = -1;
  c->last_slices = -1;
  c->last_pairs = -1;
  c->hist.clear();
  c->total_ms = 0.0;
  HB_HIP(hb::launch_fill_zero(c->mod[0], (size_t)c->n_blocks * 8, c->stream));
  HB_HIP(hb::launch_fill_zero(c->mod[1], (size_t)c->n_blocks * 8, c->stream));
  HB_HIP(hb::launch_fill_zero(c->stats, sizeof(unsigned long long) * 2 * hb::STAT_SLOTS * hb::STAT_K,
                              c->stream));
  if (c->act) HB_HIP(hb::launch_fill_zero(c->act, sizeof(int32_t) * (size_t)c->n, c->stream));
  if (c->n_graphs > 0) {
    for (auto& gd : c->graphs_host) {
      gd.t0 = 0;
      gd.done = 0;
      gd.passes = 0;
    }
    HB_HIP(hipMemcpyAsync(c->graphs, c->graphs_host.data(), sizeof(hb::GraphDev) * c->graphs_host.size(),
                          hipMemcpyHostToDevice, c->stream));
    hb::PassCtl& k = *c->ctl_host;
    k.t = 0;
    k.mode = hb::MODE_FIRST;
    k.parity = 0;
    k.n_done = 0;
    k.work = 0;
    k.rows_done = 0;
    k.batch = 1;
    HB_HIP(hipMemcpyAsync(c->ctl, c->ctl_host, sizeof(hb::PassCtl), hipMemcpyHostToDevice, c->stream));
    HB_HIP(hb::launch_init_arena(c->b, 0, c->n, c->blk_graph, c->graphs, c->cnt[0], c->cnt[1], c->S, c->H, c->E,
                                 c->lc, c->alpha_pp, c->stream));
    c->singletons = c->p <= 256;  // the first pass recomputes counters from node hashes
    HB_HIP(hipStreamSynchronize(c->stream));  // ctl_host is reused by the next readback
    return HB_OK;
  }
  if (c->n_seeds > 1) {
    std::fill(c->seed_passes.begin(), c->seed_passes.end(), -1);
    HB_HIP(hipMemcpyAsync(c->seeds_dev, c->seeds.data(), sizeof(uint64_t) * c->seeds.size(), hipMemcpyHostToDevice,
                          c->stream));
    HB_HIP(hb::launch_init_ensemble(c->b_seed, c->seg_log, c->n, c->seeds_dev, c->cnt[0], c->cnt[1], c->S, c->H,
                                    c->E, c->lc, c->alpha_pp, c->stream));
    HB_HIP(hipStreamSynchronize(c->stream));  // the seed upload reads host memory
    return HB_OK;
  }
  c->singletons = false;
  if (c->weights) {
    HB_HIP(hb::launch_init_weighted(c->b, c->n, seed, c->weights, c->cnt[0], c->cnt[1], c->S, c->H, c->D, c->E, c->lc,
                                    c->alpha_pp, c->stream));
  } else {
    HB_HIP(hb::launch_init_nodes(c->b, c->n, seed, c->cnt[0], c->cnt[1], c->S, c->H, c->E, c->lc,
                                 c->alpha_pp, c->stream));
    c->singletons = true;
    if (c->D) HB_HIP(hb::launch_fill_zero(c->D, sizeof(double) * (size_t)c->n, c->stream));
  }
  c->nf.clear();
  if (c->esum_out) {
    HB_HIP(enqueue_esum(c));
    HB_HIP(hipStreamSynchronize(c->stream));
    return take_esum(c);
  }
  return HB_OK;
}

// Pair-list buffers of sparse passes: every pair for small graphs (m + n <=
// 2^16), else about (m + n) / 16 (the sparse tail of a large graph needs far
// fewer; a pass with more pairs uses activation stamps).  About 80 bytes per
// pair of capacity.
hb_status alloc_pairs(hb_ctx* c) {
  hb::PairBufs& pb = c->pb;
  const int64_t all = c->m + c->n;
  const int64_t cap = std::min<int64_t>(all <= (1ll << 16) ? all : std::max<int64_t>(1ll << 16, all / 16),
                                        0x7fffffffLL);
  pb.cap = cap;
  pb.items_cap = cap + cap / hb::RUN_CHUNK + 1;
  pb.slots_cap = cap / (hb::RUN_CHUNK / 2) + 2;
  pb.multi_cap = cap / (hb::RUN_CHUNK + 1) + 1;
  int bits = 1;
  while (bits < 32 && (1ll << bits) < c->n) ++bits;
  pb.end_bit = bits;
  pb.tmp_bytes = hb::pair_tmp_bytes(cap, bits);
  bool ok = true;
  for (int i = 0; i < 2; ++i) {
    ok = ok && dmalloc(&pb.keys[i], (size_t)cap) == hipSuccess;
    ok = ok && dmalloc(&pb.vals[i], (size_t)cap) == hipSuccess;
  }
  uint32_t** runs[7] = {&pb.uniq, &pb.cnt, &pb.rstart, &pb.ni, &pb.ioff, &pb.mp, &pb.pbase};
  for (auto* r : runs) ok = ok && dmalloc(r, (size_t)cap) == hipSuccess;
  ok = ok && dmalloc(&pb.num_runs, 1) == hipSuccess && dmalloc(&pb.num_items, 1) == hipSuccess &&
       dmalloc(&pb.num_multi, 1) == hipSuccess && dmalloc(&pb.multi, (size_t)pb.multi_cap) == hipSuccess &&
       dmalloc(&pb.npairs, 1) == hipSuccess && dmalloc(&pb.items, (size_t)pb.items_cap) == hipSuccess &&
       dmalloc(&pb.ppos, (size_t)c->n + (size_t)(c->m / hb::PUSH_CHUNK) + 1) == hipSuccess &&
       dmalloc(&pb.partial, (size_t)pb.slots_cap * (size_t)c->p) == hipSuccess &&
       hipMalloc(&pb.tmp, pb.tmp_bytes) == hipSuccess &&
       hipHostMalloc(reinterpret_cast<void**>(&c->npairs_host), sizeof(unsigned long long), hipHostMallocDefault) ==
           hipSuccess;
  if (!ok) return fail(HB_ENOMEM, "cannot allocate the pair lists of sparse passes");
  // Unsorted lists start as valid pairs (row 0, no successor), so that a
  // pass whose pair count disagreed with its plan could not read an
  // undefined row; the host rejects such a pass after it ran.
  HB_HIP(hb::launch_fill_zero(pb.keys[0], sizeof(uint32_t) * (size_t)cap, c->stream));
  HB_HIP(hipMemsetAsync(pb.vals[0], 0xFF, sizeof(int32_t) * (size_t)cap, c->stream));
  return HB_OK;
}

constexpr int64_t DEFAULT_CHUNK_BYTES = (int64_t)256 << 20;

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Host check of a CSR: 0 if well formed, 1 for bad offsets, 2 for an index
// outside [0, n).
template <class T>
int host_csr_check(const T* off, const int32_t* idx, int64_t n, int64_t m) {
  if ((int64_t)off[0] != 0 || (int64_t)off[n] != m) return 1;
  for (int64_t v = 0; v < n; ++v)
    if (off[v + 1] < off[v]) return 1;
  for (int64_t e = 0; e < m; ++e)
    if (idx[e] < 0 || idx[e] >= n) return 2;
  return 0;
}

// Compressed streamed arcs: every row's successors sorted (the union is
// order-free, so results do not change), then each chunk's arcs coded in
// blocks of STREAM_BLOCK_ARCS consecutive arcs (hb_stream_codes.h).  Chunks
// are coded in parallel; the bytes (each chunk followed by 8 zero bytes, so
// the decoder may read a few bytes past a block) and block offsets go to
// pinned memory, and the raw arcs are freed.
hb_status compress_chunks(hb_ctx* c) {
  const int64_t nch = (int64_t)c->chunks.size();
  std::vector<std::vector<uint8_t>> bytes((size_t)nch);
  std::vector<std::vector<uint32_t>> boff((size_t)nch);
  bool too_big = false;
  const int nt = (int)std::max<int64_t>(1, std::min<int64_t>(16, nch));
  std::vector<std::thread> th;
  for (int k = 0; k < nt; ++k)
    th.emplace_back([&, k] {
      for (int64_t ci = k; ci < nch; ci += nt) {
        const StreamChunk& ch = c->chunks[(size_t)ci];
        for (int64_t v = ch.r0; v < ch.r1; ++v) std::sort(c->host_idx + c->host_off[v], c->host_idx + c->host_off[v + 1]);
        std::vector<uint8_t>& out = bytes[(size_t)ci];
        std::vector<uint32_t>& bo = boff[(size_t)ci];
        out.reserve((size_t)(ch.e1 - ch.e0) * 3);
        for (int64_t e = ch.e0; e < ch.e1; e += hb::STREAM_BLOCK_ARCS) {
          bo.push_back((uint32_t)out.size());
          hb::codes::put_block<hb::STREAM_BLOCK_ARCS>(out, c->host_idx + e,
                                                      std::min<int64_t>(hb::STREAM_BLOCK_ARCS, ch.e1 - e));
        }
        bo.push_back((uint32_t)out.size());
        if (out.size() > 0xfffff000u) too_big = true;
      }
    });
  for (auto& t : th) t.join();
  if (too_big) return fail(HB_ENOMEM, "a compressed chunk exceeds 4 GiB; lower graph_budget");
  int64_t cb = 0, bo = 0, cap = 0;
  for (int64_t ci = 0; ci < nch; ++ci) {
    StreamChunk& ch = c->chunks[(size_t)ci];
    ch.nb = (int64_t)boff[(size_t)ci].size() - 1;
    ch.bo_at = bo;
    ch.cb_at = cb;
    ch.cb_len = (int64_t)bytes[(size_t)ci].size();
    bo += ch.nb + 1;
    cb += (ch.cb_len + 8 + 3) / 4 * 4;
    cap = std::max<int64_t>(cap, (int64_t)align256(sizeof(uint32_t) * (size_t)(ch.nb + 1)) + (ch.cb_len + 8 + 3) / 4 * 4);
  }
  HB_HIP(hipHostMalloc(reinterpret_cast<void**>(&c->host_cbytes), (size_t)std::max<int64_t>(cb, 4), hipHostMallocDefault));
  HB_HIP(hipHostMalloc(reinterpret_cast<void**>(&c->host_boff), sizeof(uint32_t) * (size_t)std::max<int64_t>(bo, 1),
                       hipHostMallocDefault));
  for (int64_t ci = 0; ci < nch; ++ci) {
    const StreamChunk& ch = c->chunks[(size_t)ci];
    std::memcpy(c->host_cbytes + ch.cb_at, bytes[(size_t)ci].data(), (size_t)ch.cb_len);
    std::memset(c->host_cbytes + ch.cb_at + ch.cb_len, 0, (size_t)((ch.cb_len + 8 + 3) / 4 * 4 - ch.cb_len));
    std::memcpy(c->host_boff + ch.bo_at, boff[(size_t)ci].data(), sizeof(uint32_t) * (size_t)(ch.nb + 1));
  }
  c->cstage_bytes = std::max<int64_t>(cap, 256);
  c->compressed = true;
  c->host_graph_bytes = (int64_t)sizeof(int64_t) * (c->n + 1) + cb + (int64_t)sizeof(uint32_t) * bo;
  // the raw arcs are no longer needed on the host
  (void)hipHostFree(c->host_idx);
  c->host_idx = nullptr;
  return HB_OK;
}

// A streamed graph (paper Sec. 5.1: the graph is read from outside the
// memory that holds the counters): a pinned host copy of the CSR, row lists
// built on the host, and row chunks that fit a staging buffer.  Device
// memory holds the lists, two staging buffers, and per node a mask of the
// chunks with an arc into it (built while the first pass streams every
// chunk) for chunk selection in later passes.
hb_status setup_streamed(hb_ctx* c, const hb_csr* g) {
  const int64_t n = c->n, m = c->m;
  if (c->opt.validate) {
    const int bad = g->offsets_bits == 64
                        ? host_csr_check(static_cast<const int64_t*>(g->offsets), g->indices, n, m)
                        : host_csr_check(static_cast<const int32_t*>(g->offsets), g->indices, n, m);
    if (bad == 1) return fail(HB_EINVAL, "malformed CSR offsets (need offsets[0]=0, nondecreasing, offsets[n]=m)");
    if (bad == 2) return fail(HB_EINVAL, "CSR index outside [0, n)");
  }
  HB_HIP(hipHostMalloc(reinterpret_cast<void**>(&c->host_off), sizeof(int64_t) * (size_t)(n + 1),
                       hipHostMallocDefault));
  HB_HIP(hipHostMalloc(reinterpret_cast<void**>(&c->host_idx), sizeof(int32_t) * (size_t)(m > 0 ? m : 1),
                       hipHostMallocDefault));
  if (g->offsets_bits == 64) {
    std::memcpy(c->host_off, g->offsets, sizeof(int64_t) * (size_t)(n + 1));
  } else {
    const int32_t* o = static_cast<const int32_t*>(g->offsets);
    for (int64_t v = 0; v <= n; ++v) c->host_off[v] = o[v];
  }
  {  // the arc copy in parallel slices (it is the bulk of the graph)
    const int nt = (int)std::max<int64_t>(1, std::min<int64_t>(16, m >> 24));
    std::vector<std::thread> th;
    for (int k = 0; k < nt; ++k)
      th.emplace_back([=] {
        const int64_t a = m * k / nt, b = m * (k + 1) / nt;
        if (b > a) std::memcpy(c->host_idx + a, g->indices + a, sizeof(int32_t) * (size_t)(b - a));
      });
    for (auto& t : th) t.join();
  }
  std::vector<int32_t> light, medium;
  std::vector<hb::HeavyItem> items;
  std::vector<hb::HeavyRow> hrows;
  plan_rows_host(c->host_off, n, c->opt.light_max, c->opt.heavy_min, c->opt.chunk, light, medium, items, hrows);
  // Chunks: consecutive rows while their offsets (256-byte aligned) and arcs
  // fit one staging buffer.
  const int64_t cap = (c->opt.graph_budget > 0 ? c->opt.graph_budget / 2 : DEFAULT_CHUNK_BYTES) / 256 * 256;
  c->chunk_bytes = cap;
  auto bytes_of = [&](int64_t r0, int64_t r1) {
    return (int64_t)align256(sizeof(int64_t) * (size_t)(r1 - r0 + 1)) +
           (int64_t)sizeof(int32_t) * (c->host_off[r1] - c->host_off[r0]);
  };
  for (int64_t r0 = 0; r0 < n;) {
    if (bytes_of(r0, r0 + 1) > cap)
      return fail(HB_ENOMEM, "row " + std::to_string(r0) + " has " + std::to_string(c->host_off[r0 + 1] - c->host_off[r0]) +
                                 " arcs, more than a staging buffer of " + std::to_string(cap) + " bytes holds");
    // largest r1 with bytes_of(r0, r1) <= cap (monotone in r1)
    int64_t lo = r0 + 1, hi = n;
    while (lo < hi) {
      const int64_t mid = lo + (hi - lo + 1) / 2;
      if (bytes_of(r0, mid) <= cap) lo = mid; else hi = mid - 1;
    }
    StreamChunk ch{};
    ch.r0 = r0;
    ch.r1 = lo;
    ch.e0 = c->host_off[r0];
    ch.e1 = c->host_off[lo];
    c->chunks.push_back(ch);
    r0 = lo;
  }
  // Each chunk's entries of the (row-sorted) lists; heavy rows name their
  // first item relative to the chunk's first item, as a chunk's items are
  // numbered from 0 in its launch.
  for (StreamChunk& ch : c->chunks) {
    auto rows_lb = [](const std::vector<int32_t>& v, int64_t r) {
      return (int64_t)(std::lower_bound(v.begin(), v.end(), r, [](int32_t a, int64_t b) { return a < b; }) - v.begin());
    };
    ch.l0 = rows_lb(light, ch.r0);
    ch.l1 = rows_lb(light, ch.r1);
    ch.m0 = rows_lb(medium, ch.r0);
    ch.m1 = rows_lb(medium, ch.r1);
    auto item_lb = [&](int64_t r) {
      return (int64_t)(std::lower_bound(items.begin(), items.end(), r,
                                        [](const hb::HeavyItem& a, int64_t b) { return a.row < b; }) - items.begin());
    };
    auto hrow_lb = [&](int64_t r) {
      return (int64_t)(std::lower_bound(hrows.begin(), hrows.end(), r,
                                        [](const hb::HeavyRow& a, int64_t b) { return a.row < b; }) - hrows.begin());
    };
    ch.i0 = item_lb(ch.r0);
    ch.i1 = item_lb(ch.r1);
    ch.h0 = hrow_lb(ch.r0);
    ch.h1 = hrow_lb(ch.r1);
    for (int64_t h = ch.h0; h < ch.h1; ++h) hrows[(size_t)h].item0 -= ch.i0;
  }
  hb_status st = upload_plan(c, light, medium, items, hrows);
  if (st != HB_OK) return st;
  c->host_graph_bytes = (int64_t)sizeof(int64_t) * (n + 1) + (int64_t)sizeof(int32_t) * m;
  if (c->opt.stream_compress) {
    st = compress_chunks(c);
    if (st != HB_OK) return st;
  }
  const int32_t nch = (int32_t)c->chunks.size();
  std::vector<int64_t> first((size_t)nch + 1, n);
  for (int32_t i = 0; i < nch; ++i) first[(size_t)i] = c->chunks[(size_t)i].r0;
  HB_HIP(dmalloc(&c->chunk_rows, first.size()));
  HB_HIP(hipMemcpyAsync(c->chunk_rows, first.data(), sizeof(int64_t) * first.size(), hipMemcpyHostToDevice,
                        c->stream));
  HB_HIP(dmalloc(&c->pred_mask, (size_t)(n > 0 ? n : 1)));
  HB_HIP(hb::launch_fill_zero(c->pred_mask, sizeof(uint32_t) * (size_t)(n > 0 ? n : 1), c->stream));
  HB_HIP(dmalloc(&c->chunk_act, 1));
  HB_HIP(hipHostMalloc(reinterpret_cast<void**>(&c->chunk_act_host), sizeof(uint32_t), hipHostMallocDefault));
  for (int i = 0; i < 2; ++i) {
    if (dmalloc(&c->stage[i], (size_t)cap) != hipSuccess)
      return fail(HB_ENOMEM, "cannot allocate a staging buffer of " + std::to_string(cap) + " bytes");
    if (c->compressed && dmalloc(&c->cstage[i], (size_t)c->cstage_bytes) != hipSuccess)
      return fail(HB_ENOMEM, "cannot allocate a compressed staging buffer of " + std::to_string(c->cstage_bytes) +
                                 " bytes");
    HB_HIP(hipEventCreateWithFlags(&c->up_ev[i], hipEventDisableTiming));
    HB_HIP(hipEventCreateWithFlags(&c->done_ev[i], hipEventDisableTiming));
    HB_HIP(hipEventRecord(c->done_ev[i], c->stream));
  }
  HB_HIP(hipStreamCreateWithFlags(&c->copy_stream, hipStreamNonBlocking));
  HB_HIP(hipStreamSynchronize(c->stream));  // the chunk table above is read from the host
  c->n_nonempty = c->n_light + c->n_medium + c->n_hrows;
  return HB_OK;
}

// One pass of a streamed graph: the chunks that can have work (every chunk in
// first and dense passes), each uploaded on the copy stream into the staging
// buffer the chunk before last used, once that chunk's kernels are done, and
// run on the context stream once its upload is done.  The pass kernels see
// the chunk's offsets and arcs at their global indices.
hipError_t streamed_pass(hb_ctx* c, const hb::PassArgs& a, bool timing, hb_pass_info& info) {
  const int32_t nch = (int32_t)c->chunks.size();
  const size_t half = (size_t)hb::STAT_SLOTS * hb::STAT_K;
  hipError_t e = hb::launch_fill_zero(a.stats, sizeof(unsigned long long) * half, c->stream);
  uint32_t sel = 0xffffffffu;
  const bool all = a.mode == hb::MODE_FIRST || a.mode == hb::MODE_DENSE || !c->masks_ready;
  if (!all) {
    if (e == hipSuccess)
      e = hb::launch_chunk_activity(a.mod_prev, c->n_blocks, c->pred_mask, c->chunk_rows, nch, c->chunk_act,
                                    c->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(c->chunk_act_host, c->chunk_act, sizeof(uint32_t), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return e;
    sel = *c->chunk_act_host;
  }
  if (e == hipSuccess && timing) e = hipEventRecord(c->ev[1], c->stream);
  const bool build_masks = !c->masks_ready;
  int k = 0;
  for (int32_t ci = 0; ci < nch && e == hipSuccess; ++ci) {
    if (!((sel >> (ci & 31)) & 1u)) continue;
    const StreamChunk& ch = c->chunks[(size_t)ci];
    const int s = k & 1;
    ++k;
    int64_t* soff = reinterpret_cast<int64_t*>(c->stage[s]);
    const size_t obytes = sizeof(int64_t) * (size_t)(ch.r1 - ch.r0 + 1);
    int32_t* sidx = reinterpret_cast<int32_t*>(c->stage[s] + align256(obytes));
    const size_t ibytes = sizeof(int32_t) * (size_t)(ch.e1 - ch.e0);
    e = hipStreamWaitEvent(c->copy_stream, c->done_ev[s], 0);
    if (e == hipSuccess) e = hipMemcpyAsync(soff, c->host_off + ch.r0, obytes, hipMemcpyHostToDevice, c->copy_stream);
    size_t sent = obytes;
    uint32_t* cboff = nullptr;
    uint8_t* cbytes = nullptr;
    if (c->compressed) {
      cboff = reinterpret_cast<uint32_t*>(c->cstage[s]);
      cbytes = c->cstage[s] + align256(sizeof(uint32_t) * (size_t)(ch.nb + 1));
      const size_t bbytes = sizeof(uint32_t) * (size_t)(ch.nb + 1);
      const size_t cb = (size_t)((ch.cb_len + 8 + 3) / 4 * 4);  // with the zero padding
      if (e == hipSuccess) e = hipMemcpyAsync(cboff, c->host_boff + ch.bo_at, bbytes, hipMemcpyHostToDevice, c->copy_stream);
      if (e == hipSuccess && cb)
        e = hipMemcpyAsync(cbytes, c->host_cbytes + ch.cb_at, cb, hipMemcpyHostToDevice, c->copy_stream);
      sent += bbytes + cb;
    } else {
      if (e == hipSuccess && ibytes)
        e = hipMemcpyAsync(sidx, c->host_idx + ch.e0, ibytes, hipMemcpyHostToDevice, c->copy_stream);
      sent += ibytes;
    }
    if (e == hipSuccess) e = hipEventRecord(c->up_ev[s], c->copy_stream);
    if (e == hipSuccess) e = hipStreamWaitEvent(c->stream, c->up_ev[s], 0);
    if (e == hipSuccess && c->compressed) e = hb::launch_decode_chunk(cboff, cbytes, ch.e1 - ch.e0, sidx, c->stream);
    hb::PassArgs b = a;
    b.off = soff - ch.r0;
    b.idx = sidx - ch.e0;
    b.light = c->light + ch.l0;
    b.n_light = ch.l1 - ch.l0;
    b.medium = c->medium + ch.m0;
    b.n_medium = ch.m1 - ch.m0;
    b.items = c->items + ch.i0;
    b.n_items = ch.i1 - ch.i0;
    b.hrows = c->hrows + ch.h0;
    b.n_hrows = ch.h1 - ch.h0;
    if (e == hipSuccess) e = hb::launch_pass(c->b, b, c->stream, nullptr);
    if (e == hipSuccess && build_masks)
      e = hb::launch_pred_masks(sidx, ch.e1 - ch.e0, 1u << (ci & 31), c->pred_mask, c->stream);
    if (e == hipSuccess) e = hipEventRecord(c->done_ev[s], c->stream);
    info.host_bytes += (int64_t)sent;
    info.chunks_run += 1;
  }
  if (e == hipSuccess && build_masks) c->masks_ready = true;
  if (e == hipSuccess && timing) e = hipEventRecord(c->ev[2], c->stream);
  return e;
}

hb_status init_impl(hb_ctx* c, const hb_csr* g, int32_t log2m, uint64_t seed, const hb_options* opt,
                    void* stream, const std::vector<int32_t>* blk_graph = nullptr) {
  c->n = g->n;
  c->m = g->m;
  c->b = log2m + c->seg_log;  // row width (one counter, or an ensemble's K counters)
  c->p = 1 << c->b;
  c->b_seed = log2m;
  c->stream = reinterpret_cast<hipStream_t>(stream);
  if (opt)
    c->opt = *opt;
  else
    hb_default_options(&c->opt);
  if (c->opt.light_max <= 0) c->opt.light_max = DEFAULT_LIGHT_MAX;
  if (c->opt.heavy_min <= 0) c->opt.heavy_min = DEFAULT_HEAVY_MIN;
  if (c->opt.chunk <= 0) c->opt.chunk = DEFAULT_CHUNK;
  if (c->opt.dense_pct < 0) c->opt.dense_pct = DEFAULT_DENSE_PCT;
  if (c->opt.sparse_pct < 0) c->opt.sparse_pct = DEFAULT_SPARSE_PCT;
  if (c->opt.heavy_min <= c->opt.light_max) c->opt.heavy_min = c->opt.light_max + 1;
  const int64_t n = c->n, m = c->m;
  c->n_blocks = (n + 63) / 64;

  // A host CSR is streamed on request, or when it exceeds the graph budget.
  const int64_t csr_bytes = 8 * (n + 1) + 4 * m;
  if (c->opt.stream_graph > 0 ||
      (c->opt.stream_graph == 0 && !g->on_device && c->opt.graph_budget > 0 && csr_bytes > c->opt.graph_budget)) {
    if (g->on_device) return fail(HB_EINVAL, "a streamed graph needs a host CSR (on_device = 0)");
    if (c->n_seeds != 1 || blk_graph) return fail(HB_EINVAL, "graph streaming needs a single-graph, single-seed context");
    if (c->p > 256) return fail(HB_EINVAL, "graph streaming needs log2m <= 8");
    c->streamed = true;
    const hb_status st = setup_streamed(c, g);
    if (st != HB_OK) return st;
  }

  // Graph arrays (int32 offsets are widened on the device).
  if (c->streamed) {
    // the arcs stay in host memory (setup_streamed)
  } else if (!g->on_device) {
    HB_HIP(dmalloc(&c->off, (size_t)n + 1));
    c->own_off = true;
    if (g->offsets_bits == 64) {
      HB_HIP(hipMemcpyAsync(c->off, g->offsets, sizeof(int64_t) * ((size_t)n + 1), hipMemcpyHostToDevice,
                            c->stream));
    } else {
      int32_t* o32 = nullptr;
      HB_HIP(dmalloc(&o32, (size_t)n + 1));
      hipError_t e = hipMemcpyAsync(o32, g->offsets, sizeof(int32_t) * ((size_t)n + 1), hipMemcpyHostToDevice,
                                    c->stream);
      if (e == hipSuccess) e = hb::launch_widen_offsets(o32, c->off, n + 1, c->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
      (void)hipFree(o32);
      if (e != hipSuccess) return fail(HB_EDEVICE, std::string("offsets upload: ") + hipGetErrorString(e));
    }
    HB_HIP(dmalloc(&c->idx_owned, (size_t)m));
    if (m > 0)
      HB_HIP(hipMemcpyAsync(c->idx_owned, g->indices, sizeof(int32_t) * (size_t)m, hipMemcpyHostToDevice,
                            c->stream));
    c->idx = c->idx_owned;
  } else {
    if (g->offsets_bits == 64) {
      c->off = const_cast<int64_t*>(static_cast<const int64_t*>(g->offsets));
    } else {
      HB_HIP(dmalloc(&c->off, (size_t)n + 1));
      c->own_off = true;
      HB_HIP(hb::launch_widen_offsets(static_cast<const int32_t*>(g->offsets), c->off, n + 1, c->stream));
    }
    c->idx = g->indices;
  }

  if (c->opt.validate && !c->streamed) {
    HB_HIP(dmalloc(&c->bad, 1));
    HB_HIP(hipMemsetAsync(c->bad, 0, sizeof(int), c->stream));
    HB_HIP(hb::launch_validate(c->off, c->idx, n, m, c->bad, c->stream));
    int bad = 0;
    HB_HIP(hipMemcpyAsync(&bad, c->bad, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    HB_HIP(hipStreamSynchronize(c->stream));
    if (bad & 1) return fail(HB_EINVAL, "malformed CSR offsets (need offsets[0]=0, nondecreasing, offsets[n]=m)");
    if (bad & 2) return fail(HB_EINVAL, "CSR index outside [0, n)");
  }
  if (c->streamed) {
    // row lists made by setup_streamed
  } else if (n <= HOST_PLAN_MAX) {
    // Small graphs: one pass over the offsets on the host costs less than the
    // device planner's scratch allocation and readbacks.
    std::vector<int64_t> oh((size_t)n + 1);
    HB_HIP(hipMemcpyAsync(oh.data(), c->off, sizeof(int64_t) * ((size_t)n + 1), hipMemcpyDeviceToHost, c->stream));
    HB_HIP(hipStreamSynchronize(c->stream));
    std::vector<int32_t> light, medium;
    std::vector<hb::HeavyItem> items;
    std::vector<hb::HeavyRow> hrows;
    plan_rows_host(oh.data(), n, c->opt.light_max, c->opt.heavy_min, c->opt.chunk, light, medium, items, hrows);
    const hb_status st = upload_plan(c, light, medium, items, hrows);
    if (st != HB_OK) return st;
  } else {
    const hb_status st = plan_rows_device(c);
    if (st != HB_OK) return st;
  }
  c->n_nonempty = c->n_light + c->n_medium + c->n_hrows;

  // Reverse CSR for push activation of sparse passes (lane-group kernels only).
  if (c->opt.frontier && c->opt.push && c->p <= 256 && n > 0 && !c->streamed) {
    if (dmalloc(&c->roff, (size_t)n + 1) != hipSuccess || dmalloc(&c->ridx, (size_t)m) != hipSuccess ||
        dmalloc(&c->act, (size_t)n) != hipSuccess ||
        dmalloc(&c->push_items, (size_t)n + (size_t)(m / hb::PUSH_CHUNK) + 1) != hipSuccess ||
        dmalloc(&c->push_count, 1) != hipSuccess)
      return fail(HB_ENOMEM, "cannot allocate the reverse CSR");
    HB_HIP(hb::build_reverse(c->off, c->idx, n, m, c->roff, c->ridx, c->stream));
    if (c->opt.pairs && !blk_graph) {
      const hb_status st = alloc_pairs(c);
      if (st != HB_OK) return st;
    }
  }

  // Counters, bitmaps, accumulators.
  const size_t cbytes = (size_t)n * (size_t)c->p;
  for (int i = 0; i < 2; ++i) {
    if (dmalloc(&c->cnt[i], cbytes) != hipSuccess)
      return fail(HB_ENOMEM, "cannot allocate counter buffers (" + std::to_string(cbytes) + " bytes each)");
    if (dmalloc(&c->mod[i], (size_t)c->n_blocks) != hipSuccess) return fail(HB_ENOMEM, "cannot allocate bitmaps");
    if (c->opt.slice && c->p <= 256 && dmalloc(&c->dmask[i], (size_t)n) != hipSuccess)
      return fail(HB_ENOMEM, "cannot allocate slice masks");
  }
  const size_t nk = (size_t)n * (size_t)c->n_seeds;
  if (dmalloc(&c->S, nk) != hipSuccess || dmalloc(&c->H, nk) != hipSuccess || dmalloc(&c->E, nk) != hipSuccess)
    return fail(HB_ENOMEM, "cannot allocate accumulators");
  const int ps = 1 << c->b_seed;  // registers per counter
  HB_HIP(dmalloc(&c->lc, (size_t)ps + 1));
  if (c->n_seeds > 1) HB_HIP(dmalloc(&c->seeds_dev, (size_t)c->n_seeds));
  if (c->opt.neighbourhood && !blk_graph && c->n_seeds == 1) {
    HB_HIP(dmalloc(&c->esum_part, (size_t)3 * ESUM_BLOCKS));
    HB_HIP(dmalloc(&c->esum_out, 5));
    HB_HIP(hb::launch_fill_zero(c->esum_out, 5 * sizeof(uint64_t), c->stream));
    HB_HIP(hipHostMalloc(reinterpret_cast<void**>(&c->esum_host), 4 * sizeof(uint64_t), hipHostMallocDefault));
  }
  HB_HIP(dmalloc(&c->partial, (size_t)c->n_items * (size_t)c->p));
  HB_HIP(dmalloc(&c->stats, (size_t)2 * hb::STAT_SLOTS * hb::STAT_K));
  HB_HIP(hipHostMalloc(reinterpret_cast<void**>(&c->stats_host),
                       sizeof(unsigned long long) * hb::STAT_SLOTS * hb::STAT_K, hipHostMallocDefault));
  for (int i = 0; i < 4; ++i) HB_HIP(hipEventCreate(&c->ev[i]));

  // Estimator constants: alpha_p p^2 and the linear-counting table p ln(p/V).
  c->alpha_pp = (alpha_for(ps) * (double)ps) * (double)ps;
  std::vector<double> lc((size_t)ps + 1, 0.0);
  for (int V = 1; V <= ps; ++V) lc[(size_t)V] = (double)ps * std::log((double)ps / (double)V);
  HB_HIP(hipMemcpyAsync(c->lc, lc.data(), sizeof(double) * lc.size(), hipMemcpyHostToDevice, c->stream));
  if (blk_graph) {
    // Multi-graph context: per-graph state, block map and device pass control.
    HB_HIP(dmalloc(&c->graphs, c->graphs_host.size()));
    HB_HIP(dmalloc(&c->blk_graph, blk_graph->size()));
    if (!blk_graph->empty())
      HB_HIP(hipMemcpyAsync(c->blk_graph, blk_graph->data(), sizeof(int32_t) * blk_graph->size(),
                            hipMemcpyHostToDevice, c->stream));
    if (c->n_light > 0) {
      HB_HIP(dmalloc(&c->chunk_graph, (size_t)((c->n_light + 63) / 64)));
      HB_HIP(hb::launch_chunk_graph(c->light, c->n_light, c->blk_graph, c->chunk_graph, c->stream));
    }
    HB_HIP(dmalloc(&c->ctl, 1));
    HB_HIP(hipHostMalloc(reinterpret_cast<void**>(&c->ctl_host), sizeof(hb::PassCtl), hipHostMallocDefault));
    std::memset(c->ctl_host, 0, sizeof(hb::PassCtl));
    hb::PassCtl& k = *c->ctl_host;
    k.listed_rows = c->n_nonempty;
    k.arcs = c->m;
    k.frontier = c->opt.frontier;
    k.dense_pct = c->opt.dense_pct;
    k.sparse_pct = c->opt.sparse_pct;
    k.has_reverse = c->roff ? 1 : 0;
    k.n_graphs = c->n_graphs;
    HB_HIP(dmalloc(&c->arena_tmp, (size_t)n));
    int dev = 0;
    HB_HIP(hipGetDevice(&dev));
    hipDeviceProp_t prop;
    HB_HIP(hipGetDeviceProperties(&prop, dev));
    c->persist_wgs = prop.multiProcessorCount * (c->opt.wgs_per_cu > 0 ? c->opt.wgs_per_cu : 5);
    c->graph_passes = c->opt.graph_passes > 0 ? c->opt.graph_passes : 4;
  }
  hb_status st = do_reset(c, seed);
  if (st != HB_OK) return st;
  HB_HIP(hipStreamSynchronize(c->stream));  // host staging vectors die here
  return HB_OK;
}

}  // namespace

namespace hbh {

// Arguments of a device-driven pass (buffers, mode and pass index are
// resolved on the device from ctl).
hb::PassArgs device_args(hb_ctx* c) {
  hb::PassArgs a{};
  a.off = c->off;
  a.idx = c->idx;
  a.S = c->S;
  a.H = c->H;
  a.E = c->E;
  a.lc = c->lc;
  a.light = c->light;
  a.medium = c->medium;
  a.items = c->items;
  a.hrows = c->hrows;
  a.partial = c->partial;
  a.act = c->act;
  a.roff = c->roff;
  a.ridx = c->ridx;
  a.alpha_pp = c->alpha_pp;
  a.n = c->n;
  a.n_blocks = c->n_blocks;
  a.n_light = c->n_light;
  a.n_medium = c->n_medium;
  a.n_items = c->n_items;
  a.n_hrows = c->n_hrows;
  a.qdense = c->opt.qdense ? 1 : 0;
  a.singletons = c->singletons ? 1 : 0;  // device-driven: used only when the pass is a first pass
  a.blk_graph = c->blk_graph;
  a.chunk_graph = c->chunk_graph;
  a.graphs = c->graphs;
  a.ctl = c->ctl;
  a.cntb[0] = c->cnt[0];
  a.cntb[1] = c->cnt[1];
  a.modb[0] = c->mod[0];
  a.modb[1] = c->mod[1];
  a.stats_base = c->stats;
  a.n_graphs = c->n_graphs;
  return a;
}

hb_status read_ctl(hb_ctx* c) {
  HB_HIP(hipMemcpyAsync(c->ctl_host, c->ctl, sizeof(hb::PassCtl), hipMemcpyDeviceToHost, c->stream));
  HB_HIP(hipStreamSynchronize(c->stream));
  c->t = c->ctl_host->t;
  c->converged = c->ctl_host->n_done >= c->n_graphs;
  return HB_OK;
}

}  // namespace hbh

namespace {

// Passes of a multi-graph context until every graph converged (or
// max_passes engine passes ran): replays of a hipGraph holding graph_passes
// device-driven passes, one 64-byte readback per replay.  Passes after a
// graph converged skip its rows, so overshooting is harmless; with a pass
// cap the passes are enqueued one by one instead.
hb_status multi_run(hb_ctx* c, int32_t max_passes) {
  hb_status st = read_ctl(c);
  if (st != HB_OK) return st;
  const hb::PassArgs a = device_args(c);
  if (max_passes > 0) {
    while (!c->converged && c->t < max_passes) {
      HB_HIP(hb::launch_device_pass(c->b, a, c->persist_wgs, c->push_items, c->push_count, c->n, c->stream));
      st = read_ctl(c);
      if (st != HB_OK) return st;
    }
    return HB_OK;
  }
  if (!c->gexec) {
    hipGraph_t graph = nullptr;
    HB_HIP(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int k = 0; k < c->graph_passes && e == hipSuccess; ++k)
      e = hb::launch_device_pass(c->b, a, c->persist_wgs, c->push_items, c->push_count, c->n, c->stream);
    const hipError_t e2 = hipStreamEndCapture(c->stream, &graph);
    if (e != hipSuccess) return fail(HB_EDEVICE, std::string("pass capture: ") + hipGetErrorString(e));
    if (e2 != hipSuccess) return fail(HB_EDEVICE, std::string("hipStreamEndCapture: ") + hipGetErrorString(e2));
    e = hipGraphInstantiate(&c->gexec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (e != hipSuccess) return fail(HB_EDEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(e));
  }
  while (!c->converged) {
    HB_HIP(hipGraphLaunch(c->gexec, c->stream));
    st = read_ctl(c);
    if (st != HB_OK) return st;
  }
  return HB_OK;
}

hb_status multi_pack(hb_ctx* c, const double* src, double* dst, int32_t dst_on_device) {
  if (dst_on_device) return hb::launch_pack(src, dst, c->n, c->blk_graph, c->graphs, c->stream) == hipSuccess
                                ? HB_OK
                                : fail(HB_EDEVICE, "pack");
  double* tmp = c->arena_tmp;
  HB_HIP(hb::launch_pack(src, tmp, c->n, c->blk_graph, c->graphs, c->stream));
  HB_HIP(hipMemcpyAsync(dst, tmp, sizeof(double) * (size_t)c->n_packed, hipMemcpyDeviceToHost, c->stream));
  return HB_OK;
}

}  // namespace

extern "C" {

void hb_default_options(hb_options* opt) {
  if (!opt) return;
  opt->frontier = 1;
  opt->light_max = DEFAULT_LIGHT_MAX;
  opt->heavy_min = DEFAULT_HEAVY_MIN;
  opt->chunk = DEFAULT_CHUNK;
  opt->validate = 1;
  opt->timing = 0;
  opt->dense_pct = DEFAULT_DENSE_PCT;
  opt->push = 1;
  opt->sparse_pct = DEFAULT_SPARSE_PCT;
  opt->qdense = 0;
  opt->slice = 0;
  opt->wgs_per_cu = 5;
  opt->graph_passes = 4;
  opt->neighbourhood = 0;
  opt->pairs = 1;
  opt->stream_graph = 0;
  opt->graph_budget = 0;
  opt->stream_compress = 0;
}

hb_status hb_init(hb_ctx** out, const hb_csr* g, int32_t log2m, uint64_t seed, const hb_options* opt,
                  void* stream) {
  if (!out) return fail(HB_EINVAL, "out is NULL");
  *out = nullptr;
  if (!g) return fail(HB_EINVAL, "graph is NULL");
  if (log2m < 4 || log2m > 16) return fail(HB_EINVAL, "log2m must be in [4, 16]");
  if (g->n < 0 || g->m < 0) return fail(HB_EINVAL, "negative n or m");
  if (g->n > 0x7fffffffLL) return fail(HB_EINVAL, "n must fit int32 node ids");
  if (g->offsets_bits != 32 && g->offsets_bits != 64) return fail(HB_EINVAL, "offsets_bits must be 32 or 64");
  if (g->offsets_bits == 32 && g->m > 0x7fffffffLL) return fail(HB_EINVAL, "m too large for int32 offsets");
  if (!g->offsets) return fail(HB_EINVAL, "offsets is NULL");
  if (g->m > 0 && !g->indices) return fail(HB_EINVAL, "indices is NULL");
  if (opt && opt->chunk < 0) return fail(HB_EINVAL, "chunk must be >= 0");
  if (!g->on_device) {
    // Host arrays: check the CSR shape cheaply before copying.
    const bool o64 = g->offsets_bits == 64;
    const int64_t first = o64 ? static_cast<const int64_t*>(g->offsets)[0]
                              : static_cast<const int32_t*>(g->offsets)[0];
    const int64_t last = o64 ? static_cast<const int64_t*>(g->offsets)[g->n]
                             : static_cast<const int32_t*>(g->offsets)[g->n];
    if (first != 0 || last != g->m) return fail(HB_EINVAL, "offsets must start at 0 and end at m");
  }
  hb_ctx* c = new (std::nothrow) hb_ctx();
  if (!c) return fail(HB_ENOMEM, "cannot allocate context");
  const hb_status st = init_impl(c, g, log2m, seed, opt, stream);
  if (st != HB_OK) {
    const std::string msg = g_err;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    release(c);
    g_err = msg;
    return st;
  }
  *out = c;
  return HB_OK;
}

hb_status hb_reset(hb_ctx* c, uint64_t seed) {
  hb_status st = check_ctx(c);
  if (st != HB_OK) return st;
  if (c->n_seeds > 1) return fail(HB_EINVAL, "ensemble contexts restart with hb_ensemble_reset");
  st = do_reset(c, seed);
  if (st != HB_OK) c->failed = true;
  return st;
}

hb_status hb_iterate(hb_ctx* c, int64_t* n_modified) {
  hb_status st = check_ctx(c);
  if (st != HB_OK) return st;
  if (n_modified) *n_modified = 0;
  if (c->converged) return HB_OK;
  if (c->n_graphs > 0) {
    // One device-driven pass over every unconverged graph of the batch (its
    // mode was planned on the device at the end of the previous pass and read
    // back with the pass control).
    const int32_t t_before = c->t;
    const int32_t mode = c->ctl_host->mode;
    const bool timing = c->opt.timing != 0;
    if (timing) HB_HIP(hipEventRecord(c->ev[0], c->stream));
    HB_HIP(hb::launch_device_pass(c->b, device_args(c), c->persist_wgs, c->push_items, c->push_count, c->n,
                                  c->stream));
    if (timing) HB_HIP(hipEventRecord(c->ev[1], c->stream));
    st = read_ctl(c);
    if (st != HB_OK) return st;
    const size_t half = (size_t)hb::STAT_SLOTS * hb::STAT_K;
    HB_HIP(hipMemcpyAsync(c->stats_host, c->stats + (size_t)(t_before & 1) * half,
                          sizeof(unsigned long long) * half, hipMemcpyDeviceToHost, c->stream));
    HB_HIP(hipStreamSynchronize(c->stream));
    unsigned long long sum[hb::STAT_K] = {};
    for (int sl = 0; sl < hb::STAT_SLOTS; ++sl)
      for (int k = 0; k < hb::STAT_SEEDS; ++k) sum[k] += c->stats_host[sl * hb::STAT_K + k];
    hb_pass_info info{};
    info.counters_gathered = (int64_t)sum[0];
    info.rows_loaded = (int64_t)sum[1];
    info.rows_written = (int64_t)sum[2];
    info.rows_changed = (int64_t)sum[3];
    info.arcs_scanned = (int64_t)sum[4];
    info.slices_gathered = (int64_t)sum[5];
    info.slices_changed = (int64_t)sum[6];
    info.arcs_to_changed = c->roff ? (int64_t)sum[7] : -1;
    info.mode = mode;
    if (timing) {
      float ms = 0.f;
      (void)hipEventElapsedTime(&ms, c->ev[0], c->ev[1]);
      info.expand_ms = ms;
      c->total_ms += (double)ms;
    }
    c->hist.push_back(info);
    c->last_nmod = info.rows_changed;
    if (n_modified) *n_modified = info.rows_changed;
    return HB_OK;
  }
  hb_pass_info info{};
  if (c->n == 0) {
    c->hist.push_back(info);
    if (c->esum_out) c->nf.push_back(0.0);
    for (auto& sp : c->seed_passes)
      if (sp < 0) sp = c->t + 1;
    c->t += 1;
    c->converged = true;
    c->last_nmod = 0;
    return HB_OK;
  }
  // Pass mode from the previous pass's changes (all modes give identical
  // results; they differ only in the work they skip).
  int32_t mode = hb::MODE_DENSE;
  if (c->t == 0) {
    mode = hb::MODE_FIRST;
  } else if (c->opt.frontier) {
    const int64_t N = c->n_nonempty > 0 ? c->n_nonempty : 1;
    const bool lanes = c->p <= 256;
    // Share of arcs the next pass must gather: exact with the reverse CSR.
    const bool exact = lanes && c->roff && c->last_pairs >= 0;
    const bool dense = exact ? 100 * c->last_pairs >= (int64_t)c->opt.dense_pct * (c->m > 0 ? c->m : 1)
                             : 100 * c->last_nmod >= (int64_t)c->opt.dense_pct * N;
    if (dense)
      mode = hb::MODE_DENSE;
    else if (c->roff && 100 * c->last_nmod < (int64_t)c->opt.sparse_pct * N)
      mode = hb::MODE_SPARSE;
    else if (!lanes)
      mode = hb::MODE_SPARSE;  // the wide kernel visits every row in sparse passes without push
    else
      mode = c->dmask[0] ? hb::MODE_SLICE : hb::MODE_EDGE;
  }
  hb::PassArgs a{};
  a.off = c->off;
  a.idx = c->idx;
  a.cur = c->cnt[c->cur];
  a.nxt = c->cnt[c->cur ^ 1];
  a.mod_prev = c->mod[c->cur];
  a.mod_cur = c->mod[c->cur ^ 1];
  a.dmask_prev = c->dmask[c->cur];
  a.dmask_cur = c->dmask[c->cur ^ 1];
  a.S = c->S;
  a.H = c->H;
  a.E = c->E;
  a.lc = c->lc;
  a.light = c->light;
  a.medium = c->medium;
  a.items = c->items;
  a.hrows = c->hrows;
  a.partial = c->partial;
  a.act = (mode == hb::MODE_SPARSE) ? c->act : nullptr;
  a.roff = c->roff;
  const size_t half = (size_t)hb::STAT_SLOTS * hb::STAT_K;
  a.stats = c->stats + (size_t)(c->t & 1) * half;
  a.stats_next = c->stats + (size_t)((c->t + 1) & 1) * half;
  a.alpha_pp = c->alpha_pp;
  a.d = (double)(c->t + 1);
  a.n = c->n;
  a.n_blocks = c->n_blocks;
  a.n_light = c->n_light;
  a.n_medium = c->n_medium;
  a.n_items = c->n_items;
  a.n_hrows = c->n_hrows;
  a.epoch = c->t + 1;
  a.mode = mode;
  a.qdense = c->opt.qdense ? 1 : 0;
  a.seg_lanes = (1 << c->b_seed) / 16;
  a.D = c->D;
  a.singletons = (mode == hb::MODE_FIRST && c->singletons) ? 1 : 0;
  a.seed = c->seed;
  a.disc_f = c->disc.empty() ? 0.0 : c->disc[(size_t)std::min<int64_t>(c->t, (int64_t)c->disc.size() - 1)];
  const bool timing = c->opt.timing != 0;
  a.ridx = c->ridx;
  // Sparse passes run from pair lists when the exact pair count (arcs into
  // the counters that changed, plus those rows) fits the lists.
  const int64_t pairs = (mode == hb::MODE_SPARSE && c->pb.cap > 0 && c->last_pairs >= 0 && c->last_nmod > 0)
                            ? c->last_pairs + c->last_nmod
                            : 0;
  const bool use_pairs = pairs > 0 && pairs <= c->pb.cap;
  if (use_pairs) a.act = nullptr;
  hipError_t e = hipSuccess;
  if (timing) e = hipEventRecord(c->ev[0], c->stream);
  if (c->streamed) {
    if (e == hipSuccess) e = hb::launch_fill_zero(a.mod_cur, sizeof(uint64_t) * (size_t)c->n_blocks, c->stream);
    if (e == hipSuccess && a.dmask_cur)
      e = hb::launch_fill_zero(a.dmask_cur, sizeof(uint16_t) * (size_t)c->n, c->stream);
    if (e == hipSuccess) e = streamed_pass(c, a, timing, info);
  }
  if (!c->streamed && e == hipSuccess && a.act)
    e = hb::launch_push(a.mod_prev, c->n_blocks, c->n, c->roff, c->ridx, c->push_items, c->push_count, c->act,
                        a.epoch, c->stream);
  if (!c->streamed) {
    if (e == hipSuccess && use_pairs)
      e = hb::launch_pair_build(a, c->pb, pairs, c->push_items, c->push_count, c->stream);
    if (e == hipSuccess) e = hb::launch_fill_zero(a.mod_cur, sizeof(uint64_t) * (size_t)c->n_blocks, c->stream);
    if (e == hipSuccess && a.dmask_cur)
      e = hb::launch_fill_zero(a.dmask_cur, sizeof(uint16_t) * (size_t)c->n, c->stream);
    if (e == hipSuccess && timing) e = hipEventRecord(c->ev[1], c->stream);
    if (e == hipSuccess)
      e = use_pairs ? hb::launch_pair_pass(c->b, a, c->pb, pairs, c->stream, timing ? c->ev[2] : nullptr)
                    : hb::launch_pass(c->b, a, c->stream, timing ? c->ev[2] : nullptr);
  }
  if (e == hipSuccess && use_pairs)
    e = hipMemcpyAsync(c->npairs_host, c->pb.npairs, sizeof(unsigned long long), hipMemcpyDeviceToHost, c->stream);
  if (e == hipSuccess && timing) e = hipEventRecord(c->ev[3], c->stream);
  if (e == hipSuccess && c->esum_out) e = enqueue_esum(c);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->stats_host, a.stats, sizeof(unsigned long long) * half, hipMemcpyDeviceToHost,
                       c->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
  if (e != hipSuccess) {
    c->failed = true;
    return fail(HB_EDEVICE, std::string("pass ") + std::to_string(c->t) + ": " + hipGetErrorString(e));
  }
  if (use_pairs && *c->npairs_host != (unsigned long long)pairs) {
    c->failed = true;
    return fail(HB_EDEVICE, "pass " + std::to_string(c->t) + ": " + std::to_string(*c->npairs_host) +
                                " pairs emitted, " + std::to_string(pairs) + " planned");
  }
  unsigned long long sum[hb::STAT_K] = {};
  unsigned long long seeds_changed = 0;
  for (int s = 0; s < hb::STAT_SLOTS; ++s) {
    for (int k = 0; k < hb::STAT_SEEDS; ++k) sum[k] += c->stats_host[s * hb::STAT_K + k];
    seeds_changed |= c->stats_host[s * hb::STAT_K + hb::STAT_SEEDS];
  }
  // A seed's run ends with its first pass that changes none of its counters.
  for (int k = 0; k < c->n_seeds && c->n_seeds > 1; ++k)
    if (c->seed_passes[(size_t)k] < 0 && !((seeds_changed >> k) & 1ull)) c->seed_passes[(size_t)k] = c->t + 1;
  info.counters_gathered = (int64_t)sum[0];
  info.rows_loaded = (int64_t)sum[1];
  info.rows_written = (int64_t)sum[2];
  info.rows_changed = (int64_t)sum[3];
  info.arcs_scanned = (int64_t)sum[4];
  info.slices_gathered = (int64_t)sum[5];
  info.slices_changed = (int64_t)sum[6];
  info.arcs_to_changed = c->roff ? (int64_t)sum[7] : -1;
  info.mode = mode;
  info.path = use_pairs ? 2 : (a.singletons && c->p <= 256 && !a.D ? 1 : 0);
  if (timing) {
    float ms0 = 0.f, ms1 = 0.f, ms2 = 0.f;
    (void)hipEventElapsedTime(&ms0, c->ev[0], c->ev[1]);
    (void)hipEventElapsedTime(&ms1, c->ev[1], c->ev[2]);
    (void)hipEventElapsedTime(&ms2, c->ev[2], c->ev[3]);
    info.push_ms = ms0;
    info.expand_ms = ms1;
    info.merge_ms = ms2;
    c->total_ms += (double)ms0 + (double)ms1 + (double)ms2;
  }
  if (c->esum_out) {
    const hb_status es = take_esum(c);
    if (es != HB_OK) {
      c->failed = true;
      return es;
    }
  }
  c->hist.push_back(info);
  c->cur ^= 1;
  c->t += 1;
  c->last_nmod = info.rows_changed;
  c->last_slices = info.slices_changed;
  c->last_pairs = info.arcs_to_changed;
  if (info.rows_changed == 0) c->converged = true;
  if (n_modified) *n_modified = info.rows_changed;
  return HB_OK;
}

hb_status hb_run(hb_ctx* c, int32_t max_passes, int32_t* passes) {
  hb_status st = check_ctx(c);
  if (st != HB_OK) return st;
  if (c->n_graphs > 0) {
    st = multi_run(c, max_passes);
    if (st != HB_OK) {
      c->failed = true;
      return st;
    }
    if (passes) *passes = c->t;
    return HB_OK;
  }
  while (!c->converged && (max_passes <= 0 || c->t < max_passes)) {
    st = hb_iterate(c, nullptr);
    if (st != HB_OK) return st;
  }
  if (passes) *passes = c->t;
  return HB_OK;
}

hb_status hb_centralities(hb_ctx* c, double* closeness, double* lin, double* harmonic, double* coreach,
                          int32_t dst_on_device) {
  hb_status st = check_ctx(c);
  if (st != HB_OK) return st;
  if (c->n == 0) return HB_OK;
  // Single graphs finalise straight into device destinations; batched
  // contexts always go through the arena-layout staging below and are packed.
  const int64_t nk = c->n * c->n_seeds;  // values per output (ensembles: K per node)
  if (dst_on_device && c->n_graphs == 0) {
    HB_HIP(hb::launch_finalize(nk, c->S, c->H, c->E, closeness, lin, harmonic, coreach, c->stream));
    HB_HIP(hipStreamSynchronize(c->stream));
    return HB_OK;
  }
  const size_t n = (size_t)nk;
  if (!c->out_tmp) {
    if (dmalloc(&c->out_tmp, 4 * n) != hipSuccess) return fail(HB_ENOMEM, "cannot allocate output staging");
  }
  double* d[4] = {c->out_tmp, c->out_tmp + n, c->out_tmp + 2 * n, c->out_tmp + 3 * n};
  double* h[4] = {closeness, lin, harmonic, coreach};
  if (c->n_graphs > 0) {
    // Arena-layout results, then packed graph by graph (padding dropped).
    HB_HIP(hb::launch_finalize(c->n, c->S, c->H, c->E, d[0], d[1], d[2], d[3], c->stream));
    for (int i = 0; i < 4; ++i) {
      if (!h[i]) continue;
      if (dst_on_device) {
        HB_HIP(hb::launch_pack(d[i], h[i], c->n, c->blk_graph, c->graphs, c->stream));
      } else {
        HB_HIP(hb::launch_pack(d[i], c->arena_tmp, c->n, c->blk_graph, c->graphs, c->stream));
        HB_HIP(hipMemcpyAsync(h[i], c->arena_tmp, sizeof(double) * (size_t)c->n_packed, hipMemcpyDeviceToHost,
                              c->stream));
        HB_HIP(hipStreamSynchronize(c->stream));
      }
    }
    HB_HIP(hipStreamSynchronize(c->stream));
    return HB_OK;
  }
  HB_HIP(hb::launch_finalize(nk, c->S, c->H, c->E, h[0] ? d[0] : nullptr, h[1] ? d[1] : nullptr,
                             h[2] ? d[2] : nullptr, h[3] ? d[3] : nullptr, c->stream));
  for (int i = 0; i < 4; ++i)
    if (h[i]) HB_HIP(hipMemcpyAsync(h[i], d[i], sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
  HB_HIP(hipStreamSynchronize(c->stream));
  return HB_OK;
}

hb_status hb_get_registers(hb_ctx* c, uint8_t* dst, int32_t dst_on_device) {
  hb_status st = check_ctx(c);
  if (st != HB_OK) return st;
  if (!dst) return fail(HB_EINVAL, "dst is NULL");
  const size_t bytes = (size_t)c->n * (size_t)c->p;
  if (bytes == 0) return HB_OK;
  if (c->n_graphs > 0) {
    const uint8_t* src = c->cnt[c->ctl_host->parity];
    if (dst_on_device) {
      HB_HIP(hb::launch_pack_u8(src, dst, c->n, c->p, c->blk_graph, c->graphs, c->stream));
    } else {
      uint8_t* tmp = nullptr;
      if (dmalloc(&tmp, (size_t)c->n_packed * (size_t)c->p) != hipSuccess)
        return fail(HB_ENOMEM, "cannot allocate register staging");
      hipError_t e = hb::launch_pack_u8(src, tmp, c->n, c->p, c->blk_graph, c->graphs, c->stream);
      if (e == hipSuccess)
        e = hipMemcpyAsync(dst, tmp, (size_t)c->n_packed * (size_t)c->p, hipMemcpyDeviceToHost, c->stream);
      if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
      (void)hipFree(tmp);
      if (e != hipSuccess) return fail(HB_EDEVICE, std::string("registers: ") + hipGetErrorString(e));
    }
    HB_HIP(hipStreamSynchronize(c->stream));
    return HB_OK;
  }
  HB_HIP(hipMemcpyAsync(dst, c->cnt[c->cur], bytes,
                        dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
  HB_HIP(hipStreamSynchronize(c->stream));
  return HB_OK;
}

hb_status hb_get_accumulators(hb_ctx* c, double* S, double* H, int32_t dst_on_device) {
  hb_status st = check_ctx(c);
  if (st != HB_OK) return st;
  const size_t bytes = sizeof(double) * (size_t)c->n * (size_t)c->n_seeds;
  if (bytes == 0) return HB_OK;
  if (c->n_graphs > 0) {
    if (S) {
      st = multi_pack(c, c->S, S, dst_on_device);
      if (st != HB_OK) return st;
    }
    if (H) {
      HB_HIP(hipStreamSynchronize(c->stream));
      st = multi_pack(c, c->H, H, dst_on_device);
      if (st != HB_OK) return st;
    }
    HB_HIP(hipStreamSynchronize(c->stream));
    return HB_OK;
  }
  const hipMemcpyKind k = dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost;
  if (S) HB_HIP(hipMemcpyAsync(S, c->S, bytes, k, c->stream));
  if (H) HB_HIP(hipMemcpyAsync(H, c->H, bytes, k, c->stream));
  HB_HIP(hipStreamSynchronize(c->stream));
  return HB_OK;
}

hb_status hb_stats(hb_ctx* c, hb_stats_t* s) {
  if (!c || !s) return fail(HB_EINVAL, "NULL argument");
  s->n = c->n;
  s->m = c->m;
  s->log2m = c->b_seed;
  s->passes = c->t;
  s->converged = c->converged ? 1 : 0;
  s->last_modified = c->last_nmod;
  s->heavy_rows = c->n_hrows;
  s->heavy_chunks = c->n_items;
  s->medium_rows = c->n_medium;
  s->light_rows = c->n_light;
  s->reverse_built = c->roff ? 1 : 0;
  s->total_kernel_ms = c->total_ms;
  s->streamed = c->streamed ? 1 : 0;
  s->chunks = (int32_t)c->chunks.size();
  s->chunk_bytes = c->streamed ? c->chunk_bytes : 0;
  s->host_graph_bytes = c->streamed ? c->host_graph_bytes : 0;
  s->compressed = c->compressed ? 1 : 0;
  return HB_OK;
}

hb_status hb_pass_stats(hb_ctx* c, int32_t pass, hb_pass_info* info) {
  if (!c || !info) return fail(HB_EINVAL, "NULL argument");
  if (pass < 0 || pass >= (int32_t)c->hist.size()) return fail(HB_EINVAL, "no such pass record");
  *info = c->hist[(size_t)pass];
  return HB_OK;
}

hb_status hb_batch_init(hb_ctx** out, const hb_csr* graphs, int32_t k, int32_t log2m, const uint64_t* seeds,
                        const hb_options* opt, void* stream) {
  if (!out) return fail(HB_EINVAL, "out is NULL");
  *out = nullptr;
  if (!graphs || !seeds || k <= 0) return fail(HB_EINVAL, "need k >= 1 graphs and k seeds");
  if (log2m < 4 || log2m > 8) return fail(HB_EINVAL, "batched contexts need log2m in [4, 8]");
  // Arena: graph i owns nodes [base_i, base_i + n_i), padded to a multiple of
  // 64 so that no 64-node block spans two graphs; arcs are concatenated.
  std::vector<hb::GraphDev> gh((size_t)k);
  int64_t nodes = 0, arcs = 0, packed = 0;
  for (int32_t i = 0; i < k; ++i) {
    const hb_csr& g = graphs[i];
    if (g.on_device) return fail(HB_EINVAL, "batched graphs must be host CSRs");
    if (g.n < 0 || g.m < 0 || (g.offsets_bits != 32 && g.offsets_bits != 64) || !g.offsets ||
        (g.m > 0 && !g.indices))
      return fail(HB_EINVAL, "graph " + std::to_string(i) + ": malformed CSR description");
    gh[(size_t)i].node_base = nodes;
    gh[(size_t)i].n = g.n;
    gh[(size_t)i].packed = packed;
    gh[(size_t)i].seed = seeds[i];
    gh[(size_t)i].active = 1;
    nodes += (g.n + 63) / 64 * 64;
    arcs += g.m;
    packed += g.n;
  }
  if (nodes > 0x7fffffffLL) return fail(HB_EINVAL, "batch too large for int32 node ids");
  if (nodes == 0) return fail(HB_EINVAL, "a batch needs at least one graph with nodes");
  // Left uninitialised: the fill threads write every entry, so the pages are
  // first touched in parallel (zeroing 6.9 GB on one thread cost about as
  // much as the whole fill on the 4096-graph batch), and backed by huge pages
  // where the kernel allows it (fewer page faults).
  HostArena<int64_t> off((size_t)nodes + 1);
  HostArena<int32_t> idx((size_t)(arcs > 0 ? arcs : 1));
  if (!off || !idx) return fail(HB_ENOMEM, "cannot allocate the host arena");
  std::vector<int32_t> blk((size_t)(nodes / 64));
  std::vector<int64_t> abase((size_t)k + 1, 0);
  for (int32_t i = 0; i < k; ++i) abase[(size_t)i + 1] = abase[(size_t)i] + graphs[i].m;
  off[(size_t)nodes] = arcs;
  const bool validate = !opt || opt->validate;
  // Graphs [g0, g1) into their arena ranges; returns 0, or 1 + the kind of
  // malformation (1 offsets, 2 index) of the first bad graph.
  auto fill = [&](int32_t g0, int32_t g1, int32_t* bad_graph) -> int {
    for (int32_t i = g0; i < g1; ++i) {
      const hb_csr& g = graphs[i];
      const int64_t base = gh[(size_t)i].node_base;
      const int64_t npad = (g.n + 63) / 64 * 64;
      const int64_t a = abase[(size_t)i];
      for (int64_t b = base / 64; b < (base + npad) / 64; ++b) blk[(size_t)b] = i;
      if (g.n == 0) {  // no rows: its one offset entry belongs to the next graph
        const int64_t o = g.offsets_bits == 64 ? static_cast<const int64_t*>(g.offsets)[0]
                                               : static_cast<const int32_t*>(g.offsets)[0];
        if (validate && (o != 0 || g.m != 0)) {
          *bad_graph = i;
          return 1;
        }
        continue;
      }
      int64_t prev = 0;
      for (int64_t v = 0; v <= g.n; ++v) {
        const int64_t o = g.offsets_bits == 64 ? static_cast<const int64_t*>(g.offsets)[v]
                                               : static_cast<const int32_t*>(g.offsets)[v];
        if (validate && (o < prev || o > g.m || (v == 0 && o != 0) || (v == g.n && o != g.m))) {
          *bad_graph = i;
          return 1;
        }
        prev = o;
        // entry n belongs to the next graph (or is the arena's last) when n
        // is a multiple of 64: it gets the same value there, written once
        if (v < npad) off[(size_t)(base + v)] = a + o;
      }
      for (int64_t v = g.n + 1; v < npad; ++v) off[(size_t)(base + v)] = a + g.m;
      for (int64_t e = 0; e < g.m; ++e) {
        const int32_t w = g.indices[e];
        if (validate && (w < 0 || w >= g.n)) {
          *bad_graph = i;
          return 2;
        }
        idx[(size_t)(a + e)] = (int32_t)(base + w);
      }
    }
    return 0;
  };
  // Contiguous ranges of graphs with about equal arcs, one thread each.
  unsigned nt = std::thread::hardware_concurrency();
  nt = std::max(1u, std::min({nt, 32u, (unsigned)k}));
  std::vector<int32_t> cut(nt + 1, k);
  cut[0] = 0;
  for (unsigned t = 1, i = 0; t < nt; ++t) {
    const int64_t target = (arcs + nodes) / (int64_t)nt * (int64_t)t;
    while (i < (unsigned)k && abase[i] + gh[i].node_base < target) ++i;
    cut[t] = (int32_t)i;
  }
  std::vector<int> kind(nt, 0);
  std::vector<int32_t> badg(nt, -1);
  std::vector<std::thread> pool;
  try {
    for (unsigned t = 1; t < nt; ++t)
      pool.emplace_back([&, t] { kind[t] = fill(cut[t], std::max(cut[t], cut[t + 1]), &badg[t]); });
  } catch (...) {
    for (auto& th : pool) th.join();
    return fail(HB_ENOMEM, "cannot start arena threads");
  }
  kind[0] = fill(cut[0], std::max(cut[0], cut[1]), &badg[0]);
  for (auto& th : pool) th.join();
  for (unsigned t = 0; t < nt; ++t)
    if (kind[t])
      return fail(HB_EINVAL, "graph " + std::to_string(badg[t]) +
                                 (kind[t] == 1 ? ": malformed offsets" : ": index outside [0, n)"));
  hb_ctx* c = new (std::nothrow) hb_ctx();
  if (!c) return fail(HB_ENOMEM, "cannot allocate context");
  c->n_graphs = k;
  c->graphs_host = gh;
  c->n_packed = packed;
  hipStream_t s = reinterpret_cast<hipStream_t>(stream);
  if (!s) {
    // hipGraph capture needs a stream other than the legacy default one.
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      delete c;
      return fail(HB_EDEVICE, "cannot create a stream");
    }
    c->own_stream = true;
  }
  hb_csr arena;
  arena.n = nodes;
  arena.m = arcs;
  arena.offsets = off.get();
  arena.offsets_bits = 64;
  arena.indices = idx.get();
  arena.on_device = 0;
  const hb_status st = init_impl(c, &arena, log2m, 0, opt, s, &blk);
  if (st != HB_OK) {
    const std::string msg = g_err;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    release(c);
    g_err = msg;
    return st;
  }
  *out = c;
  return HB_OK;
}

hb_status hb_batch_reset(hb_ctx* c, const uint64_t* seeds) {
  hb_status st = check_ctx(c);
  if (st != HB_OK) return st;
  if (c->n_graphs == 0) return fail(HB_EINVAL, "not a batched context");
  if (seeds)
    for (int32_t i = 0; i < c->n_graphs; ++i) c->graphs_host[(size_t)i].seed = seeds[i];
  st = do_reset(c, 0);
  if (st != HB_OK) c->failed = true;
  return st;
}

hb_status hb_batch_graph(hb_ctx* c, int32_t g, hb_graph_info* info) {
  hb_status st = check_ctx(c);
  if (st != HB_OK) return st;
  if (!info) return fail(HB_EINVAL, "info is NULL");
  if (c->n_graphs == 0 || g < 0 || g >= c->n_graphs) return fail(HB_EINVAL, "no such graph");
  hb::GraphDev gd;
  HB_HIP(hipMemcpyAsync(&gd, c->graphs + g, sizeof(gd), hipMemcpyDeviceToHost, c->stream));
  HB_HIP(hipStreamSynchronize(c->stream));
  info->n = gd.n;
  info->packed_offset = gd.packed;
  info->passes = gd.passes;
  info->converged = gd.done;
  return HB_OK;
}

hb_status hb_batch_passes(hb_ctx* c, int32_t* passes) {
  hb_status st = check_ctx(c);
  if (st != HB_OK) return st;
  if (!passes) return fail(HB_EINVAL, "passes is NULL");
  if (c->n_graphs == 0) return fail(HB_EINVAL, "not a batched context");
  std::vector<hb::GraphDev> gh((size_t)c->n_graphs);
  HB_HIP(hipMemcpyAsync(gh.data(), c->graphs, sizeof(hb::GraphDev) * gh.size(), hipMemcpyDeviceToHost, c->stream));
  HB_HIP(hipStreamSynchronize(c->stream));
  for (size_t i = 0; i < gh.size(); ++i) passes[i] = gh[i].done ? gh[i].passes : -1;
  return HB_OK;
}

hb_status hb_set_weights(hb_ctx* c, const int32_t* weights, int32_t on_device) {
  hb_status st = check_ctx(c);
  if (st != HB_OK) return st;
  if (c->n_graphs > 0 || c->n_seeds > 1) return fail(HB_EINVAL, "node weights need a single-graph, single-seed context");
  if (!weights) {
    (void)hipStreamSynchronize(c->stream);
    (void)hipFree(c->weights);
    c->weights = nullptr;
  } else if (c->n > 0) {
    if (!on_device)
      for (int64_t v = 0; v < c->n; ++v)
        if (weights[v] < 1) return fail(HB_EINVAL, "node weights must be >= 1");
    if (!c->weights) HB_HIP(dmalloc(&c->weights, (size_t)c->n));
    HB_HIP(hipMemcpyAsync(c->weights, weights, sizeof(int32_t) * (size_t)c->n,
                          on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, c->stream));
    if (on_device) {
      if (!c->bad) HB_HIP(dmalloc(&c->bad, 1));
      HB_HIP(hb::launch_fill_zero(c->bad, sizeof(int), c->stream));
      HB_HIP(hb::launch_check_weights(c->weights, c->n, c->bad, c->stream));
      int bad = 0;
      HB_HIP(hipMemcpyAsync(&bad, c->bad, sizeof(int), hipMemcpyDeviceToHost, c->stream));
      HB_HIP(hipStreamSynchronize(c->stream));
      if (bad) {
        (void)hipFree(c->weights);
        c->weights = nullptr;
        return fail(HB_EINVAL, "node weights must be >= 1");
      }
    }
    HB_HIP(hipStreamSynchronize(c->stream));  // host weights are read before returning
  }
  st = do_reset(c, c->seed);
  if (st != HB_OK) c->failed = true;
  return st;
}

hb_status hb_set_discount(hb_ctx* c, const double* f, int32_t len) {
  hb_status st = check_ctx(c);
  if (st != HB_OK) return st;
  if (c->n_graphs > 0 || c->n_seeds > 1) return fail(HB_EINVAL, "discounts need a single-graph, single-seed context");
  if (c->p > 256) return fail(HB_EINVAL, "discounts need 2^log2m <= 256");
  if (!f || len <= 0) {
    (void)hipStreamSynchronize(c->stream);
    (void)hipFree(c->D);
    c->D = nullptr;
    c->disc.clear();
  } else {
    for (int32_t i = 0; i < len; ++i)
      if (!std::isfinite(f[i])) return fail(HB_EINVAL, "discount values must be finite");
    c->disc.assign(f, f + len);
    if (!c->D) HB_HIP(dmalloc(&c->D, (size_t)(c->n > 0 ? c->n : 1)));
  }
  st = do_reset(c, c->seed);
  if (st != HB_OK) c->failed = true;
  return st;
}

hb_status hb_discount_table(int32_t kind, int32_t len, double* f) {
  if (!f || len < 1) return fail(HB_EINVAL, "need an output of at least one entry");
  for (int32_t i = 0; i < len; ++i) {
    const double d = (double)(i + 1);
    switch (kind) {
      case HB_DISCOUNT_HARMONIC: f[i] = 1.0 / d; break;
      case HB_DISCOUNT_QUADRATIC: f[i] = 1.0 / (d * d); break;
      case HB_DISCOUNT_LOGARITHMIC: f[i] = 1.0 / std::log2(d + 1.0); break;
      case HB_DISCOUNT_CONSTANT: f[i] = 1.0; break;
      default: return fail(HB_EINVAL, "unknown discount kind");
    }
  }
  return HB_OK;
}

hb_status hb_get_discounted(hb_ctx* c, double* D, int32_t dst_on_device) {
  hb_status st = check_ctx(c);
  if (st != HB_OK) return st;
  if (!D) return fail(HB_EINVAL, "D is NULL");
  if (!c->D) return fail(HB_EINVAL, "no discount set (hb_set_discount)");
  if (c->n == 0) return HB_OK;
  HB_HIP(hipMemcpyAsync(D, c->D, sizeof(double) * (size_t)c->n,
                        dst_on_device ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, c->stream));
  HB_HIP(hipStreamSynchronize(c->stream));
  return HB_OK;
}

hb_status hb_neighbourhood(hb_ctx* c, double* N, int32_t cap, int32_t* len) {
  hb_status st = check_ctx(c);
  if (st != HB_OK) return st;
  if (!c->esum_out) return fail(HB_EINVAL, "the context was not made with opt.neighbourhood = 1");
  const int32_t have = (int32_t)c->nf.size();
  if (len) *len = have;
  if (N)
    for (int32_t t = 0; t < have && t < cap; ++t) N[t] = c->nf[(size_t)t];
  return HB_OK;
}

hb_status hb_distance_stats(const double* N, int32_t len, double alpha, hb_distance_stats_t* out) {
  if (!N || !out || len < 1) return fail(HB_EINVAL, "need N with at least one entry and an output");
  const int32_t T = len - 1;
  const double pairs = N[T] - N[0];
  double num = 0.0;
  for (int32_t t = 1; t <= T; ++t) num = num + (double)t * (N[t] - N[t - 1]);
  out->pairs = pairs;
  out->average_distance = pairs > 0.0 ? num / pairs : 0.0;
  const double target = alpha * N[T];
  double eff = 0.0;
  for (int32_t t = 0; t <= T; ++t) {
    if (N[t] >= target) {
      eff = t == 0 ? 0.0 : (double)(t - 1) + (target - N[t - 1]) / (N[t] - N[t - 1]);
      break;
    }
  }
  out->effective_diameter = eff;
  return HB_OK;
}

hb_status hb_ensemble_init(hb_ctx** out, const hb_csr* g, int32_t log2m, const uint64_t* seeds, int32_t k,
                           const hb_options* opt, void* stream) {
  if (!out) return fail(HB_EINVAL, "out is NULL");
  *out = nullptr;
  if (!seeds) return fail(HB_EINVAL, "seeds is NULL");
  if (k < 2 || k > 16 || (k & (k - 1)) != 0) return fail(HB_EINVAL, "ensembles need k in {2, 4, 8, 16}");
  int seg_log = 0;
  while ((1 << seg_log) < k) ++seg_log;
  if (log2m < 4 || log2m + seg_log > 8) return fail(HB_EINVAL, "ensembles need log2m >= 4 and k * 2^log2m <= 256");
  if (!g) return fail(HB_EINVAL, "graph is NULL");
  if (g->n < 0 || g->m < 0) return fail(HB_EINVAL, "negative n or m");
  if (g->n > 0x7fffffffLL) return fail(HB_EINVAL, "n must fit int32 node ids");
  if (g->offsets_bits != 32 && g->offsets_bits != 64) return fail(HB_EINVAL, "offsets_bits must be 32 or 64");
  if (g->offsets_bits == 32 && g->m > 0x7fffffffLL) return fail(HB_EINVAL, "m too large for int32 offsets");
  if (!g->offsets) return fail(HB_EINVAL, "offsets is NULL");
  if (g->m > 0 && !g->indices) return fail(HB_EINVAL, "indices is NULL");
  if (!g->on_device) {
    const bool o64 = g->offsets_bits == 64;
    const int64_t first = o64 ? static_cast<const int64_t*>(g->offsets)[0] : static_cast<const int32_t*>(g->offsets)[0];
    const int64_t last =
        o64 ? static_cast<const int64_t*>(g->offsets)[g->n] : static_cast<const int32_t*>(g->offsets)[g->n];
    if (first != 0 || last != g->m) return fail(HB_EINVAL, "offsets must start at 0 and end at m");
  }
  hb_ctx* c = new (std::nothrow) hb_ctx();
  if (!c) return fail(HB_ENOMEM, "cannot allocate context");
  c->n_seeds = k;
  c->seg_log = seg_log;
  c->seeds.assign(seeds, seeds + k);
  c->seed_passes.assign((size_t)k, -1);
  const hb_status st = init_impl(c, g, log2m, 0, opt, stream);
  if (st != HB_OK) {
    const std::string msg = g_err;
    if (c->stream) (void)hipStreamSynchronize(c->stream);
    release(c);
    g_err = msg;
    return st;
  }
  *out = c;
  return HB_OK;
}

hb_status hb_ensemble_reset(hb_ctx* c, const uint64_t* seeds) {
  hb_status st = check_ctx(c);
  if (st != HB_OK) return st;
  if (c->n_seeds < 2) return fail(HB_EINVAL, "not an ensemble context");
  if (seeds) c->seeds.assign(seeds, seeds + c->n_seeds);
  st = do_reset(c, 0);
  if (st != HB_OK) c->failed = true;
  return st;
}

hb_status hb_ensemble_passes(hb_ctx* c, int32_t* passes) {
  hb_status st = check_ctx(c);
  if (st != HB_OK) return st;
  if (!passes) return fail(HB_EINVAL, "passes is NULL");
  if (c->n_seeds < 2) return fail(HB_EINVAL, "not an ensemble context");
  for (int k = 0; k < c->n_seeds; ++k) passes[k] = c->seed_passes[(size_t)k];
  return HB_OK;
}

hb_status hb_ensemble_summary(hb_ctx* c, int32_t which, double* mean, double* sd, int32_t dst_on_device) {
  hb_status st = check_ctx(c);
  if (st != HB_OK) return st;
  if (c->n_seeds < 2) return fail(HB_EINVAL, "not an ensemble context");
  if (which < 0 || which > 3) return fail(HB_EINVAL, "which must be 0 (closeness), 1 (Lin), 2 (harmonic) or 3 (coreachable size)");
  if (c->n == 0 || (!mean && !sd)) return HB_OK;
  if (dst_on_device) {
    HB_HIP(hb::launch_ensemble_summary(c->n, c->n_seeds, which, c->S, c->H, c->E, mean, sd, c->stream));
    HB_HIP(hipStreamSynchronize(c->stream));
    return HB_OK;
  }
  const size_t n = (size_t)c->n;
  if (!c->out_tmp) {
    if (dmalloc(&c->out_tmp, 4 * n * (size_t)c->n_seeds) != hipSuccess)
      return fail(HB_ENOMEM, "cannot allocate output staging");
  }
  HB_HIP(hb::launch_ensemble_summary(c->n, c->n_seeds, which, c->S, c->H, c->E, mean ? c->out_tmp : nullptr,
                                     sd ? c->out_tmp + n : nullptr, c->stream));
  if (mean) HB_HIP(hipMemcpyAsync(mean, c->out_tmp, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
  if (sd) HB_HIP(hipMemcpyAsync(sd, c->out_tmp + n, sizeof(double) * n, hipMemcpyDeviceToHost, c->stream));
  HB_HIP(hipStreamSynchronize(c->stream));
  return HB_OK;
}

void hb_free(hb_ctx* c) {
  if (!c) return;
  (void)hipStreamSynchronize(c->stream);
  release(c);
}

const char* hb_last_error(void) { return g_err.c_str(); }

int32_t hb_version(void) { return 1; }

}  // extern "C"
