// A fake device for testing the serving loop of libhb on the CPU.
//
// It provides the HIP runtime calls and the kernel launchers that
// hb_serve.cpp uses, backed by host memory.  Work runs at enqueue time, which
// keeps the semantics of a single in-order stream (the serving loop only
// reads what earlier work on the same stream wrote); events report
// "not ready" for a random number of queries so that the loop's pipelining of
// ticks, snapshots and result copies is exercised.  Engine passes do not run
// HyperBall: graph g converges after fake_conv(n, seed) of its own passes, so
// every request's pass count is known in advance.  Each pass also checks the
// invariants the real kernels rely on: every row-list entry below the
// high-water marks is row 0 (the dead row) or a row of a resident graph, and
// the blocks of every resident graph map to its slot.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <random>
#include <vector>

#include "hb_ctx.h"

static std::mutex g_mu;
static std::mt19937 g_rng(1);

struct FakeEvent {
  int remaining = 0;
};

extern "C" {
hipError_t hipMalloc(void** p, size_t n) {
  *p = calloc(1, n ? n : 1);
  return *p ? hipSuccess : hipErrorOutOfMemory;
}
hipError_t hipFree(void* p) {
  free(p);
  return hipSuccess;
}
hipError_t hipMallocAsync(void** p, size_t n, hipStream_t) { return hipMalloc(p, n); }
hipError_t hipFreeAsync(void* p, hipStream_t) { return hipFree(p); }
hipError_t hipHostMalloc(void** p, size_t n, unsigned int) { return hipMalloc(p, n); }
hipError_t hipHostFree(void* p) { return hipFree(p); }
hipError_t hipMemcpyAsync(void* d, const void* s, size_t n, hipMemcpyKind, hipStream_t) {
  memcpy(d, s, n);
  return hipSuccess;
}
hipError_t hipMemsetAsync(void* d, int v, size_t n, hipStream_t) {
  memset(d, v, n);
  return hipSuccess;
}
hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned int) {
  *s = reinterpret_cast<hipStream_t>(new int(0));
  return hipSuccess;
}
hipError_t hipStreamDestroy(hipStream_t s) {
  delete reinterpret_cast<int*>(s);
  return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipEventCreateWithFlags(hipEvent_t* e, unsigned) {
  *e = reinterpret_cast<hipEvent_t>(new FakeEvent());
  return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t* e) { return hipEventCreateWithFlags(e, 0); }
hipError_t hipEventDestroy(hipEvent_t e) {
  delete reinterpret_cast<FakeEvent*>(e);
  return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t) {
  std::lock_guard<std::mutex> lk(g_mu);
  reinterpret_cast<FakeEvent*>(e)->remaining = (int)(g_rng() % 5);
  return hipSuccess;
}
hipError_t hipEventQuery(hipEvent_t e) {
  FakeEvent* f = reinterpret_cast<FakeEvent*>(e);
  if (f->remaining > 0) {
    --f->remaining;
    return hipErrorNotReady;
  }
  return hipSuccess;
}
hipError_t hipGetDevice(int* d) {
  *d = 0;
  return hipSuccess;
}
hipError_t hipSetDevice(int) { return hipSuccess; }
hipError_t hipGetDeviceProperties(hipDeviceProp_t* p, int) {
  memset(p, 0, sizeof(*p));
  p->multiProcessorCount = 256;
  return hipSuccess;
}
const char* hipGetErrorString(hipError_t) { return "fake error"; }
hipError_t hipGetLastError(void) { return hipSuccess; }
hipError_t hipGraphExecDestroy(hipGraphExec_t) { return hipSuccess; }
void hb_default_options(hb_options* opt) {
  opt->frontier = 1;
  opt->light_max = 64;
  opt->heavy_min = 8192;
  opt->chunk = 4096;
  opt->validate = 1;
  opt->timing = 0;
  opt->dense_pct = 60;
  opt->push = 1;
  opt->sparse_pct = 20;
  opt->qdense = 0;
  opt->slice = 0;
  opt->wgs_per_cu = 5;
  opt->graph_passes = 4;
}
}

// Fake convergence: a graph converges after conv(n, seed) passes.
int fake_conv(int64_t n, uint64_t seed) { return 1 + (int)((n * 7 + seed) % 9); }

namespace hb {
hipError_t launch_fill_zero(void* p, size_t bytes, hipStream_t) {
  memset(p, 0, bytes);
  return hipSuccess;
}
hipError_t launch_set_slot(GraphDev* graphs, int32_t slot, const GraphDev& val, hipStream_t) {
  graphs[slot] = val;
  return hipSuccess;
}
hipError_t launch_set_plan(PassCtl* ctl, int64_t l, int64_t a, hipStream_t) {
  ctl->listed_rows = l;
  ctl->arcs = a;
  return hipSuccess;
}
hipError_t launch_admit(PassCtl* ctl, GraphDev* graphs, int32_t slot, const GraphDev& val, int64_t m, int32_t* blk,
                        uint64_t* m0, uint64_t* m1, int64_t b0, int64_t b1, hipStream_t) {
  uint64_t* prev = ctl->parity ? m1 : m0;
  uint64_t* next = ctl->parity ? m0 : m1;
  for (int64_t b = b0; b < b1; ++b) {
    const int64_t real = val.node_base + val.n - b * 64;
    blk[b] = slot;
    prev[b] = real >= 64 ? ~0ull : (real > 0 ? (1ull << real) - 1ull : 0ull);
    next[b] = 0;
  }
  GraphDev v = val;
  v.t0 = ctl->t;
  v.done = 0;
  v.passes = 0;
  v.active = 1;
  graphs[slot] = v;
  ctl->chg += (unsigned long long)val.n;
  ctl->pairs += (unsigned long long)m;
  return hipSuccess;
}
hipError_t launch_rebase_csr(const void* off_l, int bits, int64_t n, int64_t m, int64_t nb, int64_t ab, int64_t* off,
                             int32_t* idx, hipStream_t) {
  for (int64_t v = 0; v <= n; ++v)
    off[nb + v] = ab + (bits == 64 ? ((const int64_t*)off_l)[v] : ((const int32_t*)off_l)[v]);
  for (int64_t e = 0; e < m; ++e) idx[ab + e] += (int32_t)nb;
  return hipSuccess;
}
hipError_t launch_init_arena(int, int64_t v0, int64_t v1, const int32_t*, const GraphDev*, uint8_t*, uint8_t*,
                             double* S, double* H, double* E, const double*, double, hipStream_t) {
  for (int64_t v = v0; v < v1; ++v) S[v] = H[v] = E[v] = 0.0;
  return hipSuccess;
}
hipError_t launch_finalize(int64_t, const double*, const double*, const double*, double*, double*, double*, double*,
                           hipStream_t) {
  return hipSuccess;
}
hipError_t launch_device_pass(int, const PassArgs& a, int, uint2*, unsigned long long*, int64_t, hipStream_t) {
  PassCtl* c = a.ctl;
  const int t = c->t;
  for (int g = 0; g < a.n_graphs; ++g) {
    GraphDev& gd = a.graphs[g];
    if (!gd.active || gd.done || t < gd.t0) continue;
    const int k = t - gd.t0 + 1;
    if (k >= fake_conv(gd.n, gd.seed)) {
      gd.done = 1;
      gd.passes = k;
    }
  }
  auto check_row = [&](const char* what, int64_t i, int64_t r) {
    if (r == 0) return;
    const GraphDev& gd = a.graphs[a.blk_graph[r >> 6]];
    if (!gd.active || r < gd.node_base || r >= gd.node_base + gd.n) {
      fprintf(stderr, "invariant: %s entry %lld names row %lld outside a resident graph\n", what, (long long)i,
              (long long)r);
      abort();
    }
  };
  for (int64_t i = 0; i < a.n_light; ++i) check_row("light", i, a.light[i]);
  for (int64_t i = 0; i < a.n_medium; ++i) check_row("medium", i, a.medium[i]);
  for (int64_t i = 0; i < a.n_items; ++i) check_row("item", i, a.items[i].row);
  for (int64_t i = 0; i < a.n_hrows; ++i) {
    check_row("heavy row", i, a.hrows[i].row);
    if (a.hrows[i].row != 0 && a.hrows[i].item0 + a.hrows[i].nitems > a.n_items) {
      fprintf(stderr, "invariant: heavy row %lld names items past the high-water mark\n", (long long)i);
      abort();
    }
  }
  // Change bits of the pass only ever name rows of resident graphs.
  const uint64_t* prev = a.modb[c->parity];
  for (int64_t w = 0; w < a.n / 64; ++w)
    for (uint64_t bits = prev[w]; bits; bits &= bits - 1ull) {
      const int64_t r = w * 64 + __builtin_ctzll(bits);
      const GraphDev& gd = a.graphs[a.blk_graph[r >> 6]];
      if (!gd.active || r < gd.node_base || r >= gd.node_base + gd.n) {
        fprintf(stderr, "invariant: change bit of row %lld outside a resident graph\n", (long long)r);
        abort();
      }
    }
  for (int g = 1; g < a.n_graphs; ++g) {
    const GraphDev& gd = a.graphs[g];
    if (!gd.active) continue;
    if (gd.node_base % 64 || gd.node_base < 64 || gd.node_base + gd.n >= a.n) {
      fprintf(stderr, "invariant: slot %d region [%lld, +%lld) outside the pool high-water %lld\n", g,
              (long long)gd.node_base, (long long)gd.n, (long long)a.n);
      abort();
    }
    for (int64_t b = gd.node_base / 64; b <= (gd.node_base + gd.n) / 64; ++b)
      if (a.blk_graph[b] != g) {
        fprintf(stderr, "invariant: block %lld of slot %d maps to slot %d\n", (long long)b, g, a.blk_graph[b]);
        abort();
      }
  }
  // the bitmap this pass read is the one the next pass writes: cleared
  for (int64_t w = 0; w < a.n / 64; ++w) a.modb[c->parity][w] = 0ull;
  c->t += 1;
  c->parity ^= 1;
  return hipSuccess;
}
}  // namespace hb

namespace hbh {
void release(hb_ctx* c) {
  if (!c) return;
  free(c->off);
  free(c->idx_owned);
  for (int i = 0; i < 2; ++i) {
    free(c->cnt[i]);
    free(c->mod[i]);
  }
  free(c->S);
  free(c->H);
  free(c->E);
  free(c->lc);
  free(c->light);
  free(c->medium);
  free(c->items);
  free(c->hrows);
  free(c->partial);
  free(c->stats);
  free(c->graphs);
  free(c->blk_graph);
  free(c->ctl);
  delete c;
}
hb::PassArgs device_args(hb_ctx* c) {
  hb::PassArgs a{};
  a.light = c->light;
  a.medium = c->medium;
  a.items = c->items;
  a.hrows = c->hrows;
  a.n_light = c->n_light;
  a.n_medium = c->n_medium;
  a.n_items = c->n_items;
  a.n_hrows = c->n_hrows;
  a.n = c->n;
  a.graphs = c->graphs;
  a.blk_graph = c->blk_graph;
  a.ctl = c->ctl;
  a.n_graphs = c->n_graphs;
  a.modb[0] = c->mod[0];
  a.modb[1] = c->mod[1];
  return a;
}
thread_local std::string g_err;
}  // namespace hbh
extern "C" const char* hb_last_error(void) { return hbh::g_err.c_str(); }
