// Drives the serving loop of libhb (hb_serve.cpp) on the fake device of
// fake_device.cpp and checks what a caller can observe: every request ends
// in the state its history implies (cancelled if a cancel was accepted, done
// otherwise), done requests report the pass count the fake device gives them,
// submissions that can never be admitted are refused, and the counters of
// hb_serve_stats add up.  Prints "ok" and exits 0 on success.
//
//   drive list [tight]   a fixed list of request sizes, default or small limits
//   drive stress SEED    random limits, sizes, log2m and cancellations
#include <algorithm>
#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <random>
#include <string>
#include <thread>
#include <tuple>
#include <vector>

#include "hb.h"

int fake_conv(int64_t n, uint64_t seed);

namespace {

struct Graph {
  std::vector<int64_t> off;
  std::vector<int32_t> idx;
};

// n nodes, m arcs with random endpoints; `hub` > 0 gives node 0 that many
// extra arcs (a heavy row).
Graph make_graph(int64_t n, int64_t m, int64_t hub, uint64_t seed) {
  std::mt19937_64 r(seed);
  Graph g;
  g.off.assign((size_t)n + 1, 0);
  if (n == 0) return g;
  std::vector<int64_t> deg((size_t)n, 0);
  for (int64_t e = 0; e < m; ++e) deg[(size_t)(r() % (uint64_t)n)]++;
  deg[0] += hub;
  for (int64_t v = 0; v < n; ++v) g.off[(size_t)v + 1] = g.off[(size_t)v] + deg[(size_t)v];
  g.idx.resize((size_t)g.off[(size_t)n]);
  for (auto& w : g.idx) w = (int32_t)(r() % (uint64_t)n);
  return g;
}

int failures = 0;
#define EXPECT(cond, ...)                  \
  do {                                     \
    if (!(cond)) {                         \
      fprintf(stderr, "FAIL: " __VA_ARGS__); \
      fprintf(stderr, "\n");               \
      ++failures;                          \
    }                                      \
  } while (0)

struct Sub {
  int64_t id = 0;
  int64_t n = 0;
  uint64_t seed = 0;
  bool cancelled = false;
};

hb_request_info wait_for(hb_server* s, int64_t id, hb_status* st) {
  hb_request_info info{};
  *st = hb_serve_wait(s, id, 20.0, &info);
  return info;
}

int run_list(bool tight) {
  const std::vector<std::tuple<int64_t, int64_t, int>> W = {
      {0, 0, 8},      {5, 0, 4},        {2, 1, 4},        {70, 70, 4},      {9000, 17998, 4}, {512, 6167, 8},
      {4096, 18617, 6}, {2048, 44208, 4}, {256, 4001, 6}, {128, 1713, 6},   {256, 3234, 8},   {64, 178, 8},
      {2048, 40606, 8}, {2048, 21442, 4}, {2048, 12316, 8}, {64, 510, 4},   {64, 488, 6},     {4096, 31846, 4}};
  hb_serve_config cfg;
  hb_serve_default_config(&cfg);
  int64_t biggest = 0;
  for (auto& w : W) biggest = std::max<int64_t>(biggest, 2 * std::get<0>(w) * (1ll << std::get<2>(w)));
  cfg.max_nodes = 1 << 16;
  cfg.max_arcs = 1 << 20;
  if (tight) {
    cfg.budget_bytes = biggest + 4096;
    cfg.max_resident = 3;
    cfg.max_nodes = 1 << 14;
    cfg.max_arcs = 1 << 18;
  }
  hb_server* s = nullptr;
  if (hb_serve_start(&s, &cfg) != HB_OK) {
    fprintf(stderr, "start: %s\n", hb_last_error());
    return 1;
  }
  std::vector<Graph> gs;
  std::vector<Sub> subs;
  for (size_t i = 0; i < W.size(); ++i) {
    gs.push_back(make_graph(std::get<0>(W[i]), std::get<1>(W[i]), 0, i + 1));
    hb_serve_request rq{};
    rq.graph.n = std::get<0>(W[i]);
    rq.graph.m = (int64_t)gs.back().idx.size();
    rq.graph.offsets = gs.back().off.data();
    rq.graph.offsets_bits = 64;
    rq.graph.indices = gs.back().idx.data();
    rq.log2m = std::get<2>(W[i]);
    rq.seed = 100 + i;
    Sub sb;
    sb.n = rq.graph.n;
    sb.seed = rq.seed;
    if (hb_serve_submit(s, &rq, &sb.id) != HB_OK) {
      fprintf(stderr, "submit %zu: %s\n", i, hb_last_error());
      return 1;
    }
    subs.push_back(sb);
  }
  for (const Sub& sb : subs) {
    hb_status st;
    const hb_request_info info = wait_for(s, sb.id, &st);
    EXPECT(st == HB_OK && info.state == HB_REQ_DONE, "request %lld: status %d state %d", (long long)sb.id, st,
           info.state);
    EXPECT(info.passes == fake_conv(sb.n, sb.seed), "request %lld: passes %d, want %d", (long long)sb.id,
           info.passes, fake_conv(sb.n, sb.seed));
    EXPECT(info.t_submit <= info.t_admit && info.t_admit <= info.t_done, "request %lld: times out of order",
           (long long)sb.id);
  }
  hb_serve_stats_t st{};
  hb_serve_stats(s, &st);
  EXPECT(st.completed == (int64_t)W.size() && st.resident == 0 && st.queued == 0 && st.resident_bytes == 0,
         "stats: completed %lld resident %lld queued %lld", (long long)st.completed, (long long)st.resident,
         (long long)st.queued);
  EXPECT(st.peak_resident_bytes <= cfg.budget_bytes, "peak over budget");
  if (failures) return 1;
  EXPECT(hb_serve_stop(s) == HB_OK, "stop: %s", hb_last_error());
  return failures ? 1 : 0;
}

int run_stress(uint64_t seed) {
  std::mt19937_64 r(seed);
  auto uni = [&](int64_t lo, int64_t hi) { return lo + (int64_t)(r() % (uint64_t)(hi - lo + 1)); };
  hb_serve_config cfg;
  hb_serve_default_config(&cfg);
  cfg.max_resident = (int32_t)uni(1, 8);
  cfg.max_nodes = 1ll << uni(10, 14);
  cfg.max_arcs = 1ll << uni(12, 16);
  cfg.budget_bytes = 1ll << uni(16, 22);
  cfg.passes_per_tick = (int32_t)uni(1, 3);
  // small row-class thresholds so that medium rows and chunked heavy rows occur
  cfg.opt.light_max = (int32_t)uni(2, 8);
  cfg.opt.heavy_min = (int32_t)uni(9, 60);
  cfg.opt.chunk = (int32_t)uni(4, 32);
  hb_server* s = nullptr;
  if (hb_serve_start(&s, &cfg) != HB_OK) {
    fprintf(stderr, "start: %s\n", hb_last_error());
    return 1;
  }
  const int count = 1500;
  std::vector<Graph> gs((size_t)count);
  std::vector<Sub> subs;
  int refused = 0;
  for (int i = 0; i < count; ++i) {
    const int64_t n = uni(0, 3) == 0 ? uni(0, 8) : uni(1, 1200);
    const int64_t m = n ? uni(0, 5 * n) : 0;
    const int64_t hub = n && uni(0, 4) == 0 ? uni(0, 300) : 0;
    gs[(size_t)i] = make_graph(n, m, hub, r());
    hb_serve_request rq{};
    rq.graph.n = n;
    rq.graph.m = (int64_t)gs[(size_t)i].idx.size();
    rq.graph.offsets = gs[(size_t)i].off.data();
    rq.graph.offsets_bits = 64;
    rq.graph.indices = gs[(size_t)i].idx.data();
    rq.log2m = (int32_t)uni(4, 8);
    rq.seed = r();
    Sub sb;
    sb.n = n;
    sb.seed = rq.seed;
    const hb_status st = hb_serve_submit(s, &rq, &sb.id);
    const int64_t npad = (n + 1 + 63) / 64 * 64;
    const bool fits = 2 * n * (1ll << rq.log2m) <= cfg.budget_bytes && npad <= cfg.max_nodes - 64 &&
                      rq.graph.m <= cfg.max_arcs;
    if (!fits) {
      EXPECT(st == HB_ENOMEM, "request %d that cannot fit was not refused (status %d)", i, st);
      ++refused;
      continue;
    }
    EXPECT(st == HB_OK, "submit %d: %s", i, hb_last_error());
    if (st != HB_OK) continue;
    // cancel some requests right away; a cancel only succeeds while queued
    if (uni(0, 9) == 0) sb.cancelled = hb_serve_cancel(s, sb.id) == HB_OK;
    subs.push_back(sb);
    if (uni(0, 20) == 0) std::this_thread::sleep_for(std::chrono::microseconds(uni(0, 300)));
  }
  int done = 0, cancelled = 0;
  for (size_t k = 0; k < subs.size(); ++k) {
    const Sub& sb = subs[k];
    hb_status st;
    hb_request_info info{};
    if (k % 3 == 0) {
      // poll until final
      for (int tries = 0; tries < 200000; ++tries) {
        st = hb_serve_poll(s, sb.id, &info);
        if (st != HB_OK || info.state >= HB_REQ_DONE) break;
        std::this_thread::sleep_for(std::chrono::microseconds(50));
      }
    } else {
      info = wait_for(s, sb.id, &st);
    }
    if (sb.cancelled) {
      EXPECT(st == HB_OK && info.state == HB_REQ_CANCELLED, "request %lld: cancel accepted but state %d",
             (long long)sb.id, info.state);
      ++cancelled;
    } else {
      EXPECT(st == HB_OK && info.state == HB_REQ_DONE, "request %lld: status %d state %d", (long long)sb.id, st,
             info.state);
      EXPECT(info.passes == fake_conv(sb.n, sb.seed), "request %lld (n %lld): passes %d, want %d",
             (long long)sb.id, (long long)sb.n, info.passes, fake_conv(sb.n, sb.seed));
      ++done;
    }
    if (failures > 20) break;
  }
  hb_serve_stats_t st{};
  hb_serve_stats(s, &st);
  EXPECT(st.completed == done && st.cancelled == cancelled && st.submitted == (int64_t)subs.size(),
         "stats: completed %lld/%d cancelled %lld/%d submitted %lld/%zu", (long long)st.completed, done,
         (long long)st.cancelled, cancelled, (long long)st.submitted, subs.size());
  EXPECT(st.resident == 0 && st.queued == 0 && st.resident_bytes == 0, "stats: residue after the last request");
  EXPECT(st.peak_resident_bytes <= cfg.budget_bytes, "peak %lld over budget %lld", (long long)st.peak_resident_bytes,
         (long long)cfg.budget_bytes);
  if (failures) return 1;
  EXPECT(hb_serve_stop(s) == HB_OK, "stop: %s", hb_last_error());
  printf("seed %llu: %d done, %d cancelled, %d refused, %lld ticks\n", (unsigned long long)seed, done, cancelled,
         refused, (long long)st.ticks);
  return failures ? 1 : 0;
}

}  // namespace

int main(int argc, char** argv) {
  const std::string what = argc > 1 ? argv[1] : "list";
  int rc = 1;
  if (what == "list")
    rc = run_list(argc > 2 && std::string(argv[2]) == "tight");
  else if (what == "stress")
    rc = run_stress(argc > 2 ? std::strtoull(argv[2], nullptr, 10) : 1);
  if (rc == 0) printf("ok\n");
  fflush(stdout);
  // A failed run may leave the serving thread stuck; do not wait for it.
  std::_Exit(rc);
}
