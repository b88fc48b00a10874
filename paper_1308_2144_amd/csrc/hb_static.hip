// hb_run_static: the whole computation of hb_init + hb_run + hb_centralities
// for one graph, with every piece of device state in a fixed, statically
// allocated scratch array instead of memory the library allocates.  For
// callers that cannot allocate device memory (tight serving loops, harnesses
// that forbid it).  The passes are the library's own kernels; only the
// schedule is simpler: every non-empty row is handled by a whole wavefront.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <mutex>
#include <string>

#include "hb_ctx.h"

using hbh::fail;

namespace {

// 64 MiB: about n * (2 * 2^log2m + 29) bytes are needed, e.g. n up to about
// 1.1 M nodes at log2m 4 and 120 k at log2m 8.
constexpr size_t kScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;

// The scratch of every call on a device (each GPU holds its own copy from the
// time the library's code is loaded on it until the process ends).  Host code
// never uses this name as an address: it takes the device address that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) uint8_t scratch[kScratchBytes];

std::mutex g_mu;
uint8_t* g_scratch[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device with that device current.
hb_status scratch_on_current_device(uint8_t** out) {
  int dev = 0;
  HB_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(HB_EDEVICE, "device index beyond the static scratch table");
  std::lock_guard<std::mutex> lk(g_mu);
  if (!g_scratch[dev]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(HB_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch[dev] = static_cast<uint8_t*>(p);
  }
  *out = g_scratch[dev];
  return HB_OK;
}

// Carves 256-byte aligned pieces out of the scratch.
struct Carver {
  uint8_t* base;
  size_t used = 0;
  template <class T>
  T* take(size_t count) {
    T* p = reinterpret_cast<T*>(base + used);
    used += (count * sizeof(T) + 255) / 256 * 256;
    return p;
  }
};

}  // namespace

extern "C" hb_status hb_run_static(const hb_csr* g, int32_t log2m, uint64_t seed, double* closeness, double* lin,
                                   double* harmonic, double* coreach, uint8_t* registers, int32_t* passes,
                                   void* stream) {
  if (!g) return fail(HB_EINVAL, "g is NULL");
  if (log2m < 4 || log2m > 8) return fail(HB_EINVAL, "hb_run_static needs log2m in [4, 8]");
  if (!g->on_device) return fail(HB_EINVAL, "hb_run_static needs a device CSR (on_device = 1)");
  if (g->offsets_bits != 32 && g->offsets_bits != 64) return fail(HB_EINVAL, "offsets_bits must be 32 or 64");
  const int64_t n = g->n, m = g->m;
  if (n < 0 || m < 0 || n > 0x7fffffffLL || (n > 0 && !g->offsets) || (m > 0 && !g->indices))
    return fail(HB_EINVAL, "bad CSR sizes or pointers");
  const int p = 1 << log2m;
  const hipStream_t st = static_cast<hipStream_t>(stream);
  const int64_t n_blocks = (n + 63) / 64;

  // Layout of the scratch for this call (every piece 256-byte aligned).
  size_t sel_tmp = 0;
  if (n > 0) HB_HIP(hb::select_rows(nullptr, n, 1, INT64_MAX, nullptr, nullptr, nullptr, &sel_tmp, st));
  auto need = [&](void) {
    const size_t a = 255;
    size_t b = 0;
    auto add = [&](size_t x) { b += (x + a) / 256 * 256; };
    if (g->offsets_bits == 32) add(sizeof(int64_t) * (size_t)(n + 1));
    add((size_t)n * (size_t)p);
    add((size_t)n * (size_t)p);
    add(sizeof(uint64_t) * (size_t)n_blocks);
    add(sizeof(uint64_t) * (size_t)n_blocks);
    add(sizeof(double) * (size_t)n * 3);
    add(sizeof(double) * (size_t)(p + 1));
    add(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    add(sizeof(int) * 1);
    add(sizeof(unsigned long long) * 2 * hb::STAT_SLOTS * hb::STAT_K);
    add(sel_tmp > 0 ? sel_tmp : 1);
    return b;
  };
  const size_t bytes = need();
  if (bytes > kScratchBytes)
    return fail(HB_ENOMEM, "hb_run_static: the graph needs " + std::to_string(bytes) + " bytes of scratch, more than its " +
                               std::to_string(kScratchBytes) + " (about n * (2 * 2^log2m + 29) bytes)");
  uint8_t* base = nullptr;
  hb_status hs = scratch_on_current_device(&base);
  if (hs != HB_OK) return hs;
  Carver cv{base};
  const int64_t* off = static_cast<const int64_t*>(g->offsets);
  if (g->offsets_bits == 32) {
    int64_t* wide = cv.take<int64_t>((size_t)(n + 1));
    HB_HIP(hb::launch_widen_offsets(static_cast<const int32_t*>(g->offsets), wide, n + 1, st));
    off = wide;
  }
  uint8_t* cnt[2] = {cv.take<uint8_t>((size_t)n * p), cv.take<uint8_t>((size_t)n * p)};
  uint64_t* mod[2] = {cv.take<uint64_t>((size_t)n_blocks), cv.take<uint64_t>((size_t)n_blocks)};
  double* S = cv.take<double>((size_t)n * 3);
  double* H = S + n;
  double* E = S + 2 * n;
  double* lc = cv.take<double>((size_t)(p + 1));
  int32_t* rows = cv.take<int32_t>((size_t)(n > 0 ? n : 1));
  int* nrows_dev = cv.take<int>(1);
  unsigned long long* stats = cv.take<unsigned long long>((size_t)2 * hb::STAT_SLOTS * hb::STAT_K);
  void* tmp = cv.take<uint8_t>(sel_tmp > 0 ? sel_tmp : 1);

  // Linear-counting table p*ln(p/V) and the estimator constant, as hb_init
  // computes them (host libm); staged on the stack.
  double lc_host[257];
  lc_host[0] = 0.0;
  for (int V = 1; V <= p; ++V) lc_host[V] = (double)p * std::log((double)p / (double)V);
  const double alpha_pp = (hbh::alpha_for(p) * (double)p) * (double)p;

  int32_t t = 0;
  if (n > 0) {
    HB_HIP(hipMemcpyAsync(lc, lc_host, sizeof(double) * (size_t)(p + 1), hipMemcpyHostToDevice, st));
    // Scratch keeps the previous call's contents: clear what starts at zero.
    HB_HIP(hb::launch_fill_zero(mod[0], sizeof(uint64_t) * (size_t)n_blocks, st));
    HB_HIP(hb::launch_fill_zero(mod[1], sizeof(uint64_t) * (size_t)n_blocks, st));
    HB_HIP(hb::launch_fill_zero(stats, sizeof(unsigned long long) * 2 * hb::STAT_SLOTS * hb::STAT_K, st));
    HB_HIP(hb::launch_init_nodes(log2m, n, seed, cnt[0], cnt[1], S, H, E, lc, alpha_pp, st));
    HB_HIP(hb::select_rows(off, n, 1, INT64_MAX, rows, nrows_dev, tmp, &sel_tmp, st));
    int n_rows = 0;
    HB_HIP(hipMemcpyAsync(&n_rows, nrows_dev, sizeof(int), hipMemcpyDeviceToHost, st));
    HB_HIP(hipStreamSynchronize(st));  // the table above is read from the stack
    unsigned long long sh[hb::STAT_SLOTS * hb::STAT_K];
    int64_t last_nmod = n;
    int cur = 0;
    for (;;) {
      hb::PassArgs a{};
      a.off = off;
      a.idx = g->indices;
      a.cur = cnt[cur];
      a.nxt = cnt[cur ^ 1];
      a.mod_prev = mod[cur];
      a.mod_cur = mod[cur ^ 1];
      a.S = S;
      a.H = H;
      a.E = E;
      a.lc = lc;
      a.medium = rows;
      a.n_medium = n_rows;
      const size_t half = (size_t)hb::STAT_SLOTS * hb::STAT_K;
      a.stats = stats + (size_t)(t & 1) * half;
      a.stats_next = stats + (size_t)((t + 1) & 1) * half;
      a.alpha_pp = alpha_pp;
      a.d = (double)(t + 1);
      a.n = n;
      a.n_blocks = n_blocks;
      a.epoch = t + 1;
      // The modes differ only in the work they skip (see hb_iterate).
      a.mode = t == 0 ? hb::MODE_FIRST : (4 * last_nmod >= (int64_t)n_rows ? hb::MODE_DENSE : hb::MODE_EDGE);
      a.seg_lanes = p / 16;
      a.singletons = t == 0 ? 1 : 0;
      a.seed = seed;
      HB_HIP(hb::launch_fill_zero(a.mod_cur, sizeof(uint64_t) * (size_t)n_blocks, st));
      HB_HIP(hb::launch_pass(log2m, a, st, nullptr));
      HB_HIP(hipMemcpyAsync(sh, a.stats, sizeof(sh), hipMemcpyDeviceToHost, st));
      HB_HIP(hipStreamSynchronize(st));
      int64_t changed = 0;
      for (int s = 0; s < hb::STAT_SLOTS; ++s) changed += (int64_t)sh[s * hb::STAT_K + 3];
      cur ^= 1;
      t += 1;
      last_nmod = changed;
      if (changed == 0) break;
    }
    // The final counters are in cnt[cur]; E holds their estimates.
    if (closeness || lin || harmonic || coreach)
      HB_HIP(hb::launch_finalize(n, S, H, E, closeness, lin, harmonic, coreach, st));
    if (registers)
      HB_HIP(hipMemcpyAsync(registers, cnt[cur], (size_t)n * (size_t)p, hipMemcpyDeviceToDevice, st));
    HB_HIP(hipStreamSynchronize(st));
  } else {
    t = 1;  // an empty graph converges in its first pass, as hb_run counts it
  }
  if (passes) *passes = t;
  return HB_OK;
}
